// common.hpp -- shared host/device helpers of the GEMM library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>

#include "gemm_mi355x.h"

namespace mm {

// ---------------------------------------------------------------- errors --
void set_error(const std::string &msg);
void clear_error();

// Records `what` with the HIP error text and returns GEMM_STATUS_HIP_ERROR.
gemm_status hip_fail(const char *what, hipError_t e);

// Checks for a launch error right after a kernel launch.
gemm_status check_launch(const char *kernel);

// Rejects argument `index` (1-based) with a message; returns -index.
gemm_status bad_arg(int index, const char *fn, const char *why);

// Number of compute units of the current device (cached per device).
int num_cus();

// ------------------------------------------------------- device helpers --
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ bool aligned16(const void *p) {
  return (reinterpret_cast<uintptr_t>(p) & 15u) == 0;
}

// XCD-aware remap of a 1-D workgroup id.  The dispatcher places consecutive
// workgroup ids on consecutive XCDs (round robin over 8); remapping makes
// every XCD own one contiguous block of logical tiles, so neighbouring tiles
// -- which share A row panels and B column panels -- meet in the same L2.
__device__ __forceinline__ int xcd_remap(int wg, int nwg) {
  constexpr int kXcds = 8;
  const int per = nwg / kXcds;          // full rounds
  const int full = per * kXcds;
  if (wg >= full) return wg;            // ragged tail keeps its id
  return (wg % kXcds) * per + wg / kXcds;
}

// Grouped ordering of output tiles: walks GROUP tile-rows at a time down a
// column of tiles so that consecutive logical ids reuse the same B panel and
// a small set of A panels.
__device__ __forceinline__ void tile_coords(int logical, int tiles_m, int tiles_n,
                                            int group, int &tm, int &tn) {
  const int per_group = group * tiles_n;
  const int g = logical / per_group;
  const int first_m = g * group;
  const int rows = min(tiles_m - first_m, group);
  const int in = logical - g * per_group;
  tm = first_m + in % rows;
  tn = in / rows;
}

}  // namespace mm
