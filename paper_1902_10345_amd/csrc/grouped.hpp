// grouped.hpp -- device descriptor of one problem of a grouped launch.
#pragma once

#include <vector>

#include "common.hpp"

namespace mm {

struct Desc {
  const float *A;
  const float *B;
  float *C;
  int64_t lda, ldb, ldc;
  int M, N, K;
  float alpha, beta;
  int variant;  // tile variant (0: 128 x 128, 1: 64 x 64)
  int tiles_n;  // output tiles along N for this variant (0: no MFMA work)
  int vec;      // 128-bit loads of A rows allowed
};

constexpr double kDefaultSmallCost = 1.6;

int grouped_num_variants();
int grouped_variant_bm(int v);
int grouped_pick_variant(int64_t M, int64_t N, double small_cost);
size_t grouped_ws_bytes(int count);
gemm_status grouped_build(const gemm_problem *probs, int count, const int *variant,
                          std::vector<Desc> &descs, std::vector<int> &starts, int &total);
gemm_status grouped_upload(void *ws, const std::vector<Desc> &descs, const std::vector<int> &starts,
                           hipStream_t s);
gemm_status grouped_upload_pinned(void *ws, void *pinned, const std::vector<Desc> &descs,
                                  const std::vector<int> &starts, hipStream_t s);
gemm_status grouped_enqueue(void *ws, int count, int total, int grid, hipStream_t s);
int grouped_grid(int total);

}  // namespace mm
