// noalloc.hip -- the split-K entry point for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops): the
// partial planes live in a fixed array of this library instead of a
// caller-provided workspace.
//
// The array is resolved to its device address once per device, on the
// entry point's first call with that device current, and that address (never
// the array's host-side name) is what the kernels receive.  Each device that
// runs the entry point holds its own copy of the array until the process
// ends.  Every call on one device shares that device's copy: calls that
// overlap on one device race (serialise them on one stream).  Nothing in it
// has to start at zero: every chunk's plane is written in full before the
// reduction reads it.
#include <mutex>
#include <string>

#include "common.hpp"
#include "kernels.hpp"

namespace mm {
namespace {

static __device__ __align__(256) float scratch[GEMM_NOALLOC_SCRATCH_BYTES / sizeof(float)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch`, per device

gemm_status scratch_address(const char *fn, void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(fn, e);
  if (dev < 0 || dev >= kMaxDevices) {
    set_error(std::string(fn) + ": device index beyond the library's per-device table");
    return GEMM_STATUS_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(fn, e);
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return GEMM_STATUS_OK;
}

}  // namespace
}  // namespace mm

using namespace mm;

extern "C" {

gemm_status gemm_f32_3xbf16_splitk_noalloc(int64_t M, int64_t N, int64_t K, float alpha,
                                           const float *A, int64_t lda, const float *B,
                                           int64_t ldb, float beta, float *C, int64_t ldc,
                                           int n_products, int splits, hipStream_t stream) {
  clear_error();
  const char *fn = "gemm_f32_3xbf16_splitk_noalloc";
  bool noop = false, scale_only = false;
  gemm_status st = check_f32_args(fn, M, N, K, alpha, A, lda, B, ldb, C, ldc, noop, scale_only);
  if (st) return st;
  if (n_products != 3 && n_products != 6) return bad_arg(12, fn, "(n_products) must be 3 or 6");
  if (splits < 0 || splits > 64) return bad_arg(13, fn, "(splits) must be in [0, 64]");
  if (noop) return GEMM_STATUS_OK;
  if (scale_only) return scale_c(M, N, beta, C, ldc, stream);
  if (splits == 0) splits = bx3_splitk_default(M, N, K);
  const size_t need = bx3_splitk_ws_bytes(M, N, splits);
  if (need > GEMM_NOALLOC_SCRATCH_BYTES) {
    set_error(std::string(fn) + ": " + std::to_string(splits) + " partial planes of " +
              std::to_string(M) + " x " + std::to_string(N) +
              " floats exceed the fixed scratch of GEMM_NOALLOC_SCRATCH_BYTES bytes");
    return GEMM_STATUS_NO_MEMORY;
  }
  void *P = nullptr;
  if (need > 0 && (st = scratch_address(fn, &P))) return st;
  GemmArgs g{M, N, K, alpha, beta, A, lda, B, ldb, C, ldc};
  return bx3_run_splitk(g, n_products, splits, P, stream);
}

}  // extern "C"
