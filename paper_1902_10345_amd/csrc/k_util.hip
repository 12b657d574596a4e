// k_util.hip -- small kernels: the beta-only quick path and the FP64 error norm.
#include "common.hpp"
#include "kernels.hpp"

namespace mm {

// C <- beta*C (beta == 0 writes zeros without reading C).
template <bool BETA>
__global__ __launch_bounds__(256) void scale_c_kernel(int64_t M, int64_t N, float beta,
                                                      float *__restrict__ C, int64_t ldc) {
  const int64_t total = M * N;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / N, j = e - i * N;
    float *p = C + i * ldc + j;
    *p = BETA ? beta * *p : 0.0f;
  }
}

gemm_status scale_c(int64_t M, int64_t N, float beta, float *C, int64_t ldc, hipStream_t s) {
  const int64_t total = M * N;
  const int64_t want = (total + 255) / 256;
  const unsigned grid = (unsigned)(want < 4096 ? (want > 0 ? want : 1) : 4096);
  if (beta != 0.0f)
    hipLaunchKernelGGL(scale_c_kernel<true>, dim3(grid), dim3(256), 0, s, M, N, beta, C, ldc);
  else
    hipLaunchKernelGGL(scale_c_kernel<false>, dim3(grid), dim3(256), 0, s, M, N, beta, C, ldc);
  return check_launch("scale_c_kernel");
}

// C <- beta*C for a batch of M x N blocks at stride sc (grid.y = problem).
template <bool BETA>
__global__ __launch_bounds__(256) void scale_c_batched_kernel(int64_t M, int64_t N, float beta,
                                                              float *__restrict__ C, int64_t ldc,
                                                              int64_t sc) {
  float *Cb = C + (int64_t)blockIdx.y * sc;
  const int64_t total = M * N;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / N, j = e - i * N;
    float *p = Cb + i * ldc + j;
    *p = BETA ? beta * *p : 0.0f;
  }
}

gemm_status scale_c_batched(int64_t M, int64_t N, float beta, float *C, int64_t ldc, int64_t sc,
                            int64_t batch, hipStream_t s) {
  const int64_t want = (M * N + 255) / 256;
  const unsigned gx = (unsigned)(want < 4096 ? (want > 0 ? want : 1) : 4096);
  for (int64_t b0 = 0; b0 < batch; b0 += 65535) {
    const dim3 grid(gx, (unsigned)(batch - b0 < 65535 ? batch - b0 : 65535));
    if (beta != 0.0f)
      hipLaunchKernelGGL(scale_c_batched_kernel<true>, grid, dim3(256), 0, s, M, N, beta,
                         C + b0 * sc, ldc, sc);
    else
      hipLaunchKernelGGL(scale_c_batched_kernel<false>, grid, dim3(256), 0, s, M, N, beta,
                         C + b0 * sc, ldc, sc);
    if (gemm_status st = check_launch("scale_c_batched_kernel")) return st;
  }
  return GEMM_STATUS_OK;
}

// ------------------------------------------------------- FP64 error norm --
// Stage 1: kNormBlocks blocks, each walks a fixed grid-stride subset of the
// MxN elements and reduces (sum d^2, sum ref^2, max ratio) in binary64 with a
// fixed-shape LDS tree.  Stage 2: one block reduces the per-block partials in
// a fixed order.  The result is independent of scheduling.
constexpr int kNormBlocks = 512;
constexpr int kNormThreads = 256;

__device__ __forceinline__ double nan_max(double a, double b) {
  return (b > a || b != b) ? b : a;  // NaN is sticky
}

__global__ __launch_bounds__(kNormThreads) void errnorm_stage1(
    int64_t M, int64_t N, const float *__restrict__ C, int64_t ldc,
    const double *__restrict__ R, const double *__restrict__ D, double *__restrict__ part) {
  __shared__ double s_num[kNormThreads], s_ref[kNormThreads], s_mx[kNormThreads];
  double num = 0.0, ref = 0.0, mx = 0.0;
  const int64_t total = M * N;
  for (int64_t e = (int64_t)blockIdx.x * kNormThreads + threadIdx.x; e < total;
       e += (int64_t)kNormBlocks * kNormThreads) {
    const int64_t i = e / N, j = e - i * N;
    const double r = R[e];
    const double d = (double)C[i * ldc + j] - r;
    num += d * d;
    ref += r * r;
    double q = fabs(d);
    if (D) {
      const double dd = D[e];
      q = (dd == 0.0) ? (d == 0.0 ? 0.0 : __builtin_huge_val()) : q / dd;
    }
    mx = nan_max(mx, q);
  }
  s_num[threadIdx.x] = num;
  s_ref[threadIdx.x] = ref;
  s_mx[threadIdx.x] = mx;
  __syncthreads();
  for (int w = kNormThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s_num[threadIdx.x] += s_num[threadIdx.x + w];
      s_ref[threadIdx.x] += s_ref[threadIdx.x + w];
      s_mx[threadIdx.x] = nan_max(s_mx[threadIdx.x], s_mx[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x + 0] = s_num[0];
    part[3 * blockIdx.x + 1] = s_ref[0];
    part[3 * blockIdx.x + 2] = s_mx[0];
  }
}

__global__ __launch_bounds__(kNormThreads) void errnorm_stage2(const double *__restrict__ part,
                                                               double *__restrict__ out) {
  __shared__ double s_num[kNormThreads], s_ref[kNormThreads], s_mx[kNormThreads];
  double num = 0.0, ref = 0.0, mx = 0.0;
  for (int b = threadIdx.x; b < kNormBlocks; b += kNormThreads) {
    num += part[3 * b + 0];
    ref += part[3 * b + 1];
    mx = nan_max(mx, part[3 * b + 2]);
  }
  s_num[threadIdx.x] = num;
  s_ref[threadIdx.x] = ref;
  s_mx[threadIdx.x] = mx;
  __syncthreads();
  for (int w = kNormThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s_num[threadIdx.x] += s_num[threadIdx.x + w];
      s_ref[threadIdx.x] += s_ref[threadIdx.x + w];
      s_mx[threadIdx.x] = nan_max(s_mx[threadIdx.x], s_mx[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double n = s_num[0], r = s_ref[0];
    out[0] = r > 0.0 ? sqrt(n / r) : sqrt(n);
    out[1] = n;
    out[2] = r;
    out[3] = s_mx[0];
  }
}

size_t errnorm_ws_bytes() { return sizeof(double) * 3 * kNormBlocks; }

gemm_status errnorm_run(int64_t M, int64_t N, const float *C, int64_t ldc, const double *Cref,
                        const double *den, double *out, void *ws, hipStream_t s) {
  double *part = static_cast<double *>(ws);
  hipLaunchKernelGGL(errnorm_stage1, dim3(kNormBlocks), dim3(kNormThreads), 0, s, M, N, C, ldc,
                     Cref, den, part);
  gemm_status st = check_launch("errnorm_stage1");
  if (st) return st;
  hipLaunchKernelGGL(errnorm_stage2, dim3(1), dim3(kNormThreads), 0, s, part, out);
  return check_launch("errnorm_stage2");
}

}  // namespace mm
