// kernels.hpp -- internal interface between the C-ABI layer and the kernels.
#pragma once

#include "common.hpp"

namespace mm {

// One GEMM problem after argument checking: C <- alpha*op(A)*op(B) + beta*C,
// row-major.  ta: A is stored K x M (row stride lda), op(A) = A^T; tb: B is
// stored N x K (row stride ldb), op(B) = B^T.
struct GemmArgs {
  int64_t M, N, K;
  float alpha, beta;
  const float *A;
  int64_t lda;
  const float *B;
  int64_t ldb;
  float *C;
  int64_t ldc;
  bool ta = false, tb = false;
};

struct TileConfig {
  int bm, bn, bk;
  const char *name;
};

// Plain FP32 vector-ALU path.
int f32_num_configs();
const TileConfig &f32_config(int i);
int f32_default_config(int64_t M, int64_t N, int64_t K);
gemm_status f32_run(const GemmArgs &g, int cfg, hipStream_t s);

// FP32-accurate split-precision path on bf16 MFMA.
int bx3_num_configs();
const TileConfig &bx3_config(int i);
int bx3_config_products(int i);
int bx3_default_config(int64_t M, int64_t N, int64_t K, int n_products);
gemm_status bx3_run(const GemmArgs &g, int cfg, hipStream_t s);
// Transposed-operand variants (B^T, A^T, both), for configurations 0, 2, 3,
// 4, 5, 6 and 8; bx3_run and f32mfma_run dispatch to them from g.ta / g.tb.
gemm_status bx3_run_nt(const GemmArgs &g, int cfg, hipStream_t s);
gemm_status bx3_run_tn(const GemmArgs &g, int cfg, hipStream_t s);
gemm_status bx3_run_tt(const GemmArgs &g, int cfg, hipStream_t s);
gemm_status f32mfma_run_nt(const GemmArgs &g, int which, hipStream_t s);
gemm_status f32mfma_run_tn(const GemmArgs &g, int which, hipStream_t s);
gemm_status f32mfma_run_tt(const GemmArgs &g, int which, hipStream_t s);
int bx3_splitk_default(int64_t M, int64_t N, int64_t K);
// FP32 matrix-core tiles of the plain path: 0 = 256 x 256 (8 waves), 1 = 128 x 128 (4 waves)
gemm_status f32mfma_run(const GemmArgs &g, int which, hipStream_t s);
size_t bx3_splitk_ws_bytes(int64_t M, int64_t N, int splits);
gemm_status bx3_run_splitk(const GemmArgs &g, int n_products, int splits, void *ws, hipStream_t s);
// Small products (k_small.hip): which 0 = 32 x 32 tiles, 1 = 64 x 64; np 1 =
// binary32 matrix cores, 2 / 3 = bf16 planes per operand (3 / 6 products).
gemm_status small_run(const GemmArgs &g, int which, int np, hipStream_t s);
// Batched-strided products (binary32 or split precision) on the MFMA tiles.
// Codes beyond the tile configurations: one wave per small problem (M, N <=
// 64) in binary32, or split precision with three or six products.
constexpr int kBatchedSmall3 = 100, kBatchedSmall6 = 101, kBatchedSmall1 = 102;
int batched_config(int path, int n_products, int64_t M, int64_t N, int64_t K, int64_t batch);
gemm_status batched_run(int path, int cfg, const GemmArgs &g, int64_t sa, int64_t sb, int64_t sc,
                        int batch, hipStream_t s);
gemm_status bx3_split(int64_t n, const float *x, uint16_t *p0, uint16_t *p1, uint16_t *p2,
                      hipStream_t s);

// Binary64 path (single problem: batch 1, strides unused).
struct GemmArgsF64 {
  int64_t M, N, K;
  double alpha, beta;
  const double *A;
  int64_t lda, sa;
  const double *B;
  int64_t ldb, sb;
  double *C;
  int64_t ldc, sc;
  int64_t batch;
};
int f64_num_configs();
const TileConfig &f64_config(int i);
int f64_default_config(int64_t M, int64_t N, int64_t K, int64_t batch);
gemm_status f64_run(const GemmArgsF64 &g, int cfg, hipStream_t s);
gemm_status scale_c_f64(int64_t M, int64_t N, double beta, double *C, int64_t ldc, int64_t sc,
                        int64_t batch, hipStream_t s);

// Scaled FP8 path.
size_t fp8_ws_bytes(int64_t M, int64_t N, int64_t K);
int64_t fp8_kp(int64_t K);
// ta / tb: A stored K x M (op(A) = A^T), B stored N x K (op(B) = B^T).
gemm_status fp8_quantize_run(int64_t M, int64_t N, int64_t K, const float *A, int64_t lda,
                             const float *B, int64_t ldb, void *ws, hipStream_t s,
                             bool ta = false, bool tb = false);
int fp8_num_configs();
int fp8_default_config(int64_t M, int64_t N, int64_t K);
const char *fp8_config_name(int cfg);
gemm_status fp8_gemm_run_cfg(int64_t M, int64_t N, int64_t K, float alpha, const void *ws,
                             float beta, float *C, int64_t ldc, int cfg, hipStream_t s);
gemm_status fp8_encode_run(int64_t n, const float *x, uint8_t *out, hipStream_t s);

// Argument rules of the (M,N,K,alpha,A,lda,B,ldb,beta,C,ldc) prefix shared by
// the binary32 entry points (BLAS order, -index on a bad argument); noop:
// M == 0 or N == 0; scale_only: alpha == 0 or K == 0 (C <- beta*C).
gemm_status check_f32_args(const char *fn, int64_t M, int64_t N, int64_t K, float alpha,
                           const float *A, int64_t lda, const float *B, int64_t ldb,
                           const float *C, int64_t ldc, bool &noop, bool &scale_only);
// The configuration an entry point of `path` runs (tuned, else the default).
int library_config(int path, int n_products, int64_t M, int64_t N, int64_t K);

// Autotuner table: the tuned configuration for this size bucket, or -1.
int tuned_config(int path, int n_products, int64_t M, int64_t N, int64_t K);
double tuned_small_cost();

// C <- beta*C over a batch of MxN blocks at stride sc.
gemm_status scale_c_batched(int64_t M, int64_t N, float beta, float *C, int64_t ldc, int64_t sc,
                            int64_t batch, hipStream_t s);
// C <- beta*C over an MxN block (alpha == 0 or K == 0 quick path).
gemm_status scale_c(int64_t M, int64_t N, float beta, float *C, int64_t ldc, hipStream_t s);

// FP64 error norm.
size_t errnorm_ws_bytes();
gemm_status errnorm_run(int64_t M, int64_t N, const float *C, int64_t ldc, const double *Cref,
                        const double *den, double *out, void *ws, hipStream_t s);

}  // namespace mm
