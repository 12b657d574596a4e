// api.hip -- the C-ABI boundary: argument validation, quick returns, dispatch.
//
// The validation pass mirrors the role of the SDFG validation step of the
// compilation pipeline (Sec. 4.3): nothing is enqueued until every argument
// has been checked.  Argument rules follow the BLAS-style call of the paper's
// external-code example (Sec. 2.1), read as row-major with no transposes.
#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

namespace mm {

static thread_local std::string t_err;

void set_error(const std::string &msg) { t_err = msg; }
void clear_error() { t_err.clear(); }

gemm_status hip_fail(const char *what, hipError_t e) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return GEMM_STATUS_HIP_ERROR;
}

gemm_status check_launch(const char *kernel) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(kernel, e);
  return GEMM_STATUS_OK;
}

gemm_status bad_arg(int index, const char *fn, const char *why) {
  set_error(std::string(fn) + ": argument " + std::to_string(index) + " " + why);
  return -index;
}

int num_cus() {
  static std::mutex mu;
  static std::vector<int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  std::lock_guard<std::mutex> lock(mu);
  if ((int)cache.size() <= dev) cache.resize(dev + 1, 0);
  if (cache[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
      n = 256;
    cache[dev] = n;
  }
  return cache[dev];
}

// Shared checks of the (M,N,K,alpha,A,lda,B,ldb,beta,C,ldc) prefix.
// Returns 0 and sets `quick` when the call is fully handled by a quick path
// decision (no-op or C <- beta*C); returns -index on a bad argument.
struct Checked {
  bool noop = false;      // M == 0 or N == 0
  bool scale_only = false;  // alpha == 0 or K == 0
};

template <typename T>
static gemm_status check_gemm_args(const char *fn, int64_t M, int64_t N, int64_t K, T alpha,
                                   const T *A, int64_t lda, const T *B, int64_t ldb,
                                   const T *C, int64_t ldc, Checked &ck) {
  if (M < 0) return bad_arg(1, fn, "(M) must be >= 0");
  if (N < 0) return bad_arg(2, fn, "(N) must be >= 0");
  if (K < 0) return bad_arg(3, fn, "(K) must be >= 0");
  if (M > 0x7fffffffLL || N > 0x7fffffffLL || K > 0x7fffffffLL)
    return bad_arg(M > 0x7fffffffLL ? 1 : N > 0x7fffffffLL ? 2 : 3, fn, "exceeds 2^31-1");
  if (lda < (K > 1 ? K : 1)) return bad_arg(6, fn, "(lda) must be >= max(1,K)");
  if (ldb < (N > 1 ? N : 1)) return bad_arg(8, fn, "(ldb) must be >= max(1,N)");
  if (ldc < (N > 1 ? N : 1)) return bad_arg(11, fn, "(ldc) must be >= max(1,N)");
  if (M == 0 || N == 0) { ck.noop = true; return GEMM_STATUS_OK; }
  if (!C) return bad_arg(10, fn, "(C) is NULL");
  if (alpha == (T)0 || K == 0) { ck.scale_only = true; return GEMM_STATUS_OK; }
  if (!A) return bad_arg(5, fn, "(A) is NULL");
  if (!B) return bad_arg(7, fn, "(B) is NULL");
  return GEMM_STATUS_OK;
}

static int pick_config(int path, int n_products, int64_t M, int64_t N, int64_t K) {
  if (path == GEMM_PATH_FP8_PREQUANTIZED) path = GEMM_PATH_FP8;
  const int t = tuned_config(path, n_products, M, N, K);
  if (t >= 0) return t;
  switch (path) {
    case GEMM_PATH_F32: return f32_default_config(M, N, K);
    case GEMM_PATH_3XBF16: return bx3_default_config(M, N, K, n_products);
    default: return fp8_default_config(M, N, K);
  }
}

gemm_status check_f32_args(const char *fn, int64_t M, int64_t N, int64_t K, float alpha,
                           const float *A, int64_t lda, const float *B, int64_t ldb,
                           const float *C, int64_t ldc, bool &noop, bool &scale_only) {
  Checked ck;
  const gemm_status st = check_gemm_args(fn, M, N, K, alpha, A, lda, B, ldb, C, ldc, ck);
  noop = ck.noop;
  scale_only = ck.scale_only;
  return st;
}

int library_config(int path, int n_products, int64_t M, int64_t N, int64_t K) {
  return pick_config(path, n_products, M, N, K);
}

}  // namespace mm

using namespace mm;

extern "C" {

const char *gemm_last_error(void) { return t_err.c_str(); }

const char *gemm_version(void) { return "gemm_mi355x 0.1 (gfx950)"; }

gemm_status gemm_f32(int64_t M, int64_t N, int64_t K, float alpha, const float *A, int64_t lda,
                     const float *B, int64_t ldb, float beta, float *C, int64_t ldc,
                     hipStream_t stream) {
  clear_error();
  Checked ck;
  gemm_status st = check_gemm_args("gemm_f32", M, N, K, alpha, A, lda, B, ldb, C, ldc, ck);
  if (st || ck.noop) return st;
  if (ck.scale_only) return scale_c(M, N, beta, C, ldc, stream);
  GemmArgs g{M, N, K, alpha, beta, A, lda, B, ldb, C, ldc};
  return f32_run(g, pick_config(GEMM_PATH_F32, 0, M, N, K), stream);
}

gemm_status gemm_f32_3xbf16(int64_t M, int64_t N, int64_t K, float alpha, const float *A,
                            int64_t lda, const float *B, int64_t ldb, float beta, float *C,
                            int64_t ldc, int n_products, hipStream_t stream) {
  clear_error();
  const char *fn = "gemm_f32_3xbf16";
  Checked ck;
  gemm_status st = check_gemm_args(fn, M, N, K, alpha, A, lda, B, ldb, C, ldc, ck);
  if (st) return st;
  if (n_products != 3 && n_products != 6) return bad_arg(12, fn, "(n_products) must be 3 or 6");
  if (ck.noop) return GEMM_STATUS_OK;
  if (ck.scale_only) return scale_c(M, N, beta, C, ldc, stream);
  GemmArgs g{M, N, K, alpha, beta, A, lda, B, ldb, C, ldc};
  return bx3_run(g, pick_config(GEMM_PATH_3XBF16, n_products, M, N, K), stream);
}

int gemm_splitk_default_splits(int64_t M, int64_t N, int64_t K) {
  if (M <= 0 || N <= 0 || K <= 0) return 1;
  return bx3_splitk_default(M, N, K);
}

size_t gemm_splitk_workspace_bytes(int64_t M, int64_t N, int64_t K, int splits) {
  if (M < 0 || N < 0 || K < 0 || splits < 0 || splits > 64) return 0;
  if (splits == 0) splits = gemm_splitk_default_splits(M, N, K);
  return bx3_splitk_ws_bytes(M, N, splits);
}

gemm_status gemm_f32_3xbf16_splitk(int64_t M, int64_t N, int64_t K, float alpha, const float *A,
                                   int64_t lda, const float *B, int64_t ldb, float beta, float *C,
                                   int64_t ldc, int n_products, int splits, void *workspace,
                                   size_t ws_bytes, hipStream_t stream) {
  clear_error();
  const char *fn = "gemm_f32_3xbf16_splitk";
  Checked ck;
  gemm_status st = check_gemm_args(fn, M, N, K, alpha, A, lda, B, ldb, C, ldc, ck);
  if (st) return st;
  if (n_products != 3 && n_products != 6) return bad_arg(12, fn, "(n_products) must be 3 or 6");
  if (splits < 0 || splits > 64) return bad_arg(13, fn, "(splits) must be in [0, 64]");
  if (ck.noop) return GEMM_STATUS_OK;
  if (ck.scale_only) return scale_c(M, N, beta, C, ldc, stream);
  if (splits == 0) splits = bx3_splitk_default(M, N, K);
  const size_t need = bx3_splitk_ws_bytes(M, N, splits);
  if (need > 0) {
    if (!workspace || ((uintptr_t)workspace & 255)) return bad_arg(14, fn, "(workspace) NULL or not 256-byte aligned");
    if (ws_bytes < need) return bad_arg(15, fn, "(ws_bytes) below gemm_splitk_workspace_bytes");
  }
  GemmArgs g{M, N, K, alpha, beta, A, lda, B, ldb, C, ldc};
  return bx3_run_splitk(g, n_products, splits, workspace, stream);
}

gemm_status split_bf16x3(int64_t n, const float *x, uint16_t *p0, uint16_t *p1, uint16_t *p2,
                         hipStream_t stream) {
  clear_error();
  const char *fn = "split_bf16x3";
  if (n < 0) return bad_arg(1, fn, "(n) must be >= 0");
  if (n == 0) return GEMM_STATUS_OK;
  if (!x) return bad_arg(2, fn, "(x) is NULL");
  if (!p0) return bad_arg(3, fn, "(p0) is NULL");
  if (!p1) return bad_arg(4, fn, "(p1) is NULL");
  return bx3_split(n, x, p0, p1, p2, stream);
}

size_t gemm_fp8_workspace_bytes(int64_t M, int64_t N, int64_t K) {
  if (M < 0 || N < 0 || K < 0) return 0;
  return fp8_ws_bytes(M, N, K);
}

static gemm_status fp8_check_ws(const char *fn, int idx, int64_t M, int64_t N, int64_t K,
                                const void *ws, size_t ws_bytes) {
  if (!ws) return bad_arg(idx, fn, "(workspace) is NULL");
  if (((uintptr_t)ws & 255) != 0) return bad_arg(idx, fn, "(workspace) must be 256-byte aligned");
  if (ws_bytes < fp8_ws_bytes(M, N, K)) return bad_arg(idx + 1, fn, "(ws_bytes) too small");
  return GEMM_STATUS_OK;
}

gemm_status gemm_fp8_scaled(int64_t M, int64_t N, int64_t K, float alpha, const float *A,
                            int64_t lda, const float *B, int64_t ldb, float beta, float *C,
                            int64_t ldc, void *workspace, size_t ws_bytes, hipStream_t stream) {
  clear_error();
  const char *fn = "gemm_fp8_scaled";
  Checked ck;
  gemm_status st = check_gemm_args(fn, M, N, K, alpha, A, lda, B, ldb, C, ldc, ck);
  if (st || ck.noop) return st;
  if (ck.scale_only) return scale_c(M, N, beta, C, ldc, stream);
  if ((st = fp8_check_ws(fn, 12, M, N, K, workspace, ws_bytes))) return st;
  if ((st = fp8_quantize_run(M, N, K, A, lda, B, ldb, workspace, stream))) return st;
  return fp8_gemm_run_cfg(M, N, K, alpha, workspace, beta, C, ldc,
                          pick_config(GEMM_PATH_FP8, 3, M, N, K), stream);
}

gemm_status fp8_quantize(int64_t M, int64_t N, int64_t K, const float *A, int64_t lda,
                         const float *B, int64_t ldb, void *workspace, size_t ws_bytes,
                         hipStream_t stream) {
  clear_error();
  const char *fn = "fp8_quantize";
  if (M < 0) return bad_arg(1, fn, "(M) must be >= 0");
  if (N < 0) return bad_arg(2, fn, "(N) must be >= 0");
  if (K < 0) return bad_arg(3, fn, "(K) must be >= 0");
  if (M > 0x7fffffffLL || N > 0x7fffffffLL || K > 0x7fffffffLL) return bad_arg(1, fn, "size exceeds 2^31-1");
  if (M > 0 && K > 0 && !A) return bad_arg(4, fn, "(A) is NULL");
  if (lda < (K > 1 ? K : 1)) return bad_arg(5, fn, "(lda) must be >= max(1,K)");
  if (N > 0 && K > 0 && !B) return bad_arg(6, fn, "(B) is NULL");
  if (ldb < (N > 1 ? N : 1)) return bad_arg(7, fn, "(ldb) must be >= max(1,N)");
  gemm_status st = fp8_check_ws(fn, 8, M, N, K, workspace, ws_bytes);
  if (st) return st;
  return fp8_quantize_run(M, N, K, A, lda, B, ldb, workspace, stream);
}

gemm_status gemm_fp8_prequantized(int64_t M, int64_t N, int64_t K, float alpha,
                                  const void *workspace, size_t ws_bytes, float beta, float *C,
                                  int64_t ldc, hipStream_t stream) {
  clear_error();
  const char *fn = "gemm_fp8_prequantized";
  if (M < 0) return bad_arg(1, fn, "(M) must be >= 0");
  if (N < 0) return bad_arg(2, fn, "(N) must be >= 0");
  if (K < 0) return bad_arg(3, fn, "(K) must be >= 0");
  if (M > 0x7fffffffLL || N > 0x7fffffffLL || K > 0x7fffffffLL) return bad_arg(1, fn, "size exceeds 2^31-1");
  gemm_status st = fp8_check_ws(fn, 5, M, N, K, workspace, ws_bytes);
  if (st) return st;
  if (ldc < (N > 1 ? N : 1)) return bad_arg(9, fn, "(ldc) must be >= max(1,N)");
  if (M == 0 || N == 0) return GEMM_STATUS_OK;
  if (!C) return bad_arg(8, fn, "(C) is NULL");
  if (alpha == 0.0f || K == 0) return scale_c(M, N, beta, C, ldc, stream);
  return fp8_gemm_run_cfg(M, N, K, alpha, workspace, beta, C, ldc,
                          pick_config(GEMM_PATH_FP8, 3, M, N, K), stream);
}

gemm_status fp8_e4m3_encode(int64_t n, const float *x, uint8_t *codes, hipStream_t stream) {
  clear_error();
  const char *fn = "fp8_e4m3_encode";
  if (n < 0) return bad_arg(1, fn, "(n) must be >= 0");
  if (n == 0) return GEMM_STATUS_OK;
  if (!x) return bad_arg(2, fn, "(x) is NULL");
  if (!codes) return bad_arg(3, fn, "(codes) is NULL");
  return fp8_encode_run(n, x, codes, stream);
}

int gemm_num_configs(int path) {
  switch (path) {
    case GEMM_PATH_F64: return f64_num_configs();
    case GEMM_PATH_F32: return f32_num_configs();
    case GEMM_PATH_3XBF16: return bx3_num_configs();
    case GEMM_PATH_FP8:
    case GEMM_PATH_FP8_PREQUANTIZED: return fp8_num_configs();
    default: return 0;
  }
}

const char *gemm_config_name(int path, int cfg) {
  if (cfg < 0 || cfg >= gemm_num_configs(path)) return "";
  switch (path) {
    case GEMM_PATH_F32: return f32_config(cfg).name;
    case GEMM_PATH_3XBF16: return bx3_config(cfg).name;
    case GEMM_PATH_FP8:
    case GEMM_PATH_FP8_PREQUANTIZED: return fp8_config_name(cfg);
    case GEMM_PATH_F64: return f64_config(cfg).name;
    default: return "";
  }
}

int gemm_default_config(int path, int64_t M, int64_t N, int64_t K) {
  if (path == GEMM_PATH_F64) return f64_default_config(M, N, K, 1);
  if (path < GEMM_PATH_F32 || path > GEMM_PATH_FP8_PREQUANTIZED) return -1;
  return pick_config(path, 3, M, N, K);
}

gemm_status gemm_run_config(int path, int cfg, int64_t M, int64_t N, int64_t K, float alpha,
                            const float *A, int64_t lda, const float *B, int64_t ldb, float beta,
                            float *C, int64_t ldc, int n_products, void *workspace,
                            size_t ws_bytes, hipStream_t stream) {
  clear_error();
  const char *fn = "gemm_run_config";
  if (gemm_num_configs(path) == 0) return bad_arg(1, fn, "(path) unknown or not built");
  if (path == GEMM_PATH_F64) return bad_arg(1, fn, "(path) binary64 operands go through gemm_f64_run_config");
  if (cfg < -1 || cfg >= gemm_num_configs(path)) return bad_arg(2, fn, "(cfg) out of range");
  if (path == GEMM_PATH_FP8_PREQUANTIZED) {  // operands are the workspace's codes
    if (M < 0) return bad_arg(3, fn, "(M) must be >= 0");
    if (N < 0) return bad_arg(4, fn, "(N) must be >= 0");
    if (K < 0) return bad_arg(5, fn, "(K) must be >= 0");
    if (M > 0x7fffffffLL || N > 0x7fffffffLL || K > 0x7fffffffLL)
      return bad_arg(3, fn, "size exceeds 2^31-1");
    gemm_status st = fp8_check_ws(fn, 15, M, N, K, workspace, ws_bytes);
    if (st) return st;
    if (ldc < (N > 1 ? N : 1)) return bad_arg(13, fn, "(ldc) must be >= max(1,N)");
    if (M == 0 || N == 0) return GEMM_STATUS_OK;
    if (!C) return bad_arg(12, fn, "(C) is NULL");
    if (alpha == 0.0f || K == 0) return scale_c(M, N, beta, C, ldc, stream);
    if (cfg < 0) cfg = pick_config(GEMM_PATH_FP8, 3, M, N, K);
    return fp8_gemm_run_cfg(M, N, K, alpha, workspace, beta, C, ldc, cfg, stream);
  }
  Checked ck;
  gemm_status st = check_gemm_args(fn, M, N, K, alpha, A, lda, B, ldb, C, ldc, ck);
  if (st < 0) {  // argument index shifted by (path, cfg)
    set_error(std::string(fn) + ": argument " + std::to_string(2 - st) + " invalid");
    return st - 2;
  }
  if (path == GEMM_PATH_3XBF16) {
    if (n_products != 3 && n_products != 6) return bad_arg(14, fn, "(n_products) must be 3 or 6");
    if (cfg >= 0 && bx3_config_products(cfg) != n_products)
      return bad_arg(14, fn, "(n_products) does not match the configuration");
  }
  if (st || ck.noop) return st;
  if (ck.scale_only) return scale_c(M, N, beta, C, ldc, stream);
  if (path == GEMM_PATH_FP8) {
    if ((st = fp8_check_ws(fn, 15, M, N, K, workspace, ws_bytes))) return st;
    if ((st = fp8_quantize_run(M, N, K, A, lda, B, ldb, workspace, stream))) return st;
    if (cfg < 0) cfg = pick_config(GEMM_PATH_FP8, 3, M, N, K);
    return fp8_gemm_run_cfg(M, N, K, alpha, workspace, beta, C, ldc, cfg, stream);
  }
  GemmArgs g{M, N, K, alpha, beta, A, lda, B, ldb, C, ldc};
  if (cfg < 0) cfg = pick_config(path, n_products, M, N, K);
  switch (path) {
    case GEMM_PATH_F32: return f32_run(g, cfg, stream);
    case GEMM_PATH_3XBF16: return bx3_run(g, cfg, stream);
    default: return GEMM_STATUS_UNSUPPORTED;
  }
}

gemm_status gemm_ex(int order, int trans_a, int trans_b, int64_t M, int64_t N, int64_t K,
                    float alpha, const float *A, int64_t lda, const float *B, int64_t ldb,
                    float beta, float *C, int64_t ldc, int path, int n_products, void *workspace,
                    size_t ws_bytes, hipStream_t stream) {
  clear_error();
  const char *fn = "gemm_ex";
  if (order != GEMM_ROW_MAJOR && order != GEMM_COL_MAJOR) return bad_arg(1, fn, "(order) unknown");
  auto is_trans = [](int t) { return t == GEMM_TRANS || t == GEMM_CONJ_TRANS; };
  if (trans_a != GEMM_NO_TRANS && !is_trans(trans_a)) return bad_arg(2, fn, "(trans_a) unknown");
  if (trans_b != GEMM_NO_TRANS && !is_trans(trans_b)) return bad_arg(3, fn, "(trans_b) unknown");
  const bool ta = is_trans(trans_a), tb = is_trans(trans_b);
  if (M < 0) return bad_arg(4, fn, "(M) must be >= 0");
  if (N < 0) return bad_arg(5, fn, "(N) must be >= 0");
  if (K < 0) return bad_arg(6, fn, "(K) must be >= 0");
  if (M > 0x7fffffffLL || N > 0x7fffffffLL || K > 0x7fffffffLL)
    return bad_arg(M > 0x7fffffffLL ? 4 : N > 0x7fffffffLL ? 5 : 6, fn, "exceeds 2^31-1");
  // Stored extents along the contiguous index: row-major op(A) = A is M x K
  // (row length K), A^T is stored K x M (row length M); column-major swaps
  // the roles of rows and columns.
  const bool row = order == GEMM_ROW_MAJOR;
  const int64_t min_lda = row ? (ta ? M : K) : (ta ? K : M);
  const int64_t min_ldb = row ? (tb ? K : N) : (tb ? N : K);
  const int64_t min_ldc = row ? N : M;
  if (lda < (min_lda > 1 ? min_lda : 1)) return bad_arg(9, fn, "(lda) below the stored row length");
  if (ldb < (min_ldb > 1 ? min_ldb : 1)) return bad_arg(11, fn, "(ldb) below the stored row length");
  if (ldc < (min_ldc > 1 ? min_ldc : 1)) return bad_arg(14, fn, "(ldc) below the stored row length");
  if (path != GEMM_PATH_F32 && path != GEMM_PATH_3XBF16 && path != GEMM_PATH_FP8)
    return bad_arg(15, fn, "(path) must be GEMM_PATH_F32, GEMM_PATH_3XBF16 or GEMM_PATH_FP8");
  if (path == GEMM_PATH_3XBF16 && n_products != 3 && n_products != 6)
    return bad_arg(16, fn, "(n_products) must be 3 or 6");
  if (M == 0 || N == 0) return GEMM_STATUS_OK;
  if (!C) return bad_arg(13, fn, "(C) is NULL");
  // Column-major C (M x N) is row-major C^T (N x M) = op(B)^T op(A)^T: the
  // operands swap places and each keeps its transpose flag.
  GemmArgs g = row ? GemmArgs{M, N, K, alpha, beta, A, lda, B, ldb, C, ldc}
                   : GemmArgs{N, M, K, alpha, beta, B, ldb, A, lda, C, ldc};
  g.ta = row ? ta : tb;
  g.tb = row ? tb : ta;
  if (alpha == 0.0f || K == 0) return scale_c(g.M, g.N, beta, C, ldc, stream);
  if (!A) return bad_arg(8, fn, "(A) is NULL");
  if (!B) return bad_arg(10, fn, "(B) is NULL");
  if (path == GEMM_PATH_FP8) {
    gemm_status st = fp8_check_ws(fn, 17, g.M, g.N, K, workspace, ws_bytes);
    if (st) return st;
    if ((st = fp8_quantize_run(g.M, g.N, K, g.A, g.lda, g.B, g.ldb, workspace, stream, g.ta, g.tb)))
      return st;
    return fp8_gemm_run_cfg(g.M, g.N, K, alpha, workspace, beta, C, ldc,
                            pick_config(GEMM_PATH_FP8, 3, g.M, g.N, K), stream);
  }
  const bool trans = g.ta || g.tb;
  if (path == GEMM_PATH_F32) {
    // transposed operands run on the FP32 matrix-core and small-product
    // tiles only
    int cfg = pick_config(GEMM_PATH_F32, 0, g.M, g.N, K);
    if (trans && (cfg < 5 || cfg > 8)) {
      const int64_t big = ((g.M + 255) / 256) * ((g.N + 255) / 256);
      cfg = big >= num_cus() ? 5 : 6;
    }
    return f32_run(g, cfg, stream);
  }
  int cfg = trans ? bx3_default_config(g.M, g.N, K, n_products)
                  : pick_config(GEMM_PATH_3XBF16, n_products, g.M, g.N, K);
  // the two-group tile has no transposed-operand variant: its one-group form
  if (trans && cfg == 14) cfg = 8;
  // with only B transposed the 32-deep 256 x 256 tile measured 8 % faster
  // than the 16-deep one that is the default otherwise
  if (cfg == 0 && !g.ta && g.tb) cfg = 3;
  return bx3_run(g, cfg, stream);
}

gemm_status gemm_f64(int64_t M, int64_t N, int64_t K, double alpha, const double *A,
                     int64_t lda, const double *B, int64_t ldb, double beta, double *C,
                     int64_t ldc, hipStream_t stream) {
  clear_error();
  Checked ck;
  gemm_status st = check_gemm_args("gemm_f64", M, N, K, alpha, A, lda, B, ldb, C, ldc, ck);
  if (st || ck.noop) return st;
  if (ck.scale_only) return scale_c_f64(M, N, beta, C, ldc, 0, 1, stream);
  GemmArgsF64 g{M, N, K, alpha, beta, A, lda, 0, B, ldb, 0, C, ldc, 0, 1};
  return f64_run(g, f64_default_config(M, N, K, 1), stream);
}

gemm_status gemm_f64_run_config(int cfg, int64_t M, int64_t N, int64_t K, double alpha,
                                const double *A, int64_t lda, const double *B, int64_t ldb,
                                double beta, double *C, int64_t ldc, hipStream_t stream) {
  clear_error();
  const char *fn = "gemm_f64_run_config";
  if (cfg < -1 || cfg >= f64_num_configs()) return bad_arg(1, fn, "(cfg) out of range");
  Checked ck;
  gemm_status st = check_gemm_args(fn, M, N, K, alpha, A, lda, B, ldb, C, ldc, ck);
  if (st < 0) {  // argument index shifted by cfg
    set_error(std::string(fn) + ": argument " + std::to_string(1 - st) + " invalid");
    return st - 1;
  }
  if (ck.noop) return GEMM_STATUS_OK;
  if (ck.scale_only) return scale_c_f64(M, N, beta, C, ldc, 0, 1, stream);
  GemmArgsF64 g{M, N, K, alpha, beta, A, lda, 0, B, ldb, 0, C, ldc, 0, 1};
  return f64_run(g, cfg < 0 ? f64_default_config(M, N, K, 1) : cfg, stream);
}

gemm_status gemm_f64_strided_batched(int64_t M, int64_t N, int64_t K, double alpha,
                                     const double *A, int64_t lda, int64_t stride_a,
                                     const double *B, int64_t ldb, int64_t stride_b, double beta,
                                     double *C, int64_t ldc, int64_t stride_c, int64_t batch,
                                     hipStream_t stream) {
  clear_error();
  const char *fn = "gemm_f64_strided_batched";
  if (M < 0) return bad_arg(1, fn, "(M) must be >= 0");
  if (N < 0) return bad_arg(2, fn, "(N) must be >= 0");
  if (K < 0) return bad_arg(3, fn, "(K) must be >= 0");
  if (M > 0x7fffffffLL || N > 0x7fffffffLL || K > 0x7fffffffLL)
    return bad_arg(M > 0x7fffffffLL ? 1 : N > 0x7fffffffLL ? 2 : 3, fn, "exceeds 2^31-1");
  if (lda < (K > 1 ? K : 1)) return bad_arg(6, fn, "(lda) must be >= max(1,K)");
  if (stride_a < 0) return bad_arg(7, fn, "(stride_a) must be >= 0");
  if (ldb < (N > 1 ? N : 1)) return bad_arg(9, fn, "(ldb) must be >= max(1,N)");
  if (stride_b < 0) return bad_arg(10, fn, "(stride_b) must be >= 0");
  if (ldc < (N > 1 ? N : 1)) return bad_arg(13, fn, "(ldc) must be >= max(1,N)");
  if (batch < 0) return bad_arg(15, fn, "(batch) must be >= 0");
  // outputs of different problems must not overlap (they are written concurrently)
  if (batch > 1 && M > 0 && N > 0 && stride_c < (M - 1) * ldc + N)
    return bad_arg(14, fn, "(stride_c) smaller than one output matrix");
  if (M == 0 || N == 0 || batch == 0) return GEMM_STATUS_OK;
  if (!C) return bad_arg(12, fn, "(C) is NULL");
  if (alpha == 0.0 || K == 0) {
    for (int64_t b0 = 0; b0 < batch; b0 += 65535) {
      const int64_t nb = std::min<int64_t>(65535, batch - b0);
      if (gemm_status st = scale_c_f64(M, N, beta, C + b0 * stride_c, ldc, stride_c, nb, stream))
        return st;
    }
    return GEMM_STATUS_OK;
  }
  if (!A) return bad_arg(5, fn, "(A) is NULL");
  if (!B) return bad_arg(8, fn, "(B) is NULL");
  const int cfg = f64_default_config(M, N, K, batch);
  // the grid's second dimension holds at most 65535 problems per launch
  for (int64_t b0 = 0; b0 < batch; b0 += 65535) {
    const int64_t nb = std::min<int64_t>(65535, batch - b0);
    GemmArgsF64 g{M, N, K, alpha, beta, A + b0 * stride_a, lda, stride_a, B + b0 * stride_b, ldb,
                  stride_b, C + b0 * stride_c, ldc, stride_c, nb};
    if (gemm_status st = f64_run(g, cfg, stream)) return st;
  }
  return GEMM_STATUS_OK;
}

gemm_status gemm_strided_batched(int path, int64_t M, int64_t N, int64_t K, float alpha,
                                 const float *A, int64_t lda, int64_t stride_a, const float *B,
                                 int64_t ldb, int64_t stride_b, float beta, float *C, int64_t ldc,
                                 int64_t stride_c, int64_t batch, int n_products,
                                 hipStream_t stream) {
  clear_error();
  const char *fn = "gemm_strided_batched";
  if (path != GEMM_PATH_F32 && path != GEMM_PATH_3XBF16)
    return bad_arg(1, fn, "(path) must be GEMM_PATH_F32 or GEMM_PATH_3XBF16");
  if (M < 0) return bad_arg(2, fn, "(M) must be >= 0");
  if (N < 0) return bad_arg(3, fn, "(N) must be >= 0");
  if (K < 0) return bad_arg(4, fn, "(K) must be >= 0");
  if (M > 0x7fffffffLL || N > 0x7fffffffLL || K > 0x7fffffffLL)
    return bad_arg(M > 0x7fffffffLL ? 2 : N > 0x7fffffffLL ? 3 : 4, fn, "exceeds 2^31-1");
  if (lda < (K > 1 ? K : 1)) return bad_arg(7, fn, "(lda) must be >= max(1,K)");
  if (stride_a < 0) return bad_arg(8, fn, "(stride_a) must be >= 0");
  if (ldb < (N > 1 ? N : 1)) return bad_arg(10, fn, "(ldb) must be >= max(1,N)");
  if (stride_b < 0) return bad_arg(11, fn, "(stride_b) must be >= 0");
  if (ldc < (N > 1 ? N : 1)) return bad_arg(14, fn, "(ldc) must be >= max(1,N)");
  if (batch < 0) return bad_arg(16, fn, "(batch) must be >= 0");
  if (batch > 1 && M > 0 && N > 0 && stride_c < (M - 1) * ldc + N)
    return bad_arg(15, fn, "(stride_c) smaller than one output matrix");
  if (path == GEMM_PATH_3XBF16 && n_products != 3 && n_products != 6)
    return bad_arg(17, fn, "(n_products) must be 3 or 6");
  if (M == 0 || N == 0 || batch == 0) return GEMM_STATUS_OK;
  if (!C) return bad_arg(13, fn, "(C) is NULL");
  if (alpha == 0.0f || K == 0) return scale_c_batched(M, N, beta, C, ldc, stride_c, batch, stream);
  if (!A) return bad_arg(6, fn, "(A) is NULL");
  if (!B) return bad_arg(9, fn, "(B) is NULL");
  const int cfg = batched_config(path, n_products, M, N, K, batch);
  for (int64_t b0 = 0; b0 < batch; b0 += 65535) {
    const int nb = (int)std::min<int64_t>(65535, batch - b0);
    GemmArgs g{M, N, K, alpha, beta, A + b0 * stride_a, lda, B + b0 * stride_b, ldb,
               C + b0 * stride_c, ldc};
    if (gemm_status st = batched_run(path, cfg, g, stride_a, stride_b, stride_c, nb, stream))
      return st;
  }
  return GEMM_STATUS_OK;
}

size_t err_norm_workspace_bytes(void) { return errnorm_ws_bytes(); }

gemm_status err_norm_f64(int64_t M, int64_t N, const float *C, int64_t ldc, const double *Cref,
                         const double *den, double *out, void *workspace, size_t ws_bytes,
                         hipStream_t stream) {
  clear_error();
  const char *fn = "err_norm_f64";
  if (M < 0) return bad_arg(1, fn, "(M) must be >= 0");
  if (N < 0) return bad_arg(2, fn, "(N) must be >= 0");
  if (M * N > 0 && !C) return bad_arg(3, fn, "(C) is NULL");
  if (ldc < (N > 1 ? N : 1)) return bad_arg(4, fn, "(ldc) must be >= max(1,N)");
  if (M * N > 0 && !Cref) return bad_arg(5, fn, "(Cref) is NULL");
  if (!out) return bad_arg(7, fn, "(out) is NULL");
  if (!workspace) return bad_arg(8, fn, "(workspace) is NULL");
  if (ws_bytes < errnorm_ws_bytes()) return bad_arg(9, fn, "(ws_bytes) too small");
  return errnorm_run(M, N, C, ldc, Cref, den, out, workspace, stream);
}

}  // extern "C"
