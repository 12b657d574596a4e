// bx3_launch.hpp -- kernels and launchers of the one-pass MFMA GEMM tiles
// (split-precision bf16 planes, or binary32 on the FP32 matrix cores), for
// every combination of transposed operands.
#pragma once

#include "bf16x3.hpp"

namespace mm {
namespace bx3 {

template <int BM, int BN, int BK, int WM, int WN, int NP, int NW, bool VEC, bool BETA, bool TA,
          bool TB, int ST = 2>
__global__ __launch_bounds__(64 * NW, 1) void gemm_bx3_kernel(
    int M, int N, int K, float alpha, const float *__restrict__ A, int64_t lda,
    const float *__restrict__ B, int64_t ldb, float beta, float *__restrict__ C, int64_t ldc,
    int tiles_m, int tiles_n) {
  using G = Cfg<BM, BN, BK, WM, WN, NP, NW, ST>;
  __shared__ __attribute__((aligned(16))) __bf16 lds[G::LDS_BYTES / 2];
  const int wg = xcd_remap(blockIdx.x, gridDim.x);
  int tm, tn;
  tile_coords(wg, tiles_m, tiles_n, 8, tm, tn);
  tile<BM, BN, BK, WM, WN, NP, NW, VEC, BETA, TA, TB, ST>(M, N, K, alpha, A, lda, B, ldb, beta,
                                                          C, ldc, tm * BM, tn * BN, lds);
}

// The tile with its k range split between two groups of NW waves (one
// workgroup of 2 * NW waves per tile): twice the waves per SIMD of the
// one-group tile where its tiles come to about one per CU.
template <int BM, int BN, int BK, int WM, int WN, int NP, int NW, bool VEC, bool BETA>
__global__ __launch_bounds__(128 * NW, 1) void gemm_bx3_kg_kernel(
    int M, int N, int K, float alpha, const float *__restrict__ A, int64_t lda,
    const float *__restrict__ B, int64_t ldb, float beta, float *__restrict__ C, int64_t ldc,
    int tiles_m, int tiles_n) {
  using G = Cfg<BM, BN, BK, WM, WN, NP, NW>;
  __shared__ __attribute__((aligned(16))) __bf16 lds[2 * G::LDS_BYTES / 2];
  const int wg = xcd_remap(blockIdx.x, gridDim.x);
  int tm, tn;
  tile_coords(wg, tiles_m, tiles_n, 8, tm, tn);
  tile<BM, BN, BK, WM, WN, NP, NW, VEC, BETA, false, false, 2, 0, 2>(
      M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, tm * BM, tn * BN, lds);
}

// The plain binary32 product on the FP32 matrix cores (v_mfma_f32_32x32x2f32):
// the same tile body in its FP32 mode (no split; binary32 in LDS).
template <int BM, int BN, int BK, int WM, int WN, int NW, bool VEC, bool BETA, bool TA, bool TB>
__global__ __launch_bounds__(64 * NW, 1) void gemm_f32mfma_kernel(
    int M, int N, int K, float alpha, const float *__restrict__ A, int64_t lda,
    const float *__restrict__ B, int64_t ldb, float beta, float *__restrict__ C, int64_t ldc,
    int tiles_m, int tiles_n) {
  using G = Cfg<BM, BN, BK, WM, WN, 1, NW>;
  __shared__ __attribute__((aligned(16))) __bf16 lds[G::LDS_BYTES / 2];
  const int wg = xcd_remap(blockIdx.x, gridDim.x);
  int tm, tn;
  tile_coords(wg, tiles_m, tiles_n, 8, tm, tn);
  tile<BM, BN, BK, WM, WN, 1, NW, VEC, BETA, TA, TB>(M, N, K, alpha, A, lda, B, ldb, beta, C,
                                                     ldc, tm * BM, tn * BN, lds);
}

// Byte extents the tile body addresses with 32-bit offsets: a k-contiguous
// operand's tile panel (ROWS rows of its row stride, plus K), or a
// row-index-contiguous operand's slab (BK rows of its row stride, plus the
// row-index extent).  Both must stay below 2^31.
template <int BM, int BN, int BK, bool TA, bool TB>
inline bool offsets_fit(const GemmArgs &g) {
  const int64_t ea = TA ? (int64_t)BK * g.lda + g.M : (int64_t)BM * g.lda + g.K;
  const int64_t eb = TB ? (int64_t)BN * g.ldb + g.K : (int64_t)BK * g.ldb + g.N;
  return ea * 4 < ((int64_t)1 << 31) && eb * 4 < ((int64_t)1 << 31);
}

// 128-bit staging loads need every k-contiguous operand (A unless TA, B if
// TB) to have a row stride that is a multiple of 4 floats and a 16-byte
// aligned base; the slab grid ends at K, so K must be a multiple of 4 too.
template <bool TA, bool TB>
inline bool vector_loads_ok(const GemmArgs &g) {
  if (TA && !TB) return false;  // no k-contiguous operand
  bool v = g.K % 4 == 0;
  if (!TA) v = v && g.lda % 4 == 0 && ((uintptr_t)g.A & 15) == 0;
  if (TB) v = v && g.ldb % 4 == 0 && ((uintptr_t)g.B & 15) == 0;
  return v;
}

template <int BM, int BN, int BK, int WM, int WN, int NW, bool TA = false, bool TB = false>
gemm_status launch_f32mfma(const GemmArgs &g, hipStream_t s) {
  const int tiles_m = (int)((g.M + BM - 1) / BM);
  const int tiles_n = (int)((g.N + BN - 1) / BN);
  const int64_t nwg = (int64_t)tiles_m * tiles_n;
  if (nwg > 0x7fffffff) { set_error("gemm_f32: too many tiles"); return GEMM_STATUS_UNSUPPORTED; }
  if (!offsets_fit<BM, BN, BK, TA, TB>(g)) {
    set_error("gemm_f32: lda or ldb too large for 32-bit tile offsets");
    return GEMM_STATUS_UNSUPPORTED;
  }
  const bool vec = vector_loads_ok<TA, TB>(g);
  const bool beta = g.beta != 0.0f;
  dim3 grid((unsigned)nwg), block(64 * NW);
#define MM_LAUNCH(V, BT)                                                                  \
  hipLaunchKernelGGL((gemm_f32mfma_kernel<BM, BN, BK, WM, WN, NW, V, BT, TA, TB>), grid, \
                     block, 0, s, (int)g.M, (int)g.N, (int)g.K, g.alpha, g.A, g.lda, g.B,  \
                     g.ldb, g.beta, g.C, g.ldc, tiles_m, tiles_n)
  if constexpr (!TA || TB) {
    if (vec) {
      if (beta) MM_LAUNCH(true, true); else MM_LAUNCH(true, false);
      return check_launch("gemm_f32mfma_kernel");
    }
  }
  if (beta) MM_LAUNCH(false, true); else MM_LAUNCH(false, false);
#undef MM_LAUNCH
  return check_launch("gemm_f32mfma_kernel");
}

template <int BM, int BN, int BK, int WM, int WN, int NP, int NW, bool TA = false, bool TB = false,
          int ST = 2>
gemm_status launch(const GemmArgs &g, hipStream_t s) {
  const int tiles_m = (int)((g.M + BM - 1) / BM);
  const int tiles_n = (int)((g.N + BN - 1) / BN);
  const int64_t nwg = (int64_t)tiles_m * tiles_n;
  if (nwg > 0x7fffffff) { set_error("gemm_f32_3xbf16: too many tiles"); return GEMM_STATUS_UNSUPPORTED; }
  if (!offsets_fit<BM, BN, BK, TA, TB>(g)) {
    set_error("gemm_f32_3xbf16: lda or ldb too large for 32-bit tile offsets");
    return GEMM_STATUS_UNSUPPORTED;
  }
  const bool vec = vector_loads_ok<TA, TB>(g);
  const bool beta = g.beta != 0.0f;
  dim3 grid((unsigned)nwg), block(64 * NW);
#define MM_LAUNCH(V, BT)                                                                     \
  hipLaunchKernelGGL((gemm_bx3_kernel<BM, BN, BK, WM, WN, NP, NW, V, BT, TA, TB, ST>), grid, \
                     block, 0, s, (int)g.M, (int)g.N, (int)g.K, g.alpha, g.A, g.lda, g.B,     \
                     g.ldb, g.beta, g.C, g.ldc, tiles_m, tiles_n)
  if constexpr (!TA || TB) {
    if (vec) {
      if (beta) MM_LAUNCH(true, true); else MM_LAUNCH(true, false);
      return check_launch("gemm_bx3_kernel");
    }
  }
  if (beta) MM_LAUNCH(false, true); else MM_LAUNCH(false, false);
#undef MM_LAUNCH
  return check_launch("gemm_bx3_kernel");
}

// A batch of equally shaped problems at fixed element strides: the tiles of
// one problem in the grid's first dimension (XCD-aware order), the problem in
// the second.  NP == 1 is the binary32 matrix-core mode.
template <int BM, int BN, int BK, int WM, int WN, int NP, int NW, bool VEC, bool BETA>
__global__ __launch_bounds__(64 * NW, 1) void gemm_batched_kernel(
    int M, int N, int K, float alpha, const float *__restrict__ A, int64_t lda, int64_t sa,
    const float *__restrict__ B, int64_t ldb, int64_t sb, float beta, float *__restrict__ C,
    int64_t ldc, int64_t sc, int tiles_m, int tiles_n) {
  using G = Cfg<BM, BN, BK, WM, WN, NP, NW>;
  __shared__ __attribute__((aligned(16))) __bf16 lds[G::LDS_BYTES / 2];
  const int wg = xcd_remap(blockIdx.x, gridDim.x);
  int tm, tn;
  tile_coords(wg, tiles_m, tiles_n, 8, tm, tn);
  const int64_t b = blockIdx.y;
  tile<BM, BN, BK, WM, WN, NP, NW, VEC, BETA>(M, N, K, alpha, A + b * sa, lda, B + b * sb, ldb,
                                              beta, C + b * sc, ldc, tm * BM, tn * BN, lds);
}

// Up to 65535 problems per launch (the grid's second dimension).
template <int BM, int BN, int BK, int WM, int WN, int NP, int NW>
gemm_status launch_batched(const GemmArgs &g, int64_t sa, int64_t sb, int64_t sc, int batch,
                           hipStream_t s) {
  const int tiles_m = (int)((g.M + BM - 1) / BM);
  const int tiles_n = (int)((g.N + BN - 1) / BN);
  const int64_t nwg = (int64_t)tiles_m * tiles_n;
  if (nwg > 0x7fffffff || batch > 65535) {
    set_error("gemm_strided_batched: too many tiles or problems for one launch");
    return GEMM_STATUS_UNSUPPORTED;
  }
  if (!offsets_fit<BM, BN, BK, false, false>(g)) {
    set_error("gemm_strided_batched: lda or ldb too large for 32-bit tile offsets");
    return GEMM_STATUS_UNSUPPORTED;
  }
  // 128-bit A loads need every problem's A 16-byte aligned
  const bool vec = vector_loads_ok<false, false>(g) && sa % 4 == 0;
  const bool beta = g.beta != 0.0f;
  const dim3 grid((unsigned)nwg, (unsigned)batch), block(64 * NW);
#define MM_LAUNCH(V, BT)                                                                        \
  hipLaunchKernelGGL((gemm_batched_kernel<BM, BN, BK, WM, WN, NP, NW, V, BT>), grid, block, 0, s, \
                     (int)g.M, (int)g.N, (int)g.K, g.alpha, g.A, g.lda, sa, g.B, g.ldb, sb,       \
                     g.beta, g.C, g.ldc, sc, tiles_m, tiles_n)
  if (vec) { if (beta) MM_LAUNCH(true, true); else MM_LAUNCH(true, false); }
  else     { if (beta) MM_LAUNCH(false, true); else MM_LAUNCH(false, false); }
#undef MM_LAUNCH
  return check_launch("gemm_batched_kernel");
}

// The tile configurations that have transposed-operand variants (the ones the
// library picks by default): 0, 2, 3, 4, 5, 6 and 8 of the split path, both
// FP32 matrix-core tiles.
// Two k-groups per workgroup; K odd has no equal halves (UNSUPPORTED: the
// configuration choice sends such shapes elsewhere).
template <int BM, int BN, int BK, int WM, int WN, int NP, int NW>
gemm_status launch_kg(const GemmArgs &g, hipStream_t s) {
  if (g.K % 2 != 0) {
    set_error("gemm_f32_3xbf16: the two-group configuration needs an even K");
    return GEMM_STATUS_UNSUPPORTED;
  }
  const int tiles_m = (int)((g.M + BM - 1) / BM);
  const int tiles_n = (int)((g.N + BN - 1) / BN);
  const int64_t nwg = (int64_t)tiles_m * tiles_n;
  if (nwg > 0x7fffffff) { set_error("gemm_f32_3xbf16: too many tiles"); return GEMM_STATUS_UNSUPPORTED; }
  if (!offsets_fit<BM, BN, BK, false, false>(g)) {
    set_error("gemm_f32_3xbf16: lda or ldb too large for 32-bit tile offsets");
    return GEMM_STATUS_UNSUPPORTED;
  }
  // each group's panel starts K/2 elements into a row of A
  const bool vec = vector_loads_ok<false, false>(g) && (g.K / 2) % 4 == 0;
  const bool beta = g.beta != 0.0f;
  dim3 grid((unsigned)nwg), block(128 * NW);
#define MM_LAUNCH(V, BT)                                                                   \
  hipLaunchKernelGGL((gemm_bx3_kg_kernel<BM, BN, BK, WM, WN, NP, NW, V, BT>), grid, block, \
                     0, s, (int)g.M, (int)g.N, (int)g.K, g.alpha, g.A, g.lda, g.B, g.ldb,  \
                     g.beta, g.C, g.ldc, tiles_m, tiles_n)
  if (vec) { if (beta) MM_LAUNCH(true, true); else MM_LAUNCH(true, false); }
  else     { if (beta) MM_LAUNCH(false, true); else MM_LAUNCH(false, false); }
#undef MM_LAUNCH
  return check_launch("gemm_bx3_kg_kernel");
}

template <bool TA, bool TB>
gemm_status bx3_run_trans(const GemmArgs &g, int cfg, hipStream_t s) {
  switch (cfg) {
    case 0: return launch<256, 256, 16, 128, 64, 2, 8, TA, TB>(g, s);
    case 2: return launch<256, 128, 32, 64, 64, 2, 8, TA, TB>(g, s);
    case 3: return launch<256, 256, 32, 128, 64, 2, 8, TA, TB>(g, s);
    case 4: return launch<256, 256, 16, 128, 64, 3, 8, TA, TB>(g, s);
    case 5: return launch<128, 128, 32, 64, 64, 3, 4, TA, TB>(g, s);
    case 6: return launch<64, 64, 32, 32, 32, 2, 4, TA, TB>(g, s);
    case 8: return launch<128, 128, 16, 64, 64, 2, 4, TA, TB>(g, s);
    default:
      set_error("gemm_ex: this tile configuration has no transposed-operand variant");
      return GEMM_STATUS_UNSUPPORTED;
  }
}

template <bool TA, bool TB>
gemm_status f32mfma_run_trans(const GemmArgs &g, int which, hipStream_t s) {
  if (which == 0) return launch_f32mfma<256, 256, 16, 128, 64, 8, TA, TB>(g, s);
  return launch_f32mfma<128, 128, 16, 64, 64, 4, TA, TB>(g, s);
}

}  // namespace bx3
}  // namespace mm
