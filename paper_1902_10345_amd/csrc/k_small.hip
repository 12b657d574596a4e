// k_small.hip -- products too small to fill the machine with output tiles.
//
// One BM x BN output tile per workgroup of KW waves.  The tile's k range is
// cut into KW consecutive chunks of whole k-steps, one per wave: every wave
// accumulates the whole tile over its own chunk on the matrix cores, with its
// MFMA fragments loaded straight from global memory into registers (no LDS
// staging: a wave touches each element it loads once).  The KW partial tiles
// are then summed in wave order through LDS and the epilogue applies alpha
// and beta.  This is the k-reduction of the matrix product split into
// independent partial reductions whose write conflict on C is resolved by a
// sum (Sec. 3.3, write-conflict resolution; App. A, the wcr attribute), here
// an ordered sum inside the workgroup: deterministic for a given shape and
// configuration, no workspace, one launch.
//
// Three arithmetic modes share the kernel:
//   NP == 1  binary32 products on v_mfma_f32_32x32x2f32 (the plain path);
//   NP == 2  the split-precision path, 3 bf16 products (a0b0 + a0b1 + a1b0);
//   NP == 3  the split-precision path, 6 bf16 products.
// TA / TB: A stored K x M / B stored N x K (op(A) = A^T, op(B) = B^T).
#include "bf16x3.hpp"
#include "common.hpp"
#include "kernels.hpp"

namespace mm {
namespace small {

using bx3::bf16x2;
using bx3::f32x2;
using bx3::kBufferFlags;

constexpr int KW = 8;  // waves per workgroup (k chunks per output tile)

// Per lane and k-step: E consecutive k of one row of op(A) and of one column
// of op(B) per 32 x 32 block (k-step 8 in binary32: lanes 0-31 hold k 0..3,
// lanes 32-63 k 4..7; k-step 16 in bf16: 8 k per half-wave).
template <int NP>
struct Mode {
  static constexpr int KSTEP = NP == 1 ? 8 : 16;
  static constexpr int E = NP == 1 ? 4 : 8;
};

// Loads the lane's E values of one row (A) or column (B) of the operand at
// k = k0 .. k0 + E - 1.  idx: the row of op(A) / column of op(B); valid: idx
// inside the matrix.  KC: the operand is stored with k contiguous (row-major
// A, transposed B); then VEC allows 128-bit loads (row stride a multiple of
// 4 floats, 16-byte aligned base, K % 4 == 0).  Elements outside the matrix
// read as zero: their offset is pushed past the resource.
template <int E, bool KC, bool VEC>
__device__ __forceinline__ void load_frag(__amdgpu_buffer_rsrc_t rs, int64_t ld, int idx,
                                          bool valid, int k0, int K, float (&v)[E]) {
  constexpr int kOut = (int)0x80000000;
  if constexpr (KC && VEC) {
#pragma unroll
    for (int q = 0; q < E / 4; ++q) {
      const int k = k0 + 4 * q;
      const int off = (valid && k < K) ? (int)(((unsigned)idx * (unsigned)ld + k) * 4u) : kOut;
      const float4 x =
          __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
      v[4 * q + 0] = x.x; v[4 * q + 1] = x.y; v[4 * q + 2] = x.z; v[4 * q + 3] = x.w;
    }
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int k = k0 + e;
      const unsigned el = KC ? (unsigned)idx * (unsigned)ld + k : (unsigned)k * (unsigned)ld + idx;
      const int off = (valid && k < K) ? (int)(el * 4u) : kOut;
      v[e] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0));
    }
  }
}

template <int BM, int BN, int NP, bool TA, bool TB, bool VA, bool VB, bool BETA>
__global__ __launch_bounds__(64 * KW) void gemm_small_kernel(
    int M, int N, int K, float alpha, const float *__restrict__ A, int64_t lda, int bytes_a,
    const float *__restrict__ B, int64_t ldb, int bytes_b, float beta, float *__restrict__ C,
    int64_t ldc, int tiles_n, int steps_per_wave) {
  constexpr int FM = BM / 32, FN = BN / 32;
  constexpr int KSTEP = Mode<NP>::KSTEP, E = Mode<NP>::E;
  constexpr int BLK = 16 * 64;  // floats of one 32 x 32 accumulator block
  __shared__ float red[KW * FM * FN * BLK];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int lr = lane & 31, lg = lane >> 5;
  const int m0 = (blockIdx.x / tiles_n) * BM, n0 = (blockIdx.x % tiles_n) * BN;
  const __amdgpu_buffer_rsrc_t ra =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(A), (short)0, bytes_a, kBufferFlags);
  const __amdgpu_buffer_rsrc_t rb =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(B), (short)0, bytes_b, kBufferFlags);

  f32x16 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;

  const int ks_total = (K + KSTEP - 1) / KSTEP;
  const int ks0 = w * steps_per_wave;
  const int ks1 = ks0 + steps_per_wave < ks_total ? ks0 + steps_per_wave : ks_total;

  float fa[2][FM][E], fb[2][FN][E];
  auto load = [&](int set, int ks) {
    const int k0 = ks * KSTEP + lg * E;
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      const int m = m0 + i * 32 + lr;
      load_frag<E, !TA, VA>(ra, lda, m, m < M, k0, K, fa[set][i]);
    }
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int n = n0 + j * 32 + lr;
      load_frag<E, TB, VB>(rb, ldb, n, n < N, k0, K, fb[set][j]);
    }
  };
  auto mfma = [&](int set) {
    if constexpr (NP == 1) {
      // MFMA q sums k = q of the lower half-wave's four and of the upper
      // half-wave's four: every k of the step exactly once
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[set][i][q], fb[set][j][q],
                                                             acc[i][j], 0, 0, 0);
    } else {
      bf16x8 a[NP][FM], b[NP][FN];
      // split of E = 8 binary32 values into NP bf16 planes, two at a time
      auto split8 = [&](const float (&x)[E], bf16x8 &p0, bf16x8 &p1, bf16x8 &p2) {
#pragma unroll
        for (int e = 0; e < 8; e += 2) {
          bf16x2 x0, x1, x2;
          if constexpr (NP == 2) bx3::split2(f32x2{x[e], x[e + 1]}, x0, x1);
          else bx3::split3(f32x2{x[e], x[e + 1]}, x0, x1, x2);
          p0[e] = x0.x; p0[e + 1] = x0.y;
          p1[e] = x1.x; p1[e + 1] = x1.y;
          if constexpr (NP == 3) { p2[e] = x2.x; p2[e + 1] = x2.y; }
        }
      };
#pragma unroll
      for (int i = 0; i < FM; ++i) split8(fa[set][i], a[0][i], a[1][i], a[NP - 1][i]);
#pragma unroll
      for (int j = 0; j < FN; ++j) split8(fb[set][j], b[0][j], b[1][j], b[NP - 1][j]);
      auto prod = [&](int qa, int qb) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[qa][i], b[qb][j], acc[i][j],
                                                                0, 0, 0);
      };
      // small products first, the leading product last
      if constexpr (NP == 3) {
        prod(2, 0);
        prod(1, 1);
        prod(0, 2);
      }
      prod(1, 0);
      prod(0, 1);
      prod(0, 0);
    }
  };

  // two register sets: the loads of step ks+1 are in flight while step ks
  // is multiplied
  if (ks0 < ks1) {
    load(0, ks0);
    int ks = ks0;
    for (; ks + 2 <= ks1; ks += 2) {
      load(1, ks + 1);
      mfma(0);
      if (ks + 2 < ks1) load(0, ks + 2);
      mfma(1);
    }
    if (ks < ks1) mfma(0);
  }

  // partial tiles to LDS (lane-contiguous: no bank conflicts), then the
  // ordered sum over the waves and the epilogue
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) red[((w * FM + i) * FN + j) * BLK + e * 64 + lane] = acc[i][j][e];
  __syncthreads();
  constexpr int TOT = FM * FN * BLK;
  for (int idx = tid; idx < TOT; idx += 64 * KW) {
    float s = red[idx];
#pragma unroll
    for (int v = 1; v < KW; ++v) s += red[v * TOT + idx];
    const int l = idx & 63, e = (idx >> 6) & 15, blk = idx >> 10;
    const int row = m0 + (blk / FN) * 32 + 8 * (e >> 2) + 4 * (l >> 5) + (e & 3);
    const int col = n0 + (blk % FN) * 32 + (l & 31);
    if (row < M && col < N) {
      float *p = C + (int64_t)row * ldc + col;
      const float v = alpha * s;
      *p = BETA ? fmaf(beta, *p, v) : v;
    }
  }
}

// Byte extent of a stored operand (rows x row stride, the last row cut at
// cols); the kernel addresses it with 32-bit offsets from its base.
static inline int64_t extent_bytes(int64_t rows, int64_t ld, int64_t cols) {
  return rows <= 0 || cols <= 0 ? 0 : ((rows - 1) * ld + cols) * 4;
}

template <int BM, int BN, int NP>
gemm_status launch(const GemmArgs &g, hipStream_t s) {
  const int64_t tiles_m = (g.M + BM - 1) / BM, tiles_n = (g.N + BN - 1) / BN;
  const int64_t ea = g.ta ? extent_bytes(g.K, g.lda, g.M) : extent_bytes(g.M, g.lda, g.K);
  const int64_t eb = g.tb ? extent_bytes(g.N, g.ldb, g.K) : extent_bytes(g.K, g.ldb, g.N);
  // every element offset (and the out-of-range marker) must fit in 31 bits
  if (tiles_m * tiles_n > 0x7fffffff || ea >= ((int64_t)1 << 31) || eb >= ((int64_t)1 << 31)) {
    set_error("small-product configuration: operands too large for 32-bit offsets");
    return GEMM_STATUS_UNSUPPORTED;
  }
  const int ks_total = (int)((g.K + Mode<NP>::KSTEP - 1) / Mode<NP>::KSTEP);
  const int spw = (ks_total + KW - 1) / KW;
  const bool va = !g.ta && g.lda % 4 == 0 && g.K % 4 == 0 && ((uintptr_t)g.A & 15) == 0;
  const bool vb = g.tb && g.ldb % 4 == 0 && g.K % 4 == 0 && ((uintptr_t)g.B & 15) == 0;
  const bool beta = g.beta != 0.0f;
  const dim3 grid((unsigned)(tiles_m * tiles_n)), block(64 * KW);
#define MM_SMALL(TA, TB, VA, VB, BT)                                                           \
  hipLaunchKernelGGL((gemm_small_kernel<BM, BN, NP, TA, TB, VA, VB, BT>), grid, block, 0, s,   \
                     (int)g.M, (int)g.N, (int)g.K, g.alpha, g.A, g.lda, (int)ea, g.B, g.ldb,    \
                     (int)eb, g.beta, g.C, g.ldc, (int)tiles_n, spw)
#define MM_SMALL_BETA(TA, TB, VA, VB) \
  do { if (beta) MM_SMALL(TA, TB, VA, VB, true); else MM_SMALL(TA, TB, VA, VB, false); } while (0)
  if (!g.ta && !g.tb) {
    if (va) MM_SMALL_BETA(false, false, true, false);
    else MM_SMALL_BETA(false, false, false, false);
  } else if (!g.ta && g.tb) {
    if (va && vb) MM_SMALL_BETA(false, true, true, true);
    else MM_SMALL_BETA(false, true, false, false);
  } else if (g.ta && !g.tb) {
    MM_SMALL_BETA(true, false, false, false);
  } else {
    if (vb) MM_SMALL_BETA(true, true, false, true);
    else MM_SMALL_BETA(true, true, false, false);
  }
#undef MM_SMALL_BETA
#undef MM_SMALL
  return check_launch("gemm_small_kernel");
}

}  // namespace small

// which: 0 = 32 x 32 tiles, 1 = 64 x 64 tiles; np: 1 (binary32), 2 or 3
// (bf16 planes per operand).
gemm_status small_run(const GemmArgs &g, int which, int np, hipStream_t s) {
  if (np == 1) return which == 0 ? small::launch<32, 32, 1>(g, s) : small::launch<64, 64, 1>(g, s);
  if (np == 2) return which == 0 ? small::launch<32, 32, 2>(g, s) : small::launch<64, 64, 2>(g, s);
  return which == 0 ? small::launch<32, 32, 3>(g, s) : small::launch<64, 64, 3>(g, s);
}

}  // namespace mm
