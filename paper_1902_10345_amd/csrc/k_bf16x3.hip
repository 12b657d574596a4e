// k_bf16x3.hip -- FP32-accurate split-precision GEMM on bf16 MFMA (gfx950).
#include <algorithm>

#include "bx3_launch.hpp"

namespace mm {
namespace bx3 {

// ---- split-K ----------------------------------------------------------------
// Workgroup (chunk c, output tile) multiplies K range [c*chunk, min(K, (c+1)*chunk))
// of its tile (alpha 1, beta 0) into partial plane c of P (M x N, ld N).
// Chunks are whole slabs, so the slab grid of every chunk ends on its own
// boundary and only a chunk's first slab can be partial.
template <int BM, int BN, int BK, int WM, int WN, int NP, int NW, bool VEC>
__global__ __launch_bounds__(64 * NW, 1) void gemm_bx3_splitk_kernel(
    int M, int N, int K, int chunk, const float *__restrict__ A, int64_t lda,
    const float *__restrict__ B, int64_t ldb, float *__restrict__ P, int tiles_m, int tiles_n) {
  using G = Cfg<BM, BN, BK, WM, WN, NP, NW>;
  __shared__ __attribute__((aligned(16))) __bf16 lds[G::LDS_BYTES / 2];
  const int wg = xcd_remap(blockIdx.x, gridDim.x);
  const int tiles = tiles_m * tiles_n;
  const int c = wg / tiles;
  int tm, tn;
  tile_coords(wg - c * tiles, tiles_m, tiles_n, 8, tm, tn);
  const int k0 = c * chunk;
  const int kc = (K - k0 < chunk ? K - k0 : chunk);
  tile<BM, BN, BK, WM, WN, NP, NW, VEC, false>(M, N, kc, 1.0f, A + k0, lda, B + (int64_t)k0 * ldb,
                                               ldb, 0.0f, P + (int64_t)c * M * N, N, tm * BM,
                                               tn * BN, lds);
}

// The write-conflict resolution of the chunks: C = alpha * (P_0 + P_1 + ...)
// + beta * C, summed in chunk order (deterministic), the same epilogue
// arithmetic as the single-pass kernel.  VEC: N, ldc multiples of 4 and C
// 16-byte aligned.
template <bool VEC, bool BETA>
__global__ __launch_bounds__(256) void splitk_reduce_kernel(int M, int N, int S,
                                                            const float *__restrict__ P,
                                                            float alpha, float beta,
                                                            float *__restrict__ C, int64_t ldc) {
  const int64_t plane = (int64_t)M * N;
  if (VEC) {
    const int64_t n4 = plane / 4;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n4; q += (int64_t)gridDim.x * 256) {
      float4 acc = reinterpret_cast<const float4 *>(P)[q];
      for (int c = 1; c < S; ++c) {
        const float4 v = reinterpret_cast<const float4 *>(P + c * plane)[q];
        acc.x += v.x; acc.y += v.y; acc.z += v.z; acc.w += v.w;
      }
      const int64_t e = 4 * q;
      const int64_t i = e / N, j = e - i * N;
      float4 *cp = reinterpret_cast<float4 *>(C + i * ldc + j);
      float4 out = make_float4(alpha * acc.x, alpha * acc.y, alpha * acc.z, alpha * acc.w);
      if (BETA) {
        const float4 c0 = *cp;
        out = make_float4(fmaf(beta, c0.x, out.x), fmaf(beta, c0.y, out.y),
                          fmaf(beta, c0.z, out.z), fmaf(beta, c0.w, out.w));
      }
      *cp = out;
    }
  } else {
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < plane; e += (int64_t)gridDim.x * 256) {
      float acc = P[e];
      for (int c = 1; c < S; ++c) acc += P[c * plane + e];
      const int64_t i = e / N, j = e - i * N;
      float *cp = C + i * ldc + j;
      const float v = alpha * acc;
      *cp = BETA ? fmaf(beta, *cp, v) : v;
    }
  }
}

template <int BM, int BN, int BK, int WM, int WN, int NP, int NW>
gemm_status launch_splitk(const GemmArgs &g, int S, float *P, hipStream_t s) {
  const int tiles_m = (int)((g.M + BM - 1) / BM);
  const int tiles_n = (int)((g.N + BN - 1) / BN);
  const int64_t nwg = (int64_t)tiles_m * tiles_n * S;
  if (nwg > 0x7fffffff) { set_error("gemm_f32_3xbf16_splitk: too many workgroups"); return GEMM_STATUS_UNSUPPORTED; }
  if (((int64_t)BM * g.lda + g.K) * 4 >= (int64_t)1 << 31 ||
      ((int64_t)BK * g.ldb + g.N) * 4 >= ((int64_t)1 << 31)) {
    set_error("gemm_f32_3xbf16_splitk: lda or ldb too large for 32-bit tile offsets");
    return GEMM_STATUS_UNSUPPORTED;
  }
  const int chunk = (int)(((g.K + S - 1) / S + BK - 1) / BK * BK);
  S = (int)((g.K + chunk - 1) / chunk);  // chunks that hold work (<= requested)
  const int64_t nwg_used = (int64_t)tiles_m * tiles_n * S;
  const bool vec = g.lda % 4 == 0 && g.K % 4 == 0 && ((uintptr_t)g.A & 15) == 0;
  if (vec)
    hipLaunchKernelGGL((gemm_bx3_splitk_kernel<BM, BN, BK, WM, WN, NP, NW, true>), dim3((unsigned)nwg_used),
                       dim3(64 * NW), 0, s, (int)g.M, (int)g.N, (int)g.K, chunk, g.A, g.lda, g.B,
                       g.ldb, P, tiles_m, tiles_n);
  else
    hipLaunchKernelGGL((gemm_bx3_splitk_kernel<BM, BN, BK, WM, WN, NP, NW, false>), dim3((unsigned)nwg_used),
                       dim3(64 * NW), 0, s, (int)g.M, (int)g.N, (int)g.K, chunk, g.A, g.lda, g.B,
                       g.ldb, P, tiles_m, tiles_n);
  if (gemm_status st = check_launch("gemm_bx3_splitk_kernel")) return st;
  const bool rvec = g.N % 4 == 0 && g.ldc % 4 == 0 && ((uintptr_t)g.C & 15) == 0;
  const int64_t items = rvec ? g.M * g.N / 4 : g.M * g.N;
  const unsigned grid = (unsigned)std::min<int64_t>((items + 255) / 256, 4096);
#define MM_RED(V, BT)                                                                              \
  hipLaunchKernelGGL((splitk_reduce_kernel<V, BT>), dim3(grid), dim3(256), 0, s, (int)g.M,        \
                     (int)g.N, S, P, g.alpha, g.beta, g.C, g.ldc)
  if (rvec) { if (g.beta != 0.0f) MM_RED(true, true); else MM_RED(true, false); }
  else      { if (g.beta != 0.0f) MM_RED(false, true); else MM_RED(false, false); }
#undef MM_RED
  return check_launch("splitk_reduce_kernel");
}

// Split kernel used to verify the staging split bit for bit.
__global__ __launch_bounds__(256) void split_kernel(int64_t n, const float *__restrict__ x,
                                                    unsigned short *__restrict__ p0,
                                                    unsigned short *__restrict__ p1,
                                                    unsigned short *__restrict__ p2) {
  // pairs (x[2q], x[2q+1]) through the same pair split the tile body uses
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; 2 * q < n; q += (int64_t)gridDim.x * 256) {
    const int64_t i = 2 * q;
    const bool two = i + 1 < n;
    bf16x2 h, m, l;
    split3(f32x2{x[i], two ? x[i + 1] : 0.0f}, h, m, l);
    // bit-cast whole pairs (a bit_cast of a vector element is not
    // element-indexed in this compiler) and take the halves
    const unsigned hb = __builtin_bit_cast(unsigned, h), mb = __builtin_bit_cast(unsigned, m),
                   lb = __builtin_bit_cast(unsigned, l);
    p0[i] = (unsigned short)(hb & 0xffffu);
    p1[i] = (unsigned short)(mb & 0xffffu);
    if (p2) p2[i] = (unsigned short)(lb & 0xffffu);
    if (two) {
      p0[i + 1] = (unsigned short)(hb >> 16);
      p1[i + 1] = (unsigned short)(mb >> 16);
      if (p2) p2[i + 1] = (unsigned short)(lb >> 16);
    }
  }
}

// ---- batched small problems --------------------------------------------------
// M, N <= 32 SB: one wave per problem, four problems per workgroup.  The
// operands go from memory straight into MFMA fragments (and are split in
// registers, NP = 2 or 3 planes; NP = 1 is binary32 on the FP32 matrix
// cores): every element is used by one wave only, so staging through LDS
// would add traffic and barriers, and the 64 x 64 tile of four waves would
// leave three of them on padding for a 32 x 32 problem.  A lane holds 8 k of
// its A row (two 128-bit loads) and of its B column (eight loads, consecutive
// lanes on consecutive columns) per 16-deep k-step: 8 consecutive k on the
// split path, two runs of 4 in binary32 (the FP32 tile's fragment order).
// The k-steps lie on the grid that ends at K (only the first can be partial)
// and the products come in the tile kernels' order, so every element is the
// same sum as in the LDS-staged tile of the same arithmetic.
// C stores with the non-temporal cache policy (the slc bit, NT on gfx950; a
// hint only): 32^3 x 29 297 at beta = 0 63.2 -> 55.4 us, 48^3 x 12 000 63.6
// -> 53.9 us.  The same hint on the operand loads was slower.
constexpr int kStoreNT = 2;

template <int SB, int NP, bool VEC, bool BETA>
__global__ __launch_bounds__(256) void small_batched_bx3_kernel(
    int M, int N, int K, float alpha, const float *__restrict__ A, int64_t lda, int64_t sa,
    const float *__restrict__ B, int64_t ldb, int64_t sb, float beta, float *__restrict__ C,
    int64_t ldc, int64_t sc, int batch) {
  const int lane = threadIdx.x & 63;
  // the wave index is uniform across the wave; saying so keeps the problem's
  // buffer resources in scalar registers
  const int prob = (int)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  if (prob >= batch) return;
  const int lr = lane & 31, lg = lane >> 5;
  // rows past M and columns past N read zero through the range check (their
  // results are never stored); k below 0 is masked per element
  const __amdgpu_buffer_rsrc_t rA = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float *>(A + (int64_t)prob * sa), (short)0,
      (int)(((int64_t)(M - 1) * lda + K) * 4), kBufferFlags);
  const __amdgpu_buffer_rsrc_t rB = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float *>(B + (int64_t)prob * sb), (short)0,
      (int)(((int64_t)(K - 1) * ldb + N) * 4), kBufferFlags);
  const __amdgpu_buffer_rsrc_t rC = __builtin_amdgcn_make_buffer_rsrc(
      C + (int64_t)prob * sc, (short)0, (int)(((int64_t)(M - 1) * ldc + N) * 4), kBufferFlags);
  int arow[SB], bcol[SB];
#pragma unroll
  for (int i = 0; i < SB; ++i) {
    const int r = 32 * i + lr;
    arow[i] = r < M ? r * (int)lda * 4 : (int)0x80000000;
  }
#pragma unroll
  for (int j = 0; j < SB; ++j) {
    const int n = 32 * j + lr;
    bcol[j] = n < N ? n * 4 : (int)0x80000000;
  }
  const int ldb4 = (int)ldb * 4;
  f32x16 acc[SB][SB];
#pragma unroll
  for (int i = 0; i < SB; ++i)
#pragma unroll
    for (int j = 0; j < SB; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;
  auto ld = [](__amdgpu_buffer_rsrc_t r, int off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
  };
  // the 8 values of one block as NP bf16 planes (plane 0 the leading part)
  constexpr int NPL = NP > 1 ? NP : 2;
  auto split8 = [](const float (&x)[8], bf16x8 (&pl)[NPL]) {
#pragma unroll
    for (int e = 0; e < 8; e += 2) {
      bf16x2 x0, x1, x2;
      if constexpr (NP == 2) split2(f32x2{x[e], x[e + 1]}, x0, x1);
      else split3(f32x2{x[e], x[e + 1]}, x0, x1, x2);
      pl[0][e] = x0.x; pl[0][e + 1] = x0.y;
      pl[1][e] = x1.x; pl[1][e + 1] = x1.y;
      if constexpr (NP == 3) { pl[2][e] = x2.x; pl[2][e + 1] = x2.y; }
    }
  };
  const int KT = (K + 15) / 16;
  const int kbase = K - KT * 16;
  for (int s = 0; s < KT; ++s) {
    if constexpr (NP == 1) {
      // binary32 on v_mfma_f32_32x32x2f32, as in the FP32 tile: lane group g
      // holds k = 4g + q and 8 + 4g + q (q < 4) of the step, and MFMA
      // 4h + q takes element 4h + q of both groups
      const int kb = kbase + 16 * s + 4 * lg;
      float a[SB][8], b[SB][8];
      if (s > 0 || kbase == 0) {
#pragma unroll
        for (int i = 0; i < SB; ++i) {
          if (VEC) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const f32x4 v = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(
                                                            rA, arow[i] + (kb + 8 * h) * 4, 0, 0));
              a[i][4 * h] = v.x; a[i][4 * h + 1] = v.y;
              a[i][4 * h + 2] = v.z; a[i][4 * h + 3] = v.w;
            }
          } else {
#pragma unroll
            for (int e = 0; e < 8; ++e)
              a[i][e] = ld(rA, arow[i] + (kb + 8 * (e >> 2) + (e & 3)) * 4);
          }
        }
#pragma unroll
        for (int j = 0; j < SB; ++j)
#pragma unroll
          for (int e = 0; e < 8; ++e)
            b[j][e] = ld(rB, bcol[j] + (kb + 8 * (e >> 2) + (e & 3)) * ldb4);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int k = kb + 8 * (e >> 2) + (e & 3);
#pragma unroll
          for (int i = 0; i < SB; ++i)
            a[i][e] = ld(rA, k >= 0 ? arow[i] + k * 4 : (int)0x80000000);
#pragma unroll
          for (int j = 0; j < SB; ++j)
            b[j][e] = ld(rB, k >= 0 ? bcol[j] + k * ldb4 : (int)0x80000000);
        }
      }
#pragma unroll
      for (int e = 0; e < 8; ++e)
#pragma unroll
        for (int i = 0; i < SB; ++i)
#pragma unroll
          for (int j = 0; j < SB; ++j)
            acc[i][j] =
                __builtin_amdgcn_mfma_f32_32x32x2f32(a[i][e], b[j][e], acc[i][j], 0, 0, 0);
      continue;
    }
    const int k0 = kbase + 16 * s + 8 * lg;  // the lane's first k of this step
    float a[SB][8], b[SB][8];
    if (s > 0 || kbase == 0) {
#pragma unroll
      for (int i = 0; i < SB; ++i) {
        if (VEC) {
          const f32x4 v0 = __builtin_bit_cast(
              f32x4, __builtin_amdgcn_raw_buffer_load_b128(rA, arow[i] + k0 * 4, 0, 0));
          const f32x4 v1 = __builtin_bit_cast(
              f32x4, __builtin_amdgcn_raw_buffer_load_b128(rA, arow[i] + k0 * 4 + 16, 0, 0));
          a[i][0] = v0.x; a[i][1] = v0.y; a[i][2] = v0.z; a[i][3] = v0.w;
          a[i][4] = v1.x; a[i][5] = v1.y; a[i][6] = v1.z; a[i][7] = v1.w;
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e) a[i][e] = ld(rA, arow[i] + (k0 + e) * 4);
        }
      }
#pragma unroll
      for (int j = 0; j < SB; ++j)
#pragma unroll
        for (int e = 0; e < 8; ++e) b[j][e] = ld(rB, bcol[j] + (k0 + e) * ldb4);
    } else {
      // the partial first step: k in [kbase, kbase + 16) with kbase < 0
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const bool kin = k0 + e >= 0;
#pragma unroll
        for (int i = 0; i < SB; ++i)
          a[i][e] = ld(rA, kin ? arow[i] + (k0 + e) * 4 : (int)0x80000000);
#pragma unroll
        for (int j = 0; j < SB; ++j)
          b[j][e] = ld(rB, kin ? bcol[j] + (k0 + e) * ldb4 : (int)0x80000000);
      }
    }
    bf16x8 pa[SB][NPL], pb[SB][NPL];
#pragma unroll
    for (int i = 0; i < SB; ++i) split8(a[i], pa[i]);
#pragma unroll
    for (int j = 0; j < SB; ++j) split8(b[j], pb[j]);
    auto prod = [&](int qa, int qb) {
#pragma unroll
      for (int i = 0; i < SB; ++i)
#pragma unroll
        for (int j = 0; j < SB; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(pa[i][qa], pb[j][qb], acc[i][j],
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
  // 32 x 32 block layout: lane l, element e -> row 8*(e/4) + 4*(l/32) + e%4,
  // column l%32.  Columns past N get an out-of-range offset; rows past M fall
  // beyond the resource and their stores are dropped.  With beta != 0 every
  // read of C is issued before the first store.
  const int ldc4 = (int)ldc * 4;
  int vb[SB][SB];
  float cold[SB][SB][16];
#pragma unroll
  for (int i = 0; i < SB; ++i)
#pragma unroll
    for (int j = 0; j < SB; ++j) {
      const int col = 32 * j + lr;
      vb[i][j] = col < N ? (32 * i + 4 * lg) * ldc4 + col * 4 : (int)0x80000000;
      if (BETA) {
#pragma unroll
        for (int e = 0; e < 16; ++e)
          cold[i][j][e] = __builtin_bit_cast(
              float, __builtin_amdgcn_raw_buffer_load_b32(rC, vb[i][j],
                                                          (8 * (e >> 2) + (e & 3)) * ldc4, 0));
      }
    }
#pragma unroll
  for (int i = 0; i < SB; ++i)
#pragma unroll
    for (int j = 0; j < SB; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        float v = alpha * acc[i][j][e];
        if (BETA) v = fmaf(beta, cold[i][j][e], v);
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), rC, vb[i][j],
                                              (8 * (e >> 2) + (e & 3)) * ldc4, kStoreNT);
      }
}

// Offsets of the small-problem kernel stay below 2^31: 64 rows of A and of C,
// K rows of B.
bool small_batched_fits(const GemmArgs &g) {
  const int64_t lim = (int64_t)1 << 31;
  return ((int64_t)64 * g.lda + g.K) * 4 < lim && ((int64_t)g.K * g.ldb + g.N) * 4 < lim &&
         ((int64_t)64 * g.ldc + g.N) * 4 < lim;
}

// At most 65535 problems per launch (the caller's chunks).
template <int SB, int NP>
gemm_status launch_small_batched(const GemmArgs &g, int64_t sa, int64_t sb, int64_t sc,
                                 int batch, hipStream_t s) {
  // 128-bit A loads: 16-byte aligned rows and k offsets (K % 4 == 0 keeps the
  // step grid on multiples of 4)
  const bool vec = g.lda % 4 == 0 && g.K % 4 == 0 && sa % 4 == 0 && ((uintptr_t)g.A & 15) == 0;
  const bool beta = g.beta != 0.0f;
  const dim3 grid((unsigned)((batch + 3) / 4)), block(256);
#define MM_LAUNCH(V, BT)                                                                         \
  hipLaunchKernelGGL((small_batched_bx3_kernel<SB, NP, V, BT>), grid, block, 0, s, (int)g.M,      \
                     (int)g.N, (int)g.K, g.alpha, g.A, g.lda, sa, g.B, g.ldb, sb, g.beta, g.C,     \
                     g.ldc, sc, batch)
  if (vec) { if (beta) MM_LAUNCH(true, true); else MM_LAUNCH(true, false); }
  else     { if (beta) MM_LAUNCH(false, true); else MM_LAUNCH(false, false); }
#undef MM_LAUNCH
  return check_launch("small_batched_bx3_kernel");
}

}  // namespace bx3

constexpr int kSplitKMax = 64;

// Tile configurations of the split-precision path.  np = planes per operand
// (2 -> 3 products, 3 -> 6 products).
struct Bx3Config {
  TileConfig t;
  int np;
};
static const Bx3Config kBx3Configs[] = {
    {{256, 256, 16, "bx3_256x256x16_8w128x64_p3"}, 2},
    {{128, 128, 32, "bx3_128x128x32_4w64x64_p3"}, 2},
    {{256, 128, 32, "bx3_256x128x32_8w64x64_p3"}, 2},
    {{256, 256, 32, "bx3_256x256x32_8w128x64_p3"}, 2},
    {{256, 256, 16, "bx3_256x256x16_8w128x64_p6"}, 3},
    {{128, 128, 32, "bx3_128x128x32_4w64x64_p6"}, 3},
    {{64, 64, 32, "bx3_64x64x32_4w32x32_p3"}, 2},
    {{256, 256, 16, "bx3_256x256x16_4w128x128_p3"}, 2},
    {{128, 128, 16, "bx3_128x128x16_4w64x64_p3"}, 2},
    // small products: one tile per workgroup of 8 waves, its k range split
    // over the waves (fragments straight from global memory, ordered sum
    // through LDS)
    {{32, 32, 16, "bx3_small_32x32_8wk_p3"}, 2},
    {{64, 64, 16, "bx3_small_64x64_8wk_p3"}, 2},
    {{32, 32, 16, "bx3_small_32x32_8wk_p6"}, 3},
    {{64, 64, 16, "bx3_small_64x64_8wk_p6"}, 3},
    // the 256 x 256 x 16 tile with a ring of three LDS stages: the first
    // product's fragments of the next slab are read before the barrier
    {{256, 256, 16, "bx3_256x256x16_8w128x64_p3_ring3"}, 2},
    // 128 x 128 x 16 tiles, the k range split between two groups of four
    // waves (partial tiles summed through LDS in group order)
    {{128, 128, 16, "bx3_128x128x16_2x4w64x64_p3_kg2"}, 2},
};

int bx3_num_configs() { return (int)(sizeof(kBx3Configs) / sizeof(kBx3Configs[0])); }
const TileConfig &bx3_config(int i) { return kBx3Configs[i].t; }
int bx3_config_products(int i) { return kBx3Configs[i].np == 2 ? 3 : 6; }

int bx3_default_config(int64_t M, int64_t N, int64_t K, int n_products) {
  const int64_t cus = num_cus();
  auto tiles = [&](int bm, int bn) { return ((M + bm - 1) / bm) * ((N + bn - 1) / bn); };
  const int64_t big = tiles(256, 256);
  // Shapes whose 128 x 128 tiles leave CUs idle: the small-product tiles (the
  // k range split over a workgroup's eight waves), measured by graph replay
  // over 19 shapes: 32 x 32 tiles up to two per CU (256^3: 3.7 us against
  // 6.1 for the 64 x 64 LDS tile; 512^3 5.0 against 9.6), 64 x 64 tiles
  // while those stay below two per CU (768^3, 1024^3), the 64 x 64 LDS tile
  // beyond.
  auto small = [&](int p3_32, int p3_64, int lds64) {
    if (tiles(32, 32) <= 2 * cus) return p3_32;
    return tiles(64, 64) < 2 * cus ? p3_64 : lds64;
  };
  if (n_products == 6) {
    if (big >= cus) return 4;
    // six products: the small-product tiles beat the 128 x 128 LDS tile on
    // every underfilled shape swept but one (1536^2 x 512, 3 % behind)
    return tiles(128, 128) >= cus ? 5 : small(11, 12, 12);
  }
  // 256 x 256 x 16: 1.5-2.4 % ahead of the 32-deep slabs at 4096^3,
  // 8192 x 2048 x 4096 and 8192^2 x 4096 (same box, alternating)
  if (big >= cus) return 0;
  // Below that, measured on one box (all configurations, alternating): the
  // 8-wave 256 x 128 tiles win by 7-11 % when they come to about one wave of
  // the machine (4096 x 2048^2, 2560^3, 2048 x 4096^2; with and without
  // beta); 128 x 128 x 16 tiles while they fill every CU (at one tile per CU
  // they win by 6 % with beta == 0, the paper's C = A*B at 2048^3, and lose
  // by 4 % with beta != 0); the small-product tiles below that.
  const int64_t mid = tiles(256, 128);
  if (mid * 4 >= cus * 3 && mid <= cus) return 2;
  // 128 x 128 tiles for more than half of the CUs and at most all of them:
  // the tile with its k range split between two groups of four waves (two
  // waves per SIMD instead of one), measured over eight shapes: 2048^3 64.9
  // -> 57.6 us, 1792^3 62.2 -> 44.5 (the 64 x 64 tile before), 1536^3 42.0 ->
  // 37.6; at half of the CUs and below the 64 x 64 tiles stay ahead
  const int64_t t128 = tiles(128, 128);
  if (t128 <= cus && 2 * t128 > cus && K % 2 == 0) return 14;
  if (t128 >= cus) return 8;
  return small(9, 10, 6);
}

gemm_status bx3_run(const GemmArgs &g, int cfg, hipStream_t s) {
  if (cfg >= 9 && cfg <= 12) return small_run(g, (cfg - 9) & 1, cfg <= 10 ? 2 : 3, s);
  if (g.ta || g.tb) return g.ta ? (g.tb ? bx3_run_tt(g, cfg, s) : bx3_run_tn(g, cfg, s)) : bx3_run_nt(g, cfg, s);
  switch (cfg) {
    case 0: return bx3::launch<256, 256, 16, 128, 64, 2, 8>(g, s);
    case 1: return bx3::launch<128, 128, 32, 64, 64, 2, 4>(g, s);
    case 2: return bx3::launch<256, 128, 32, 64, 64, 2, 8>(g, s);
    case 3: return bx3::launch<256, 256, 32, 128, 64, 2, 8>(g, s);
    case 4: return bx3::launch<256, 256, 16, 128, 64, 3, 8>(g, s);
    case 5: return bx3::launch<128, 128, 32, 64, 64, 3, 4>(g, s);
    case 6: return bx3::launch<64, 64, 32, 32, 32, 2, 4>(g, s);
    case 7: return bx3::launch<256, 256, 16, 128, 128, 2, 4>(g, s);
    case 8: return bx3::launch<128, 128, 16, 64, 64, 2, 4>(g, s);
    case 13: return bx3::launch<256, 256, 16, 128, 64, 2, 8, false, false, 3>(g, s);
    case 14: return bx3::launch_kg<128, 128, 16, 64, 64, 2, 4>(g, s);
    default: set_error("gemm_f32_3xbf16: bad tile config"); return GEMM_STATUS_UNSUPPORTED;
  }
}

// Split-K uses the 128 x 128 tiles (16-deep slabs for three products,
// 32-deep for six); a chunk is at least 256 deep.
int bx3_splitk_default(int64_t M, int64_t N, int64_t K) {
  const int64_t tiles = ((M + 127) / 128) * ((N + 127) / 128);
  int64_t s = (2 * (int64_t)num_cus() + tiles - 1) / tiles;
  const int64_t by_k = K / 256;
  if (s > by_k) s = by_k;
  if (s > kSplitKMax) s = kSplitKMax;
  return (int)(s < 1 ? 1 : s);
}

size_t bx3_splitk_ws_bytes(int64_t M, int64_t N, int splits) {
  return splits <= 1 ? 0 : (((size_t)splits * (size_t)M * (size_t)N * 4 + 255) / 256) * 256;
}

gemm_status bx3_run_splitk(const GemmArgs &g, int n_products, int splits, void *ws, hipStream_t s) {
  float *P = static_cast<float *>(ws);
  if (splits <= 1) return bx3_run(g, n_products == 6 ? 5 : 8, s);  // same tile, one pass
  if (n_products == 6) return bx3::launch_splitk<128, 128, 32, 64, 64, 3, 4>(g, splits, P, s);
  return bx3::launch_splitk<128, 128, 16, 64, 64, 2, 4>(g, splits, P, s);
}

gemm_status f32mfma_run(const GemmArgs &g, int which, hipStream_t s) {
  if (which == 2) {
    if (g.ta || g.tb) {
      set_error("gemm_ex: the two-group FP32 matrix-core tile takes no transposed operands");
      return GEMM_STATUS_UNSUPPORTED;
    }
    return bx3::launch_kg<128, 128, 16, 64, 64, 1, 4>(g, s);
  }
  if (g.ta || g.tb)
    return g.ta ? (g.tb ? f32mfma_run_tt(g, which, s) : f32mfma_run_tn(g, which, s))
                : f32mfma_run_nt(g, which, s);
  if (which == 0) return bx3::launch_f32mfma<256, 256, 16, 128, 64, 8>(g, s);
  return bx3::launch_f32mfma<128, 128, 16, 64, 64, 4>(g, s);
}

// Batched-strided products.  Small problems, one wave per problem
// (small_batched_bx3_kernel): binary32 and six products for M, N <= 64, three
// products while M N <= 48^2 (beyond that the 64 x 64 tile of four waves is
// faster: 64^3 x 8000 71 against 78 us).  Otherwise the tile follows the
// problem's size and the batch's total tile count: the single-GEMM choice for
// a problem stacked batch times along M (binary32: 256 x 256 or 128 x 128
// tiles on the FP32 matrix cores).
int batched_config(int path, int n_products, int64_t M, int64_t N, int64_t K, int64_t batch) {
  if (path == GEMM_PATH_F32) {
    if (M <= 64 && N <= 64) return kBatchedSmall1;
    const int64_t tiles = ((M + 255) / 256) * ((N + 255) / 256);
    if (tiles <= 0) return 1;
    return batch >= (num_cus() + tiles - 1) / tiles ? 0 : 1;  // f32mfma 256 x 256 / 128 x 128
  }
  if (M <= 64 && N <= 64) {
    if (n_products == 6) return kBatchedSmall6;
    return M * N <= 48 * 48 ? kBatchedSmall3 : 6;
  }
  // M stacked batch times (saturated: only the tile count's size matters)
  const int64_t stacked = M <= 0 ? 0 : batch > ((int64_t)1 << 40) / M ? ((int64_t)1 << 40) : M * batch;
  const int cfg = bx3_default_config(stacked, N, K, n_products);
  // the small-product tiles have no batched variant: their LDS-staged
  // counterparts of the same width take the batch
  if (cfg >= 9) return n_products == 6 ? 5 : 6;
  return cfg;
}

gemm_status batched_run(int path, int cfg, const GemmArgs &g, int64_t sa, int64_t sb, int64_t sc,
                        int batch, hipStream_t s) {
  if (path == GEMM_PATH_F32) {
    if (cfg == kBatchedSmall1 && bx3::small_batched_fits(g))
      return g.M <= 32 && g.N <= 32 ? bx3::launch_small_batched<1, 1>(g, sa, sb, sc, batch, s)
                                    : bx3::launch_small_batched<2, 1>(g, sa, sb, sc, batch, s);
    return cfg == 0 ? bx3::launch_batched<256, 256, 16, 128, 64, 1, 8>(g, sa, sb, sc, batch, s)
                    : bx3::launch_batched<128, 128, 16, 64, 64, 1, 4>(g, sa, sb, sc, batch, s);
  }
  if (cfg == kBatchedSmall3 || cfg == kBatchedSmall6) {
    // one wave per problem; offsets beyond 32 bits take the LDS-staged tile
    // of the same product count (the same per-element sums)
    const bool six = cfg == kBatchedSmall6, one = g.M <= 32 && g.N <= 32;
    if (bx3::small_batched_fits(g)) {
      if (six) return one ? bx3::launch_small_batched<1, 3>(g, sa, sb, sc, batch, s)
                          : bx3::launch_small_batched<2, 3>(g, sa, sb, sc, batch, s);
      return one ? bx3::launch_small_batched<1, 2>(g, sa, sb, sc, batch, s)
                 : bx3::launch_small_batched<2, 2>(g, sa, sb, sc, batch, s);
    }
    cfg = six ? 5 : 6;
  }
  switch (cfg) {
    case 0: return bx3::launch_batched<256, 256, 16, 128, 64, 2, 8>(g, sa, sb, sc, batch, s);
    case 2: return bx3::launch_batched<256, 128, 32, 64, 64, 2, 8>(g, sa, sb, sc, batch, s);
    case 3: return bx3::launch_batched<256, 256, 32, 128, 64, 2, 8>(g, sa, sb, sc, batch, s);
    case 4: return bx3::launch_batched<256, 256, 16, 128, 64, 3, 8>(g, sa, sb, sc, batch, s);
    case 5: return bx3::launch_batched<128, 128, 32, 64, 64, 3, 4>(g, sa, sb, sc, batch, s);
    case 6: return bx3::launch_batched<64, 64, 32, 32, 32, 2, 4>(g, sa, sb, sc, batch, s);
    case 8: return bx3::launch_batched<128, 128, 16, 64, 64, 2, 4>(g, sa, sb, sc, batch, s);
    default:
      set_error("gemm_strided_batched: configuration without a batched variant");
      return GEMM_STATUS_UNSUPPORTED;
  }
}

gemm_status bx3_split(int64_t n, const float *x, uint16_t *p0, uint16_t *p1, uint16_t *p2,
                      hipStream_t s) {
  const int64_t want = ((n + 1) / 2 + 255) / 256;
  const unsigned grid = (unsigned)(want < 8192 ? (want > 0 ? want : 1) : 8192);
  hipLaunchKernelGGL(bx3::split_kernel, dim3(grid), dim3(256), 0, s, n, x, p0, p1, p2);
  return check_launch("split_kernel");
}

}  // namespace mm
