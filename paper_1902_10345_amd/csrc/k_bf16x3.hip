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

// Batched-strided products on the matrix-core tiles.  The tile follows the
// problem's size and the batch's total tile count: 64 x 64 tiles for small
// problems (128 x 128 for six products and for binary32), otherwise the
// single-GEMM choice for a problem stacked batch times along M.
int batched_config(int path, int n_products, int64_t M, int64_t N, int64_t K, int64_t batch) {
  if (path == GEMM_PATH_F32) {
    const int64_t tiles = ((M + 255) / 256) * ((N + 255) / 256);
    if (tiles <= 0) return 1;
    return batch >= (num_cus() + tiles - 1) / tiles ? 0 : 1;  // f32mfma 256 x 256 / 128 x 128
  }
  if (M <= 64 && N <= 64) return n_products == 6 ? 5 : 6;
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
  if (path == GEMM_PATH_F32)
    return cfg == 0 ? bx3::launch_batched<256, 256, 16, 128, 64, 1, 8>(g, sa, sb, sc, batch, s)
                    : bx3::launch_batched<128, 128, 16, 64, 64, 1, 4>(g, sa, sb, sc, batch, s);
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
