// k_bf16x3.hip -- FP32-accurate split-precision GEMM on bf16 MFMA (gfx950).
#include "bf16x3.hpp"

namespace mm {
namespace bx3 {

template <int BM, int BN, int BK, int WM, int WN, int NP, int NW, bool VEC, bool BETA>
__global__ __launch_bounds__(64 * NW, 1) void gemm_bx3_kernel(
    int M, int N, int K, float alpha, const float *__restrict__ A, int64_t lda,
    const float *__restrict__ B, int64_t ldb, float beta, float *__restrict__ C, int64_t ldc,
    int tiles_m, int tiles_n) {
  using G = Cfg<BM, BN, BK, WM, WN, NP, NW>;
  __shared__ __attribute__((aligned(16))) __bf16 lds[G::LDS_BYTES / 2];
  const int wg = xcd_remap(blockIdx.x, gridDim.x);
  int tm, tn;
  tile_coords(wg, tiles_m, tiles_n, 8, tm, tn);
  tile<BM, BN, BK, WM, WN, NP, NW, VEC, BETA>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
                                         tm * BM, tn * BN, lds);
}

template <int BM, int BN, int BK, int WM, int WN, int NP, int NW>
gemm_status launch(const GemmArgs &g, hipStream_t s) {
  const int tiles_m = (int)((g.M + BM - 1) / BM);
  const int tiles_n = (int)((g.N + BN - 1) / BN);
  const int64_t nwg = (int64_t)tiles_m * tiles_n;
  if (nwg > 0x7fffffff) { set_error("gemm_f32_3xbf16: too many tiles"); return GEMM_STATUS_UNSUPPORTED; }
  if (((int64_t)BM * g.lda + g.K) * 4 >= (int64_t)1 << 31 ||
      ((int64_t)BK * g.ldb + g.N) * 4 >= ((int64_t)1 << 31)) {
    set_error("gemm_f32_3xbf16: lda too large for 32-bit tile offsets");
    return GEMM_STATUS_UNSUPPORTED;
  }
  // 128-bit loads of A rows need 16-byte aligned slab starts: the slab grid
  // ends at K, so K must be a multiple of 4 as well as lda.
  const bool vec = g.lda % 4 == 0 && g.K % 4 == 0 && ((uintptr_t)g.A & 15) == 0;
  const bool beta = g.beta != 0.0f;
  dim3 grid((unsigned)nwg), block(64 * NW);
#define MM_LAUNCH(V, BT)                                                                    \
  hipLaunchKernelGGL((gemm_bx3_kernel<BM, BN, BK, WM, WN, NP, NW, V, BT>), grid, block, 0, s, \
                     (int)g.M, (int)g.N, (int)g.K, g.alpha, g.A, g.lda, g.B, g.ldb, g.beta, \
                     g.C, g.ldc, tiles_m, tiles_n)
  if (vec) { if (beta) MM_LAUNCH(true, true); else MM_LAUNCH(true, false); }
  else     { if (beta) MM_LAUNCH(false, true); else MM_LAUNCH(false, false); }
#undef MM_LAUNCH
  return check_launch("gemm_bx3_kernel");
}

// Split kernel used to verify the staging split bit for bit.
__global__ __launch_bounds__(256) void split_kernel(int64_t n, const float *__restrict__ x,
                                                    unsigned short *__restrict__ p0,
                                                    unsigned short *__restrict__ p1,
                                                    unsigned short *__restrict__ p2) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    __bf16 h, m, l;
    split3(x[i], h, m, l);
    p0[i] = __builtin_bit_cast(unsigned short, h);
    p1[i] = __builtin_bit_cast(unsigned short, m);
    if (p2) p2[i] = __builtin_bit_cast(unsigned short, l);
  }
}

}  // namespace bx3

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
};

int bx3_num_configs() { return (int)(sizeof(kBx3Configs) / sizeof(kBx3Configs[0])); }
const TileConfig &bx3_config(int i) { return kBx3Configs[i].t; }
int bx3_config_products(int i) { return kBx3Configs[i].np == 2 ? 3 : 6; }

int bx3_default_config(int64_t M, int64_t N, int64_t K, int n_products) {
  (void)K;
  const int64_t cus = num_cus();
  const int64_t big = ((M + 255) / 256) * ((N + 255) / 256);
  if (n_products == 6) return big >= cus ? 4 : 5;
  if (big >= cus) return 0;
  // measured: once 256 x 256 tiles leave CUs idle, 128 x 128 x 16 tiles win
  // while they still fill every CU, below that 64 x 64 tiles
  const int64_t small = ((M + 127) / 128) * ((N + 127) / 128);
  if (small >= cus) return 8;
  return 6;
}

gemm_status bx3_run(const GemmArgs &g, int cfg, hipStream_t s) {
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
    default: set_error("gemm_f32_3xbf16: bad tile config"); return GEMM_STATUS_UNSUPPORTED;
  }
}

gemm_status bx3_split(int64_t n, const float *x, uint16_t *p0, uint16_t *p1, uint16_t *p2,
                      hipStream_t s) {
  const int64_t want = (n + 255) / 256;
  const unsigned grid = (unsigned)(want < 8192 ? (want > 0 ? want : 1) : 8192);
  hipLaunchKernelGGL(bx3::split_kernel, dim3(grid), dim3(256), 0, s, n, x, p0, p1, p2);
  return check_launch("split_kernel");
}

}  // namespace mm
