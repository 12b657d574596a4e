// k_f32.hip -- plain FP32 GEMM on the gfx950 vector ALU.
//
// C <- alpha*A*B + beta*C, row-major, binary32 FMA accumulation.
//
// Mapping of the paper's matrix-multiplication transformation chain (Sec. 6.2;
// transformation table of App. B) onto CDNA4:
//   MapTiling (cache level)      -> BM x BN output tile per 256-lane workgroup,
//                                   sequential K loop over BK-deep slabs
//   MapTiling (register level)   -> RM x RN register micro-tile per lane
//   LocalStorage (pack A/B)      -> A and B slabs staged in LDS
//   DoubleBuffering              -> two LDS stages; global loads of slab t+1
//                                   are in flight while slab t is consumed
//   Vectorization                -> 128-bit global loads/stores, ds_read_b128
//   LocalStorage (C tile)        -> accumulators stay in VGPRs for the whole K loop
//   MapReduceFusion              -> the k-reduction is fused into the FMA chain
//   ReducePeeling                -> alpha/beta applied once, in the epilogue
#include "common.hpp"
#include "kernels.hpp"

namespace mm {
namespace f32 {

// Word 3 of a raw buffer resource (32-bit data format, no swizzle).
constexpr int kBufferFlags = 0x00020000;

// Guarded load of the four consecutive elements (r, c..c+3) of a row-major
// matrix with R rows and Cc columns; out-of-range elements read as zero.
template <bool VEC>
__device__ __forceinline__ float4 load4(const float *__restrict__ base, int64_t ld,
                                        int r, int c, int R, int Cc) {
  float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
  if (r < R) {
    const float *p = base + (int64_t)r * ld + c;
    if (VEC && c + 3 < Cc) {
      v = *reinterpret_cast<const float4 *>(p);
    } else {
      if (c + 0 < Cc) v.x = p[0];
      if (c + 1 < Cc) v.y = p[1];
      if (c + 2 < Cc) v.z = p[2];
      if (c + 3 < Cc) v.w = p[3];
    }
  }
  return v;
}

// BM x BN tile, BK-deep slabs, RM x RN micro-tile per lane, 256 lanes.
// Lane (tx, ty): rows ty + TY*r (r < RM), columns h*(BN/NH) + tx*4 + c.
template <int BM, int BN, int BK, int RM, int RN, int U, bool VEC, bool BETA>
__global__ __launch_bounds__(256, 2) void gemm_f32_kernel(
    int M, int N, int K, float alpha, const float *__restrict__ A, int64_t lda,
    const float *__restrict__ B, int64_t ldb, float beta, float *__restrict__ C,
    int64_t ldc, int tiles_m, int tiles_n) {
  constexpr int NT = 256;
  constexpr int TX = BN / RN;            // lanes along N
  constexpr int TY = BM / RM;            // lanes along M
  static_assert(TX * TY == NT, "256 lanes");
  constexpr int NH = RN / 4;             // float4 column groups per lane
  constexpr int HS = BN / NH;            // stride between column groups
  constexpr int SA = BK + 4;             // padded LDS row stride of A (floats)
  constexpr int SB = BN + 4;             // padded LDS row stride of B (floats)
  constexpr int A_ST = BM * SA;
  constexpr int B_ST = BK * SB;
  constexpr int LA = BM * BK / 4 / NT;   // float4 loads of A per lane per slab
  constexpr int LB = BK * BN / 4 / NT;   // float4 loads of B per lane per slab
  static_assert(LA * NT * 4 == BM * BK && LB * NT * 4 == BK * BN, "even split");

  __shared__ __attribute__((aligned(16))) float lds[2 * (A_ST + B_ST)];

  const int tid = threadIdx.x;
  const int wg = xcd_remap(blockIdx.x, gridDim.x);
  int tm, tn;
  tile_coords(wg, tiles_m, tiles_n, 8, tm, tn);
  const int m0 = tm * BM, n0 = tn * BN;
  const int Mr = M - m0, Nr = N - n0;
  const float *Ab = A + (int64_t)m0 * lda;
  const float *Bb = B + n0;

  float4 ra[LA], rb[LB];
  // Interior slabs use raw buffer loads: an SGPR resource per operand (the
  // B resource is rebased to the slab's first row) and fixed 32-bit lane
  // offsets, so no 64-bit address arithmetic runs per load.  Edge slabs take
  // the guarded path.  The launcher guarantees 32-bit byte offsets.
  const bool interior = Mr >= BM && Nr >= BN;
  const __amdgpu_buffer_rsrc_t rsrcA = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float *>(Ab), (short)0, interior ? (int)(((int64_t)(BM - 1) * lda + K) * 4) : 0,
      kBufferFlags);
  int a_voff[LA], b_voff[LB];
#pragma unroll
  for (int i = 0; i < LA; ++i) {
    const int idx = tid + NT * i;
    a_voff[i] = ((idx / (BK / 4)) * (int)lda + (idx % (BK / 4)) * 4) * 4;
  }
#pragma unroll
  for (int i = 0; i < LB; ++i) {
    const int idx = tid + NT * i;
    b_voff[i] = ((idx / (BN / 4)) * (int)ldb + (idx % (BN / 4)) * 4) * 4;
  }
  auto gload = [&](int k0) {
    if (VEC && interior && k0 + BK <= K) {
      const __amdgpu_buffer_rsrc_t rsrcB = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<float *>(Bb + (int64_t)k0 * ldb), (short)0,
          (int)(((int64_t)(BK - 1) * ldb + BN) * 4), kBufferFlags);
#pragma unroll
      for (int i = 0; i < LA; ++i)
        ra[i] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rsrcA, a_voff[i] + k0 * 4, 0, 0));
#pragma unroll
      for (int i = 0; i < LB; ++i)
        rb[i] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rsrcB, b_voff[i], 0, 0));
      return;
    }
#pragma unroll
    for (int i = 0; i < LA; ++i) {
      const int idx = tid + NT * i;
      ra[i] = load4<VEC>(Ab, lda, idx / (BK / 4), k0 + (idx % (BK / 4)) * 4, Mr, K);
    }
#pragma unroll
    for (int i = 0; i < LB; ++i) {
      const int idx = tid + NT * i;
      rb[i] = load4<VEC>(Bb + (int64_t)k0 * ldb, ldb, idx / (BN / 4), (idx % (BN / 4)) * 4,
                         K - k0, Nr);
    }
  };
  auto sstore = [&](int s) {
    float *As = lds + s * (A_ST + B_ST);
    float *Bs = As + A_ST;
#pragma unroll
    for (int i = 0; i < LA; ++i) {
      const int idx = tid + NT * i;
      *reinterpret_cast<float4 *>(&As[(idx / (BK / 4)) * SA + (idx % (BK / 4)) * 4]) = ra[i];
    }
#pragma unroll
    for (int i = 0; i < LB; ++i) {
      const int idx = tid + NT * i;
      *reinterpret_cast<float4 *>(&Bs[(idx / (BN / 4)) * SB + (idx % (BN / 4)) * 4]) = rb[i];
    }
  };

  const int tx = tid % TX, ty = tid / TX;
  float acc[RM][RN];
#pragma unroll
  for (int r = 0; r < RM; ++r)
#pragma unroll
    for (int c = 0; c < RN; ++c) acc[r][c] = 0.f;

  auto compute = [&](int s) {
    const float *As = lds + s * (A_ST + B_ST);
    const float *Bs = As + A_ST;
    // Unrolled U times (1 or 2): a full unroll lets the scheduler hoist every
    // slab read and spill; two steps let the next step's LDS reads overlap
    // the current step's FMAs.  One 4-deep step issues RM*RN*4 independent FMAs.
#pragma unroll U
    for (int kk = 0; kk < BK; kk += 4) {
      float4 a[RM];
      float4 b[4][NH];
#pragma unroll
      for (int r = 0; r < RM; ++r)
        a[r] = *reinterpret_cast<const float4 *>(&As[(ty + TY * r) * SA + kk]);
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int h = 0; h < NH; ++h)
          b[q][h] = *reinterpret_cast<const float4 *>(&Bs[(kk + q) * SB + h * HS + tx * 4]);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int r = 0; r < RM; ++r) {
          const float av = q == 0 ? a[r].x : q == 1 ? a[r].y : q == 2 ? a[r].z : a[r].w;
#pragma unroll
          for (int h = 0; h < NH; ++h) {
            acc[r][h * 4 + 0] = fmaf(av, b[q][h].x, acc[r][h * 4 + 0]);
            acc[r][h * 4 + 1] = fmaf(av, b[q][h].y, acc[r][h * 4 + 1]);
            acc[r][h * 4 + 2] = fmaf(av, b[q][h].z, acc[r][h * 4 + 2]);
            acc[r][h * 4 + 3] = fmaf(av, b[q][h].w, acc[r][h * 4 + 3]);
          }
        }
      }
    }
  };

  const int KT = (K + BK - 1) / BK;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int t = 0; t < KT; ++t) {
    if (t + 1 < KT) gload((t + 1) * BK);
    compute(t & 1);
    if (t + 1 < KT) sstore((t + 1) & 1);
    __syncthreads();
  }

  // Peeled epilogue: C = alpha*acc + beta*C (C not read when beta == 0).
#pragma unroll
  for (int r = 0; r < RM; ++r) {
    const int row = ty + TY * r;
    if (row >= Mr) continue;
    float *Crow = C + (int64_t)(m0 + row) * ldc + n0;
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      const int col = h * HS + tx * 4;
      float v0 = alpha * acc[r][h * 4 + 0], v1 = alpha * acc[r][h * 4 + 1];
      float v2 = alpha * acc[r][h * 4 + 2], v3 = alpha * acc[r][h * 4 + 3];
      if (VEC && col + 3 < Nr) {
        float4 *p = reinterpret_cast<float4 *>(Crow + col);
        if (BETA) {
          const float4 o = *p;
          v0 = fmaf(beta, o.x, v0); v1 = fmaf(beta, o.y, v1);
          v2 = fmaf(beta, o.z, v2); v3 = fmaf(beta, o.w, v3);
        }
        *p = make_float4(v0, v1, v2, v3);
      } else {
        const float v[4] = {v0, v1, v2, v3};
#pragma unroll
        for (int c = 0; c < 4; ++c)
          if (col + c < Nr) Crow[col + c] = BETA ? fmaf(beta, Crow[col + c], v[c]) : v[c];
      }
    }
  }
}

template <int BM, int BN, int BK, int RM, int RN, int U>
gemm_status launch(const GemmArgs &g, hipStream_t s) {
  const int tiles_m = (int)((g.M + BM - 1) / BM);
  const int tiles_n = (int)((g.N + BN - 1) / BN);
  const int64_t nwg = (int64_t)tiles_m * tiles_n;
  if (nwg > 0x7fffffff) { set_error("gemm_f32: too many tiles"); return GEMM_STATUS_UNSUPPORTED; }
  if (((int64_t)BM * g.lda + g.K) * 4 >= ((int64_t)1 << 31) ||
      ((int64_t)BK * g.ldb + BN) * 4 >= ((int64_t)1 << 31)) {
    set_error("gemm_f32: leading dimension too large for 32-bit tile offsets");
    return GEMM_STATUS_UNSUPPORTED;
  }
  const bool vec = g.lda % 4 == 0 && g.ldb % 4 == 0 && g.ldc % 4 == 0 &&
                   ((uintptr_t)g.A & 15) == 0 && ((uintptr_t)g.B & 15) == 0 &&
                   ((uintptr_t)g.C & 15) == 0;
  const bool beta = g.beta != 0.0f;
  dim3 grid((unsigned)nwg), block(256);
#define MM_LAUNCH(V, BT)                                                                     \
  hipLaunchKernelGGL((gemm_f32_kernel<BM, BN, BK, RM, RN, U, V, BT>), grid, block, 0, s,     \
                     (int)g.M, (int)g.N, (int)g.K, g.alpha, g.A, g.lda, g.B, g.ldb, g.beta, \
                     g.C, g.ldc, tiles_m, tiles_n)
  if (vec) { if (beta) MM_LAUNCH(true, true); else MM_LAUNCH(true, false); }
  else     { if (beta) MM_LAUNCH(false, true); else MM_LAUNCH(false, false); }
#undef MM_LAUNCH
  return check_launch("gemm_f32_kernel");
}

}  // namespace f32

// Tile configurations of the FP32 path (index = config id).
static const TileConfig kF32Configs[] = {
    {128, 128, 32, "f32_128x128x32_r8x8"},
    {64, 64, 32, "f32_64x64x32_r4x4"},
    {128, 64, 32, "f32_128x64x32_r8x4"},
    {128, 128, 32, "f32_128x128x32_r8x8_u2"},
    {128, 64, 32, "f32_128x64x32_r8x4_u2"},
    // binary32 products on the FP32 matrix cores (same arithmetic; the tile
    // body of the split-precision path in its FP32 mode)
    {256, 256, 16, "f32mfma_256x256x16_8w128x64"},
    {128, 128, 16, "f32mfma_128x128x16_4w64x64"},
    // small products: one tile per workgroup of 8 waves, its k range split
    // over the waves (binary32 matrix cores, ordered sum through LDS)
    {32, 32, 8, "f32_small_32x32_8wk"},
    {64, 64, 8, "f32_small_64x64_8wk"},
    // the FP32 matrix-core 128 x 128 tile with its k range split between two
    // groups of four waves (partial tiles summed through LDS in group order)
    {128, 128, 16, "f32mfma_128x128x16_2x4w64x64_kg2"},
};

int f32_num_configs() { return (int)(sizeof(kF32Configs) / sizeof(kF32Configs[0])); }
const TileConfig &f32_config(int i) { return kF32Configs[i]; }

int f32_default_config(int64_t M, int64_t N, int64_t K) {
  // measured: the FP32 matrix-core tiles win while they fill every CU (256 x
  // 256: 140 TFLOP/s at 4096^3 against 90 on the vector ALU).  Below that the
  // small-product tiles (the k range split over a workgroup's eight waves)
  // win on every shape swept, 1.7-4.3x over the 64 x 64 vector-ALU tile
  // (256^3: 4.1 against 17.5 us; graph-replayed launches): 64 x 64 tiles
  // once they fill the CUs, 32 x 32 tiles before.
  const int64_t cus = num_cus();
  auto tiles = [&](int64_t b) { return ((M + b - 1) / b) * ((N + b - 1) / b); };
  if (tiles(256) >= cus) return 5;
  // 128 x 128 tiles for more than three quarters of the CUs and at most all
  // of them: the matrix-core tile with its k range split between two groups
  // of four waves (2048^3 166.8 -> 151.6 us, 1792^3 126.6 against 147.9 for
  // the small-product tiles); fewer tiles: the small-product tiles
  const int64_t t128 = tiles(128);
  if (t128 <= cus && 4 * t128 > 3 * cus && K % 2 == 0) return 9;
  if (t128 >= cus) return 6;
  return tiles(64) >= cus ? 8 : 7;
}

gemm_status f32_run(const GemmArgs &g, int cfg, hipStream_t s) {
  if ((g.ta || g.tb) && cfg != 5 && cfg != 6 && cfg != 7 && cfg != 8) {
    set_error("gemm_ex: only the FP32 matrix-core and small-product tiles take transposed operands");
    return GEMM_STATUS_UNSUPPORTED;
  }
  switch (cfg) {
    case 0: return f32::launch<128, 128, 32, 8, 8, 1>(g, s);
    case 1: return f32::launch<64, 64, 32, 4, 4, 1>(g, s);
    case 2: return f32::launch<128, 64, 32, 8, 4, 1>(g, s);
    case 3: return f32::launch<128, 128, 32, 8, 8, 2>(g, s);
    case 4: return f32::launch<128, 64, 32, 8, 4, 2>(g, s);
    case 5: return f32mfma_run(g, 0, s);
    case 6: return f32mfma_run(g, 1, s);
    case 7: return small_run(g, 0, 1, s);
    case 8: return small_run(g, 1, 1, s);
    case 9: return f32mfma_run(g, 2, s);
    default: set_error("gemm_f32: bad tile config"); return GEMM_STATUS_UNSUPPORTED;
  }
}

}  // namespace mm
