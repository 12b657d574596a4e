// k_f64.hip -- binary64 GEMM on the FP64 matrix cores (gfx950).
//
// C <- alpha*A*B + beta*C in binary64 with v_mfma_f64_16x16x4f64 (every
// product and sum rounded in binary64).  The structure follows the paper's MM
// transformation chain (Sec. 6.2) the same way the binary32 kernels do:
//   MapTiling       BM x BN workgroup tile, waves of WM x WN, each a grid of
//                   16 x 16 MFMA blocks; K in 16-deep slabs.
//   LocalStorage /  A slab as [BM][16] and B slab transposed as [BN][16]
//   DoubleBuffering binary64 in LDS (128-byte rows, XOR-swizzled 16-byte
//                   chunks), two stages; slab t+1 is loaded while slab t is
//                   multiplied.
//   Vectorization   128-bit loads of A rows, 128-bit LDS writes and reads.
//   ReducePeeling   alpha/beta applied once in the epilogue.
// A batch of equally shaped problems at fixed element strides (the
// batched-strided product of the paper's quantum-transport case study,
// Sec. 6.4) runs the same tiles with the batch index in the grid's second
// dimension.
//
// MFMA operand layout (16x16x4, measured on gfx950): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator element e of lane l
// is D[l / 16 + 4 e][l % 16].  Here lane group g = l / 16 owns k = 4g..4g+3
// of each slab and MFMA step q multiplies k = 4g + q, so each lane's k values
// are contiguous (two 16-byte LDS reads per 16 x 16 block and slab) and every
// k of the slab enters exactly once.
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace mm {
namespace f64 {

typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int BK = 16;       // k per slab
constexpr int CH = BK / 2;   // 16-byte chunks (two binary64) per LDS row
constexpr int kBufferFlags = 0x00020000;

// 128-byte rows: 16 consecutive rows at one logical chunk occupy 16 distinct
// 16-byte bank groups.
__device__ __forceinline__ int swz(int r) { return (r ^ (r >> 3)) & 7; }

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const double *p, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double *>(p), (short)0,
                                           bytes > 0 ? (int)bytes : 0, kBufferFlags);
}

__device__ __forceinline__ double ld1(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

__device__ __forceinline__ f64x2 ld2(__amdgpu_buffer_rsrc_t r, int voff) {
  return __builtin_bit_cast(f64x2, __builtin_amdgcn_raw_buffer_load_b128(r, voff, 0, 0));
}

template <int BM, int BN, int WM, int WN>
struct Cfg {
  static constexpr int NW = (BM / WM) * (BN / WN);
  static constexpr int NT = 64 * NW;
  static constexpr int WAVES_N = BN / WN;
  static constexpr int FM = WM / 16, FN = WN / 16;   // 16 x 16 blocks per wave
  static constexpr int A_ITEMS = BM * CH / NT;        // 16-byte items per lane
  static constexpr int B_ITEMS = BN * CH / NT;
  static_assert(A_ITEMS * NT == BM * CH && B_ITEMS * NT == BN * CH, "even split");
  // a wave's 64 lanes cover 64 consecutive B columns at one chunk index, so
  // the chunk's k-row offset is wave-uniform (a scalar offset)
  static_assert(BN % 64 == 0, "B chunk index must be wave-uniform");
  static constexpr int MIN_WG = NW >= 8 ? 1 : 2;   // workgroups per CU to plan registers for
  static constexpr int STAGE = (BM + BN) * BK;        // binary64 elements per stage
};

// One output tile of one problem.  VEC: lda even, K even and A 16-byte
// aligned (128-bit loads of A rows).  The launcher guarantees that the byte
// extents of an A row panel (BM rows) and of a B slab (16 rows) stay below
// 2^31.
template <int BM, int BN, int WM, int WN, bool VEC, bool BETA>
__device__ __forceinline__ void tile(int M, int N, int K, double alpha, const double *__restrict__ A,
                                     int64_t lda, const double *__restrict__ B, int64_t ldb,
                                     double beta, double *__restrict__ C, int64_t ldc, int m0,
                                     int n0, double *lds) {
  using G = Cfg<BM, BN, WM, WN>;
  constexpr int NT = G::NT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int Mr = M - m0, Nr = N - n0;
  const bool interior = Mr >= BM && Nr >= BN;
  const int rowsA = Mr < BM ? Mr : BM;
  const int colsB = Nr < BN ? Nr : BN;
  // A row panel: valid bytes end with the last valid row's K elements
  const __amdgpu_buffer_rsrc_t rA = rsrc(A + (int64_t)m0 * lda, ((int64_t)(rowsA - 1) * lda + K) * 8);
  int a_off[G::A_ITEMS];
#pragma unroll
  for (int i = 0; i < G::A_ITEMS; ++i) {
    const int idx = tid + NT * i;
    a_off[i] = ((idx / CH) * (int)lda + (idx % CH) * 2) * 8;
  }
  // B: this lane's column (out-of-range columns get an offset past any slab)
  // and the item's first k row (wave-uniform)
  int b_col[G::B_ITEMS], b_row[G::B_ITEMS];
  const int ldb8 = (int)ldb * 8;
#pragma unroll
  for (int i = 0; i < G::B_ITEMS; ++i) {
    const int idx = tid + NT * i;
    const int n = idx % BN;
    b_col[i] = n < colsB ? n * 8 : (int)0x80000000;
    b_row[i] = __builtin_amdgcn_readfirstlane(2 * (idx / BN)) * ldb8;
  }

  double ra[G::A_ITEMS][2], rb[G::B_ITEMS][2];
  // FAST: the slab lies inside [0, K); otherwise k outside [0, K) read as 0.
  auto gload = [&](auto F, int k0) {
    constexpr bool FAST = decltype(F)::value;
#pragma unroll
    for (int i = 0; i < G::A_ITEMS; ++i) {
      if (FAST) {
        const int off = a_off[i] + k0 * 8;
        if (VEC) {
          const f64x2 v = ld2(rA, off);
          ra[i][0] = v.x;
          ra[i][1] = v.y;
        } else {
          ra[i][0] = ld1(rA, off, 0);
          ra[i][1] = ld1(rA, off + 8, 0);
        }
      } else {
        const int k = k0 + ((tid + NT * i) % CH) * 2;
#pragma unroll
        for (int e = 0; e < 2; ++e)
          ra[i][e] = ld1(rA, (k + e >= 0 && k + e < K) ? a_off[i] + (k0 + e) * 8 : (int)0x80000000, 0);
      }
    }
    if (FAST) {
      const __amdgpu_buffer_rsrc_t rB = rsrc(B + (int64_t)k0 * ldb + n0, ((int64_t)(BK - 1) * ldb + colsB) * 8);
#pragma unroll
      for (int i = 0; i < G::B_ITEMS; ++i)
#pragma unroll
        for (int e = 0; e < 2; ++e) rb[i][e] = ld1(rB, b_col[i], b_row[i] + e * ldb8);
    } else {
#pragma unroll
      for (int i = 0; i < G::B_ITEMS; ++i) {
        const int idx = tid + NT * i;
        const int c = __builtin_amdgcn_readfirstlane(idx / BN);
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int k = k0 + 2 * c + e;
          const bool kin = k >= 0 && k < K;
          const __amdgpu_buffer_rsrc_t r = rsrc(B + (int64_t)(kin ? k : 0) * ldb + n0, kin ? colsB * 8 : 0);
          rb[i][e] = ld1(r, (idx % BN) * 8, 0);
        }
      }
    }
  };
  auto sstore = [&](int stage) {
    double *sA = lds + stage * G::STAGE;
    double *sB = sA + BM * BK;
#pragma unroll
    for (int i = 0; i < G::A_ITEMS; ++i) {
      const int idx = tid + NT * i;
      const int r = idx / CH, c = idx % CH;
      *reinterpret_cast<f64x2 *>(sA + r * BK + ((c ^ swz(r)) << 1)) = f64x2{ra[i][0], ra[i][1]};
    }
#pragma unroll
    for (int i = 0; i < G::B_ITEMS; ++i) {
      const int idx = tid + NT * i;
      const int n = idx % BN, c = idx / BN;
      *reinterpret_cast<f64x2 *>(sB + n * BK + ((c ^ swz(n)) << 1)) = f64x2{rb[i][0], rb[i][1]};
    }
  };

  const int wm0 = (wave / G::WAVES_N) * WM, wn0 = (wave % G::WAVES_N) * WN;
  const int lr = lane & 15, lg = lane >> 4;
  f64x4 acc[G::FM][G::FN];
#pragma unroll
  for (int i = 0; i < G::FM; ++i)
#pragma unroll
    for (int j = 0; j < G::FN; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};

  // One slab: per half h, each lane reads its chunk 2 lg + h (k = 4 lg + 2 h,
  // +1) of every block and runs MFMA steps q = 2 h and 2 h + 1.
  auto mfma_stage = [&](int stage) {
    const double *sA = lds + stage * G::STAGE;
    const double *sB = sA + BM * BK;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      f64x2 a[G::FM], b[G::FN];
#pragma unroll
      for (int j = 0; j < G::FN; ++j) {
        const int n = wn0 + 16 * j + lr;
        b[j] = *reinterpret_cast<const f64x2 *>(sB + n * BK + (((2 * lg + h) ^ swz(n)) << 1));
      }
#pragma unroll
      for (int i = 0; i < G::FM; ++i) {
        const int r = wm0 + 16 * i + lr;
        a[i] = *reinterpret_cast<const f64x2 *>(sA + r * BK + (((2 * lg + h) ^ swz(r)) << 1));
      }
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int i = 0; i < G::FM; ++i)
#pragma unroll
          for (int j = 0; j < G::FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i][q], b[j][q], acc[i][j], 0, 0, 0);
    }
  };

  // The slab grid ends exactly at K: slab s covers [kbase + 16 s, +16) with
  // kbase = K - KT*16 <= 0, so only slab 0 can be partial (loaded masked in
  // the prologue).  Loads past the last slab are clamped to it (in bounds,
  // never consumed), so both halves of the loop issue the same instructions.
  using Fast = std::true_type;
  using Masked = std::false_type;
  const int KT = (K + BK - 1) / BK;
  const int kbase = K - KT * BK;
  auto kslab = [&](int s) { return kbase + (s < KT ? s : KT - 1) * BK; };
  gload(Masked{}, kbase);
  sstore(0);
  __syncthreads();
  int t = 0;
  for (; t + 2 <= KT; t += 2) {
    gload(Fast{}, kslab(t + 1));
    __builtin_amdgcn_sched_barrier(0);
    mfma_stage(0);
    sstore(1);
    __syncthreads();
    gload(Fast{}, kslab(t + 2));
    __builtin_amdgcn_sched_barrier(0);
    mfma_stage(1);
    sstore(0);
    __syncthreads();
  }
  if (t < KT) mfma_stage(0);

  // Epilogue: element e of lane l is row lg + 4 e, column lr of its block.
#pragma unroll
  for (int i = 0; i < G::FM; ++i)
#pragma unroll
    for (int j = 0; j < G::FN; ++j) {
      const int col = wn0 + 16 * j + lr;
      if (!interior && col >= Nr) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = wm0 + 16 * i + lg + 4 * e;
        if (interior || row < Mr) {
          double *p = C + (int64_t)(m0 + row) * ldc + (n0 + col);
          const double v = alpha * acc[i][j][e];
          *p = BETA ? fma(beta, *p, v) : v;
        }
      }
    }
}

// Grid: x = output tiles of one problem (XCD-aware order), y = problem of the
// batch (element strides sa, sb, sc between consecutive problems).
template <int BM, int BN, int WM, int WN, bool VEC, bool BETA>
__global__ __launch_bounds__((Cfg<BM, BN, WM, WN>::NT), (Cfg<BM, BN, WM, WN>::MIN_WG)) void gemm_f64_kernel(
    int M, int N, int K, double alpha, const double *__restrict__ A, int64_t lda, int64_t sa,
    const double *__restrict__ B, int64_t ldb, int64_t sb, double beta, double *__restrict__ C,
    int64_t ldc, int64_t sc, int tiles_m, int tiles_n) {
  using G = Cfg<BM, BN, WM, WN>;
  __shared__ __attribute__((aligned(16))) double lds[2 * G::STAGE];
  const int wg = xcd_remap(blockIdx.x, gridDim.x);
  int tm, tn;
  tile_coords(wg, tiles_m, tiles_n, 8, tm, tn);
  const int64_t b = blockIdx.y;
  tile<BM, BN, WM, WN, VEC, BETA>(M, N, K, alpha, A + b * sa, lda, B + b * sb, ldb, beta, C + b * sc,
                                  ldc, tm * BM, tn * BN, lds);
}

template <int BM, int BN, int WM, int WN>
gemm_status launch(const GemmArgsF64 &g, hipStream_t s) {
  using G = Cfg<BM, BN, WM, WN>;
  const int tiles_m = (int)((g.M + BM - 1) / BM);
  const int tiles_n = (int)((g.N + BN - 1) / BN);
  const int64_t nwg = (int64_t)tiles_m * tiles_n;
  if (nwg > 0x7fffffff || g.batch > 65535) {
    set_error("gemm_f64: too many tiles or problems for one launch");
    return GEMM_STATUS_UNSUPPORTED;
  }
  if (((int64_t)BM * g.lda + g.K) * 8 >= ((int64_t)1 << 31) ||
      ((int64_t)BK * g.ldb + g.N) * 8 >= ((int64_t)1 << 31)) {
    set_error("gemm_f64: lda or ldb too large for 32-bit tile offsets");
    return GEMM_STATUS_UNSUPPORTED;
  }
  // 128-bit loads need every problem's A to be 16-byte aligned
  const bool vec = g.lda % 2 == 0 && g.K % 2 == 0 && g.sa % 2 == 0 && ((uintptr_t)g.A & 15) == 0;
  const bool beta = g.beta != 0.0;
  const dim3 grid((unsigned)nwg, (unsigned)g.batch), block(G::NT);
#define MM_LAUNCH(V, BT)                                                                        \
  hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, WM, WN, V, BT>), grid, block, 0, s, (int)g.M,      \
                     (int)g.N, (int)g.K, g.alpha, g.A, g.lda, g.sa, g.B, g.ldb, g.sb, g.beta, g.C, \
                     g.ldc, g.sc, tiles_m, tiles_n)
  if (vec) { if (beta) MM_LAUNCH(true, true); else MM_LAUNCH(true, false); }
  else     { if (beta) MM_LAUNCH(false, true); else MM_LAUNCH(false, false); }
#undef MM_LAUNCH
  return check_launch("gemm_f64_kernel");
}

// Batched small problems (M, N <= 16 SB): one wave per problem, four
// problems per workgroup, operands loaded from memory straight into MFMA
// fragments (each element is used by one wave only, so staging through LDS
// would only add traffic).  The k range is walked in chunks of 16: lane group
// g takes four k of every block (two 128-bit loads of an A row when the
// chunk lies inside [0, K) and lda is even, else four 64-bit loads) and the
// four B values of its column at those k (64-bit loads, consecutive lanes on
// consecutive columns); MFMA step q multiplies the group's q-th k.
// Rows past M and columns past N read zero through the buffer range check;
// k past K is masked per element.
template <int SB, bool VEC, bool BETA>
__global__ __launch_bounds__(256, 2) void small_batched_kernel(
    int M, int N, int K, double alpha, const double *__restrict__ A, int64_t lda, int64_t sa,
    const double *__restrict__ B, int64_t ldb, int64_t sb, double beta, double *__restrict__ C,
    int64_t ldc, int64_t sc, int64_t batch) {
  const int lane = threadIdx.x & 63;
  // the wave index is uniform across the wave; saying so keeps the problem's
  // buffer resources in scalar registers (no per-lane resource loops)
  const int64_t prob = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (prob >= batch) return;
  const int lr = lane & 15, lg = lane >> 4;
  const __amdgpu_buffer_rsrc_t rA = rsrc(A + prob * sa, ((int64_t)(M - 1) * lda + K) * 8);
  const __amdgpu_buffer_rsrc_t rB = rsrc(B + prob * sb, ((int64_t)(K - 1) * ldb + N) * 8);
  double *Cp = C + prob * sc;
  // column offsets of this lane's B blocks; columns past N read zero
  int bcol[SB];
#pragma unroll
  for (int j = 0; j < SB; ++j) {
    const int n = 16 * j + lr;
    bcol[j] = n < N ? n * 8 : (int)0x80000000;
  }
  int arow[SB];
#pragma unroll
  for (int i = 0; i < SB; ++i) {
    const int r = 16 * i + lr;
    arow[i] = r < M ? r * (int)lda * 8 : (int)0x80000000;
  }
  f64x4 acc[SB][SB];
#pragma unroll
  for (int i = 0; i < SB; ++i)
#pragma unroll
    for (int j = 0; j < SB; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < K; k0 += 16) {
    // lane group g takes k = k0 + 2g, +1 (q = 0, 1) and k0 + 8 + 2g, +1
    // (q = 2, 3): one 128-bit load of the four groups reads 64 contiguous
    // bytes of each A row
    auto kq = [&](int q) { return k0 + 2 * lg + (q & 1) + 8 * (q >> 1); };
    double a[SB][4], b[SB][4];
    if (k0 + 16 <= K) {
#pragma unroll
      for (int i = 0; i < SB; ++i) {
        if (VEC) {
          const f64x2 v0 = ld2(rA, arow[i] + kq(0) * 8), v1 = ld2(rA, arow[i] + kq(2) * 8);
          a[i][0] = v0.x; a[i][1] = v0.y; a[i][2] = v1.x; a[i][3] = v1.y;
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) a[i][q] = ld1(rA, arow[i] + kq(q) * 8, 0);
        }
      }
#pragma unroll
      for (int j = 0; j < SB; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) b[j][q] = ld1(rB, bcol[j] + kq(q) * (int)ldb * 8, 0);
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const bool kin = kq(q) < K;
#pragma unroll
        for (int i = 0; i < SB; ++i) a[i][q] = ld1(rA, kin ? arow[i] + kq(q) * 8 : (int)0x80000000, 0);
#pragma unroll
        for (int j = 0; j < SB; ++j)
          b[j][q] = ld1(rB, kin ? bcol[j] + kq(q) * (int)ldb * 8 : (int)0x80000000, 0);
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int i = 0; i < SB; ++i)
#pragma unroll
        for (int j = 0; j < SB; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i][q], b[j][q], acc[i][j], 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < SB; ++i)
#pragma unroll
    for (int j = 0; j < SB; ++j) {
      const int col = 16 * j + lr;
      if (col >= N) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = 16 * i + lg + 4 * e;
        if (row < M) {
          double *p = Cp + (int64_t)row * ldc + col;
          const double v = alpha * acc[i][j][e];
          // non-temporal store (a cache hint): 32^3 x 29 297 134.2 -> 131.0
          // us, 48^3 x 12 000 135.1 -> 125.9 us at beta = 0
          __builtin_nontemporal_store(BETA ? fma(beta, *p, v) : v, p);
        }
      }
    }
}

template <int SB>
gemm_status launch_small(const GemmArgsF64 &g, hipStream_t s) {
  if (((int64_t)(16 * SB) * g.lda + g.K) * 8 >= ((int64_t)1 << 31) ||
      ((int64_t)g.K * g.ldb + g.N) * 8 >= ((int64_t)1 << 31)) {
    set_error("gemm_f64: lda or ldb too large for 32-bit offsets of the small-problem kernel");
    return GEMM_STATUS_UNSUPPORTED;
  }
  const bool vec = g.lda % 2 == 0 && g.sa % 2 == 0 && ((uintptr_t)g.A & 15) == 0;
  const bool beta = g.beta != 0.0;
  const int64_t nwg = (g.batch + 3) / 4;
  if (nwg > 0x7fffffff) { set_error("gemm_f64: batch too large"); return GEMM_STATUS_UNSUPPORTED; }
#define MM_LAUNCH(V, BT)                                                                            \
  hipLaunchKernelGGL((small_batched_kernel<SB, V, BT>), dim3((unsigned)nwg), dim3(256), 0, s,       \
                     (int)g.M, (int)g.N, (int)g.K, g.alpha, g.A, g.lda, g.sa, g.B, g.ldb, g.sb,     \
                     g.beta, g.C, g.ldc, g.sc, g.batch)
  if (vec) { if (beta) MM_LAUNCH(true, true); else MM_LAUNCH(true, false); }
  else     { if (beta) MM_LAUNCH(false, true); else MM_LAUNCH(false, false); }
#undef MM_LAUNCH
  return check_launch("small_batched_kernel");
}

// C <- beta*C over a batch (alpha == 0 or K == 0).
template <bool BETA>
__global__ __launch_bounds__(256) void scale_kernel(int64_t M, int64_t N, double beta,
                                                    double *__restrict__ C, int64_t ldc,
                                                    int64_t sc) {
  double *Cb = C + (int64_t)blockIdx.y * sc;
  const int64_t total = M * N;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / N, j = e - i * N;
    double *p = Cb + i * ldc + j;
    *p = BETA ? beta * *p : 0.0;
  }
}

}  // namespace f64

struct F64Config {
  TileConfig t;
};
static const F64Config kF64Configs[] = {
    {{128, 128, 16, "f64_128x128x16_4w64x64"}},
    {{256, 128, 16, "f64_256x128x16_8w64x64"}},
    {{64, 64, 16, "f64_64x64x16_4w32x32"}},
    // one wave per problem, operands straight into MFMA fragments (M, N <= 16 / 32 / 64)
    {{16, 16, 16, "f64_small_16"}},
    {{32, 32, 16, "f64_small_32"}},
    {{64, 64, 16, "f64_small_64"}},
};

int f64_num_configs() { return (int)(sizeof(kF64Configs) / sizeof(kF64Configs[0])); }
const TileConfig &f64_config(int i) { return kF64Configs[i].t; }

int f64_default_config(int64_t M, int64_t N, int64_t K, int64_t batch) {
  (void)K;
  // batches of small problems: one wave per problem
  if (batch > 1 && M <= 64 && N <= 64) return M <= 16 && N <= 16 ? 3 : (M <= 32 && N <= 32 ? 4 : 5);
  // 128 x 128 tiles once there are two per CU; 64 x 64 below that.  Measured
  // on one box: the kernel is matrix-core bound and the tiles tie within 1 %
  // at 4096^3, but 64 x 64 tiles read 10x the minimum HBM bytes there (5.3
  // against 1.9 GB per launch), which costs clock under the power limit; at
  // 2048^3 (one 128 x 128 tile per CU) 64 x 64 tiles are 11 % faster.
  const int64_t t = ((M + 127) / 128) * ((N + 127) / 128);
  const int64_t need = (2 * (int64_t)num_cus() + t - 1) / (t > 0 ? t : 1);  // problems needed
  return batch >= need ? 0 : 2;
}

gemm_status f64_run(const GemmArgsF64 &g, int cfg, hipStream_t s) {
  switch (cfg) {
    case 0: return f64::launch<128, 128, 64, 64>(g, s);
    case 1: return f64::launch<256, 128, 64, 64>(g, s);
    case 2: return f64::launch<64, 64, 32, 32>(g, s);
    case 3:
    case 4:
    case 5: {
      const int lim = cfg == 3 ? 16 : cfg == 4 ? 32 : 64;
      if (g.M > lim || g.N > lim) {
        set_error("gemm_f64: problem larger than the small-problem configuration");
        return GEMM_STATUS_UNSUPPORTED;
      }
      return cfg == 3 ? f64::launch_small<1>(g, s)
                      : cfg == 4 ? f64::launch_small<2>(g, s) : f64::launch_small<4>(g, s);
    }
    default: set_error("gemm_f64: bad tile config"); return GEMM_STATUS_UNSUPPORTED;
  }
}

gemm_status scale_c_f64(int64_t M, int64_t N, double beta, double *C, int64_t ldc, int64_t sc,
                        int64_t batch, hipStream_t s) {
  const int64_t want = (M * N + 255) / 256;
  const unsigned gx = (unsigned)(want < 4096 ? (want > 0 ? want : 1) : 4096);
  const dim3 grid(gx, (unsigned)batch);
  if (beta != 0.0)
    hipLaunchKernelGGL(f64::scale_kernel<true>, grid, dim3(256), 0, s, M, N, beta, C, ldc, sc);
  else
    hipLaunchKernelGGL(f64::scale_kernel<false>, grid, dim3(256), 0, s, M, N, beta, C, ldc, sc);
  return check_launch("scale_kernel_f64");
}

}  // namespace mm
