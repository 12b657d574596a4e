// k_fp8.hip -- scaled FP8 (OCP E4M3) GEMM on gfx950 matrix cores.
//
//   sa[i] = max_k |A[i,k]| / 448,  sb[j] = max_k |B[k,j]| / 448  (0 -> 1)
//   qa = e4m3(A / sa),  qb = e4m3(B / sb)   (round to nearest even, saturating)
//   C <- alpha * sa[i] * sb[j] * sum_k qa*qb + beta*C   (binary32 accumulation)
//
// Workspace layout (each region 256-byte aligned, Kp = K rounded up to 128):
//   [qa: M x Kp bytes][qbT: N x Kp bytes][sa: M floats][sb: N floats]
//   [amax bits of B's columns: N uint32]
// qbT is B's code matrix transposed (column j contiguous), so both operands are
// k-contiguous and stage into LDS without a transpose.  Codes in [K, Kp) are 0.
#include <algorithm>
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"

namespace mm {
namespace fp8 {

constexpr int KP_ALIGN = 128;
// Word 3 of a raw buffer resource (32-bit data format, no swizzle).
constexpr int kBufferFlags = 0x00020000;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

struct Layout {
  int64_t Kp;
  size_t qa, qb, sa, sb, amax, total;
};

static inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

Layout layout(int64_t M, int64_t N, int64_t K) {
  Layout L;
  L.Kp = ((K + KP_ALIGN - 1) / KP_ALIGN) * KP_ALIGN;
  size_t off = 0;
  L.qa = off; off = align256(off + (size_t)(M * L.Kp));
  L.qb = off; off = align256(off + (size_t)(N * L.Kp));
  L.sa = off; off = align256(off + sizeof(float) * (size_t)M);
  L.sb = off; off = align256(off + sizeof(float) * (size_t)N);
  // column-amax scratch, shared by the column quantisations of both operands
  L.amax = off; off = align256(off + sizeof(uint32_t) * (size_t)(M > N ? M : N));
  L.total = off;
  return L;
}

// Binary32 -> E4M3 code, round to nearest even, saturating at +-448.  NaN ->
// 0x7F.  The sign bit is kept, so negative values that round to zero give 0x80.
// Branch-free: every candidate is computed and the right one selected.
//  - |x| < 2^-6 lies on the subnormal grid 2^-9: the code is |x| * 512 rounded
//    to an integer, ties to even (8 is the smallest normal), done by adding
//    2^23, whose ulp is 1, and taking the low mantissa bits;
//  - otherwise the 23-bit mantissa is rounded to 3 bits, ties to even, a carry
//    moving to the next binade by itself, and the exponent rebiased from 127
//    to 7; codes above 0x7E (|x| beyond 448, infinities) saturate to 0x7E.
__device__ __forceinline__ uint32_t e4m3_encode(float x) {
  const uint32_t u = __builtin_bit_cast(uint32_t, x);
  const uint32_t sign = (u >> 24) & 0x80u;
  const uint32_t a = u & 0x7fffffffu;
  const uint32_t sub =
      __builtin_bit_cast(uint32_t, __builtin_bit_cast(float, a) * 512.0f + 0x1p23f) - 0x4b000000u;
  const uint32_t code = ((a + 0x7ffffu + ((a >> 20) & 1u)) >> 20) - ((127u - 7u) << 3);
  const uint32_t normal = code > 0x7eu ? 0x7eu : code;
  const uint32_t is_sub = 0u - (uint32_t)(a < 0x3c800000u);  // all ones or zero: a
  const uint32_t mag = (sub & is_sub) | (normal & ~is_sub);   // mask, not a branch
  return a > 0x7f800000u ? 0x7fu : (sign | mag);
}

// v / s rounded to nearest, as the IEEE division gives it, from r = 1 / s
// (rounded to nearest): q0 = |v| r is within one ulp of the quotient, the
// remainder |v| - q0 s is exact with one FMA, and the corrected q0 + r * rem
// rounds correctly (Markstein's theorem).  Needs s, r and the remainders that
// decide a code normal, which holds for scales in [2^-60, 2^60] (quotients
// below 2^-12 all encode to a signed zero); other scales use the division.
// Three FMA-class operations instead of the ten of a binary32 division.
__device__ __forceinline__ bool quot_ok(float s) { return s >= 0x1p-60f && s <= 0x1p60f; }

template <bool FAST>
__device__ __forceinline__ float quot(float v, float s, float r) {
  if (!FAST) return v / s;
  const float a = __builtin_fabsf(v);
  const float q0 = a * r;
  const float rem = __builtin_fmaf(-q0, s, a);
  return __builtin_copysignf(__builtin_fmaf(rem, r, q0), v);
}

// Codes of 4 values, packed little-endian (element 0 in the low byte).  The
// callers load values past the end of a row as +0, whose code is 0.
//  MODE 2: hardware conversion.  v_cvt_pk_fp8_f32 rounds to nearest even onto
//          E4M3; after clamping to [-448, 448] it gives the codes of
//          e4m3_encode for every non-NaN input (compared over all 2^32
//          binary32 inputs on gfx950), so this mode is used only for values
//          that hold no NaN, with a quotient from quot<true>.
//  MODE 1: quot<true> and e4m3_encode (NaN present).
//  MODE 0: the division and e4m3_encode (scale outside [2^-60, 2^60]).
template <int MODE>
using Mode = std::integral_constant<int, MODE>;

template <int MODE>
__device__ __forceinline__ uint32_t codes4(const float (&v)[4], float s, float r) {
  if constexpr (MODE == 2) {
    float c[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) c[e] = __builtin_amdgcn_fmed3f(quot<true>(v[e], s, r), -448.0f, 448.0f);
    const int lo = __builtin_amdgcn_cvt_pk_fp8_f32(c[0], c[1], 0, false);
    return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(c[2], c[3], lo, true);
  } else {
    uint32_t word = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) word |= e4m3_encode(quot<MODE == 1>(v[e], s, r)) << (8 * e);
    return word;
  }
}

// Runs emit(Mode<m>{}) with the mode that the scale and the lane's NaN flag allow.
template <typename F>
__device__ __forceinline__ void with_mode(float s, bool has_nan, F &&emit) {
  if (!quot_ok(s)) emit(Mode<0>{});
  else if (has_nan) emit(Mode<1>{});
  else emit(Mode<2>{});
}

// The row quantisers also clear nzero words (the column-amax words that a
// later column quantisation on the same stream accumulates into), one per
// thread of the grid, so that it needs no clearing launch of its own.  The
// host passes nzero = 0 when the grid has fewer threads than words.
__device__ __forceinline__ void clear_words(uint32_t *__restrict__ p, int64_t n) {
  const int64_t z = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (z < n) p[z] = 0u;
}

__device__ __forceinline__ float warp_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

// One workgroup per row of A: amax over the row, scale, then codes of the row
// (16 consecutive k per lane per step, one 16-byte store).
__global__ __launch_bounds__(256) void quant_rows_kernel(int M, int K, int64_t Kp,
                                                         const float *__restrict__ A, int64_t lda,
                                                         uint8_t *__restrict__ qa,
                                                         float *__restrict__ sa,
                                                         uint32_t *__restrict__ zero, int64_t nzero) {
  clear_words(zero, nzero);
  __shared__ float red[4];
  const int i = blockIdx.x;
  const float *row = A + (int64_t)i * lda;
  float m = 0.0f;
  for (int k = threadIdx.x; k < K; k += 256) m = fmaxf(m, fabsf(row[k]));
  m = warp_max(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
  const float s = (m == 0.0f) ? 1.0f : m / 448.0f;
  if (threadIdx.x == 0) sa[i] = s;
  const float r = 1.0f / s;
  uint8_t *q = qa + (int64_t)i * Kp;
  // Rows this long are re-read here; the NaN-safe mode 1 serves every value.
  auto emit = [&](auto mode) {
    constexpr int MD = decltype(mode)::value;
    for (int64_t k0 = (int64_t)threadIdx.x * 16; k0 < Kp; k0 += 256 * 16) {
      uint32_t w[4];
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int64_t k = k0 + g * 4;
        float v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = k + e < K ? row[k + e] : 0.0f;
        w[g] = codes4<MD>(v, s, r);
      }
      *reinterpret_cast<uint4 *>(q + k0) = make_uint4(w[0], w[1], w[2], w[3]);
    }
  };
  with_mode(s, true, emit);
}

// Single-pass variant for rows of at most 256*4*CH elements: the row stays
// in registers between the amax reduction and the encoding (one HBM read).
// Lane t owns elements 4t + 1024j .. +3 (j < CH) and stores their 4 codes as
// one 32-bit word.  VEC: lda % 4 == 0 and A 16-byte aligned.
template <int CH, bool VEC>
__global__ __launch_bounds__(256) void quant_rows_reg_kernel(int M, int K, int64_t Kp,
                                                             const float *__restrict__ A,
                                                             int64_t lda, uint8_t *__restrict__ qa,
                                                             float *__restrict__ sa,
                                                             uint32_t *__restrict__ zero,
                                                             int64_t nzero) {
  clear_words(zero, nzero);
  __shared__ float red[4];
  const int i = blockIdx.x;
  const float *row = A + (int64_t)i * lda;
  float v[CH][4];
  float m = 0.0f;
  bool nan = false;
#pragma unroll
  for (int j = 0; j < CH; ++j) {
    const int k = 4 * (int)threadIdx.x + 1024 * j;
    if (VEC && k + 3 < K) {
      const float4 x = *reinterpret_cast<const float4 *>(row + k);
      v[j][0] = x.x; v[j][1] = x.y; v[j][2] = x.z; v[j][3] = x.w;
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) v[j][e] = k + e < K ? row[k + e] : 0.0f;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      m = fmaxf(m, fabsf(v[j][e]));
      nan |= v[j][e] != v[j][e];
    }
  }
  m = warp_max(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
  const float s = (m == 0.0f) ? 1.0f : m / 448.0f;
  if (threadIdx.x == 0) sa[i] = s;
  const float r = 1.0f / s;
  uint8_t *q = qa + (int64_t)i * Kp;
  auto emit = [&](auto mode) {
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      const int k = 4 * (int)threadIdx.x + 1024 * j;
      if (k < Kp) *reinterpret_cast<uint32_t *>(q + k) = codes4<decltype(mode)::value>(v[j], s, r);
    }
  };
  with_mode(s, nan, emit);
}

// One wave per row (four rows per workgroup) for rows of at most 256 * CH
// padded elements: lane t holds elements 4t + 256j (j < CH) in registers, the amax
// is a wave reduction (no LDS, no barrier), and each lane stores the 4 codes
// of each of its groups as one 32-bit word.  VEC: ld % 4 == 0 and the base
// 16-byte aligned.
template <int CH, bool VEC>
__global__ __launch_bounds__(256) void quant_rows_wave_kernel(int M, int K, int64_t Kp,
                                                              const float *__restrict__ A,
                                                              int64_t lda, uint8_t *__restrict__ qa,
                                                              float *__restrict__ sa,
                                                              uint32_t *__restrict__ zero,
                                                              int64_t nzero) {
  clear_words(zero, nzero);
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (i >= M) return;
  const float *row = A + (int64_t)i * lda;
  float v[CH][4];
  float m = 0.0f;
  bool nan = false;
#pragma unroll
  for (int j = 0; j < CH; ++j) {
    const int k = 4 * lane + 256 * j;
    if (VEC && k + 3 < K) {
      const float4 x = *reinterpret_cast<const float4 *>(row + k);
      v[j][0] = x.x; v[j][1] = x.y; v[j][2] = x.z; v[j][3] = x.w;
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) v[j][e] = k + e < K ? row[k + e] : 0.0f;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      m = fmaxf(m, fabsf(v[j][e]));
      nan |= v[j][e] != v[j][e];
    }
  }
  m = warp_max(m);
  const float s = (m == 0.0f) ? 1.0f : m / 448.0f;
  if (lane == 0) sa[i] = s;
  const float r = 1.0f / s;
  uint8_t *q = qa + (int64_t)i * Kp;
  auto emit = [&](auto mode) {
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      const int k = 4 * lane + 256 * j;
      if (k < Kp) *reinterpret_cast<uint32_t *>(q + k) = codes4<decltype(mode)::value>(v[j], s, r);
    }
  };
  with_mode(s, nan, emit);
}

__global__ __launch_bounds__(256) void fill_u32_kernel(uint32_t *__restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    p[i] = 0u;
}

// Column amax over a 256-row x 64-column block: 16 lanes x float4 span the
// 64 columns, 16 lane-rows step through the 256 rows; an LDS reduction over
// the lane-rows, then one atomicMax per column.  VEC: ldb % 4 == 0, B aligned.
template <bool VEC>
__global__ __launch_bounds__(256) void col_amax4_kernel(int K, int N, const float *__restrict__ B,
                                                        int64_t ldb,
                                                        uint32_t *__restrict__ amax_bits) {
  __shared__ float red[16][65];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int j0 = blockIdx.x * 64 + tx * 4;
  const int k0 = blockIdx.y * 256;
  float m[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int r = ty; r < 256; r += 16) {
    const int k = k0 + r;
    if (k >= K) break;
    const float *p = B + (int64_t)k * ldb + j0;
    if (VEC && j0 + 3 < N) {
      const float4 x = *reinterpret_cast<const float4 *>(p);
      m[0] = fmaxf(m[0], fabsf(x.x)); m[1] = fmaxf(m[1], fabsf(x.y));
      m[2] = fmaxf(m[2], fabsf(x.z)); m[3] = fmaxf(m[3], fabsf(x.w));
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (j0 + e < N) m[e] = fmaxf(m[e], fabsf(p[e]));
    }
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) red[ty][tx * 4 + e] = m[e];
  __syncthreads();
  if (threadIdx.x < 64) {
    float x = 0.0f;
#pragma unroll
    for (int r = 0; r < 16; ++r) x = fmaxf(x, red[r][threadIdx.x]);
    const int j = blockIdx.x * 64 + (int)threadIdx.x;
    if (j < N) atomicMax(amax_bits + j, __builtin_bit_cast(uint32_t, x));
  }
}

// Quantise a 64(k) x 64(n) block of B with the column scales and store it
// transposed into qbT (row j holds column j of B, k contiguous).
__global__ __launch_bounds__(256) void quant_cols_t_kernel(int K, int N, int64_t Kp,
                                                           const float *__restrict__ B, int64_t ldb,
                                                           const uint32_t *__restrict__ amax_bits,
                                                           uint8_t *__restrict__ qbT,
                                                           float *__restrict__ sb) {
  // Rows of 68 bytes (17 words): the 64 lanes of a wave store to 64 different
  // banks when each writes one word of its own row.
  __shared__ __attribute__((aligned(16))) uint8_t tileT[64][64 + 4];
  const int kb = blockIdx.x * 64, nb = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int j = nb + tx;
  float s = 1.0f;
  if (j < N) {
    const float m = __builtin_bit_cast(float, amax_bits[j]);
    s = (m == 0.0f) ? 1.0f : m / 448.0f;
    if (blockIdx.x == 0 && ty == 0) sb[j] = s;
  }
  const float rs = 1.0f / s;
  // Lane (tx, ty) holds rows 16 ty + i (i < 16) of its column; for each i the
  // wave reads 64 consecutive floats of one row.
  float x[16];
  bool nan = false;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int k = kb + 16 * ty + i;
    x[i] = (k < K && j < N) ? B[(int64_t)k * ldb + j] : 0.0f;
    nan |= x[i] != x[i];
  }
  auto emit = [&](auto mode) {
#pragma unroll
    for (int i = 0; i < 16; i += 4) {
      const float g[4] = {x[i], x[i + 1], x[i + 2], x[i + 3]};
      *reinterpret_cast<uint32_t *>(&tileT[tx][16 * ty + i]) = codes4<decltype(mode)::value>(g, s, rs);
    }
  };
  with_mode(s, nan, emit);  // per column: lanes may take different modes
  __syncthreads();
  // 64 rows (n) x 64 bytes (k): each lane stores 16 bytes.
  const int row = threadIdx.x >> 2, seg = (threadIdx.x & 3) * 16;
  const int jn = nb + row;
  if (jn < N) {
    const uint32_t *src = reinterpret_cast<const uint32_t *>(&tileT[row][seg]);
    *reinterpret_cast<uint4 *>(qbT + (int64_t)jn * Kp + kb + seg) =
        make_uint4(src[0], src[1], src[2], src[3]);
  }
}

// One-pass column quantisation for K <= 1024 * CQ: a workgroup of 1024 lanes
// holds a stripe of 16 columns of the K x Nc matrix in registers between the
// amax reduction and the encoding, so the matrix is read from HBM once (the
// two-pass path reads it for the amax and again for the codes).  Lane (tx, ty)
// = (tid & 3, tid >> 2) holds columns j0 + 4 tx .. + 3 of rows 4 (ty + 256 i)
// .. + 3 (i < CQ): 4 consecutive k of each of its 4 columns, so each column's
// codes come out as 32-bit words of 4 consecutive k, stored straight into the
// transposed layout (row j of qT holds column j, k contiguous) -- the 16 lanes
// of a wave with one tx write 64 contiguous bytes of each of their columns.
// Stripes are remapped so that the two stripes of one 128-byte row segment
// run on one XCD (their shared lines meet in its L2).  VEC: ld % 4 == 0 and
// the base 16-byte aligned.
template <int CQ, bool VEC>
__global__ __launch_bounds__(1024) void quant_cols_reg_kernel(int K, int Nc, int64_t Kp,
                                                              const float *__restrict__ B,
                                                              int64_t ldb,
                                                              uint8_t *__restrict__ qT,
                                                              float *__restrict__ scales) {
  __shared__ float red[16][16];
  const int tid = threadIdx.x, tx = tid & 3, ty = tid >> 2;
  const int stripe = xcd_remap(blockIdx.x, gridDim.x);
  const int j0 = stripe * 16 + tx * 4;  // the lane's first column
  float x[CQ][4][4];                    // [block i][row e][column c]
  float m[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  bool nan[4] = {false, false, false, false};
#pragma unroll
  for (int i = 0; i < CQ; ++i)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = 4 * (ty + 256 * i) + e;
      const float *p = B + (int64_t)k * ldb + j0;
      if (VEC && k < K && j0 + 3 < Nc) {
        const float4 v = *reinterpret_cast<const float4 *>(p);
        x[i][e][0] = v.x; x[i][e][1] = v.y; x[i][e][2] = v.z; x[i][e][3] = v.w;
      } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) x[i][e][c] = (k < K && j0 + c < Nc) ? p[c] : 0.0f;
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        m[c] = fmaxf(m[c], fabsf(x[i][e][c]));
        nan[c] |= x[i][e][c] != x[i][e][c];
      }
    }
  // column maxima: over the 16 lanes of a wave with the same tx, then over
  // the 16 waves
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int o = 4; o < 64; o <<= 1) m[c] = fmaxf(m[c], __shfl_xor(m[c], o, 64));
  const int wave = tid >> 6;
  if ((tid & 63) < 4) {
#pragma unroll
    for (int c = 0; c < 4; ++c) red[wave][tx * 4 + c] = m[c];
  }
  __syncthreads();
  float sc[4], rc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    float a = red[0][tx * 4 + c];
#pragma unroll
    for (int w = 1; w < 16; ++w) a = fmaxf(a, red[w][tx * 4 + c]);
    sc[c] = (a == 0.0f) ? 1.0f : a / 448.0f;
    rc[c] = 1.0f / sc[c];
    if (ty == 0 && j0 + c < Nc) scales[j0 + c] = sc[c];
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if (j0 + c >= Nc) continue;
    uint8_t *q = qT + (int64_t)(j0 + c) * Kp;
    auto emit = [&](auto mode) {
#pragma unroll
      for (int i = 0; i < CQ; ++i) {
        const int k = 4 * (ty + 256 * i);
        const float g[4] = {x[i][0][c], x[i][1][c], x[i][2][c], x[i][3][c]};
        if (k < Kp) *reinterpret_cast<uint32_t *>(q + k) = codes4<decltype(mode)::value>(g, sc[c], rc[c]);
      }
    };
    with_mode(sc[c], nan[c], emit);  // per column: lanes may take different modes
  }
}

// ---------------------------------------------------------------- GEMM ----
// 256 x 256 tile, 128-byte K slabs, 2 x 2 waves of 128 x 128, MFMA
// v_mfma_f32_32x32x64_f8f6f4 with both operands E4M3.  LDS rows are 128
// bytes with an XOR swizzle of the 16-byte chunk index.
template <int BM, int BN, int WM, int WN>
struct Fp8Cfg {
  static constexpr int NT = 64 * (BM / WM) * (BN / WN);
  static constexpr int BK = 128;
  static constexpr int WAVES_N = BN / WN;
  static_assert((BM / WM) * WAVES_N == 4 || (BM / WM) * WAVES_N == 8, "4 or 8 waves");
  static constexpr int FM = WM / 32, FN = WN / 32;
  static constexpr int A_CH = BM * BK / 16 / NT;   // 16-byte chunks per lane per slab
  static constexpr int B_CH = BN * BK / 16 / NT;
  static constexpr int STAGE = (BM + BN) * BK;     // bytes
  static constexpr int LDS_BYTES = 2 * STAGE;
};

__device__ __forceinline__ int swz8(int r) { return (r ^ (r >> 3)) & 7; }

// Cache policy of the C stores: non-temporal (the slc bit of the buffer
// instruction, NT on gfx950), a hint only.  C is written once at the end of a
// tile; streaming it keeps the A and B code panels that the next round of
// tiles reads in L2 (8192^2 x 4096: 329 -> 312 us; 4096^3 1 % faster).
constexpr int kStoreNT = 2;

// Epilogue of both FP8 kernels: C <- (sa[i] * (sb[j] * alpha)) * acc + beta * C
// over the wave's FM x FN blocks of 32 x 32.  Through buffer resources over
// the tile's valid part of C and of the scale vectors (rows and columns past
// the matrix read as zero and their stores are dropped), one block row at a
// time: its scales and, with beta != 0, its C values are all loaded before
// its first store (a buffer load is never moved above a buffer store through
// the same resource, so a read-modify-write per element would wait out one
// memory round trip per element).  A C row stride too large for 32-bit
// offsets takes the element-wise path.
template <int FM, int FN, int BM, int BN, bool BETA>
__device__ __forceinline__ void epilogue(const f32x16 (&acc)[FM][FN], int Mr, int Nr, int m0,
                                         int n0, int wm0, int wn0, int lrow, int lgrp,
                                         float alpha, const float *__restrict__ sa,
                                         const float *__restrict__ sb, float beta,
                                         float *__restrict__ C, int64_t ldc) {
  const int rowsC = Mr < BM ? Mr : BM, cols = Nr < BN ? Nr : BN;
  if ((int64_t)BM * ldc * 4 < ((int64_t)1 << 31)) {
    const __amdgpu_buffer_rsrc_t rC = __builtin_amdgcn_make_buffer_rsrc(
        C + (int64_t)m0 * ldc + n0, (short)0, (int)(((int64_t)(rowsC - 1) * ldc + cols) * 4),
        kBufferFlags);
    const __amdgpu_buffer_rsrc_t rSa = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float *>(sa + m0), (short)0, rowsC * 4, kBufferFlags);
    const __amdgpu_buffer_rsrc_t rSb = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float *>(sb + n0), (short)0, cols * 4, kBufferFlags);
    const int ldc4 = (int)ldc * 4;
    float sj[FN];
    int vb[FN];
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int col = wn0 + j * 32 + lrow;
      const bool in = col < cols;
      sj[j] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                            rSb, in ? col * 4 : (int)0x80000000, 0, 0)) * alpha;
      vb[j] = in ? col * 4 : (int)0x80000000;
    }
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      const int r0 = wm0 + i * 32 + 4 * lgrp;  // row of element 0; element e adds 8(e/4) + e%4
      float si[16], cold[FN][16];
#pragma unroll
      for (int e = 0; e < 16; ++e)
        si[e] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                              rSa, (r0 + 8 * (e >> 2) + (e & 3)) * 4, 0, 0));
      if (BETA) {
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int e = 0; e < 16; ++e)
            cold[j][e] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                                       rC, vb[j], (r0 + 8 * (e >> 2) + (e & 3)) * ldc4, 0));
      }
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          float v = (si[e] * sj[j]) * acc[i][j][e];
          if (BETA) v = fmaf(beta, cold[j][e], v);
          __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), rC, vb[j],
                                                (r0 + 8 * (e >> 2) + (e & 3)) * ldc4,
                                                kStoreNT);
        }
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int col = wn0 + j * 32 + lrow;
      if (col >= Nr) continue;
      const float sj = sb[n0 + col] * alpha;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int row = wm0 + i * 32 + 8 * (e >> 2) + 4 * lgrp + (e & 3);
        if (row < Mr) {
          float *p = C + (int64_t)(m0 + row) * ldc + (n0 + col);
          const float v = (sa[m0 + row] * sj) * acc[i][j][e];
          *p = BETA ? fmaf(beta, *p, v) : v;
        }
      }
    }
}

template <int BM, int BN, int WM, int WN, bool BETA>
__global__ __launch_bounds__(64 * (BM / WM) * (BN / WN), 1) void gemm_fp8_kernel(
    int M, int N, int64_t Kp, float alpha, const uint8_t *__restrict__ qa,
    const uint8_t *__restrict__ qbT, const float *__restrict__ sa, const float *__restrict__ sb,
    float beta, float *__restrict__ C, int64_t ldc, int tiles_m, int tiles_n) {
  using G = Fp8Cfg<BM, BN, WM, WN>;
  __shared__ __attribute__((aligned(16))) uint8_t lds[G::LDS_BYTES];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wg = xcd_remap(blockIdx.x, gridDim.x);
  int tm, tn;
  tile_coords(wg, tiles_m, tiles_n, 8, tm, tn);
  const int m0 = tm * BM, n0 = tn * BN;
  const int Mr = M - m0, Nr = N - n0;

  // Raw buffer loads: rows past M (N) lie beyond num_records and read as 0;
  // lane offsets are 32-bit (the launcher bounds 256 * Kp < 2^31).
  const int rowsA = Mr < BM ? Mr : BM, rowsB = Nr < BN ? Nr : BN;
  const __amdgpu_buffer_rsrc_t rsA = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<uint8_t *>(qa + (int64_t)m0 * Kp), (short)0, (int)(rowsA * Kp), kBufferFlags);
  const __amdgpu_buffer_rsrc_t rsB = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<uint8_t *>(qbT + (int64_t)n0 * Kp), (short)0, (int)(rowsB * Kp), kBufferFlags);
  int voA[G::A_CH], voB[G::B_CH];
#pragma unroll
  for (int i = 0; i < G::A_CH; ++i) {
    const int idx = tid + G::NT * i;
    voA[i] = (idx >> 3) * (int)Kp + (idx & 7) * 16;
  }
#pragma unroll
  for (int i = 0; i < G::B_CH; ++i) {
    const int idx = tid + G::NT * i;
    voB[i] = (idx >> 3) * (int)Kp + (idx & 7) * 16;
  }
  u32x4 ra[2][G::A_CH], rb[2][G::B_CH];
  auto gload = [&](auto S, int k0) {
    constexpr int set = decltype(S)::value;
#pragma unroll
    for (int i = 0; i < G::A_CH; ++i)
      ra[set][i] = __builtin_amdgcn_raw_buffer_load_b128(rsA, voA[i] + k0, 0, 0);
#pragma unroll
    for (int i = 0; i < G::B_CH; ++i)
      rb[set][i] = __builtin_amdgcn_raw_buffer_load_b128(rsB, voB[i] + k0, 0, 0);
  };
  auto sstore = [&](auto S, int stage) {
    constexpr int set = decltype(S)::value;
    uint8_t *sA = lds + stage * G::STAGE;
    uint8_t *sB = sA + BM * G::BK;
#pragma unroll
    for (int i = 0; i < G::A_CH; ++i) {
      const int idx = tid + G::NT * i;
      const int r = idx >> 3, c = idx & 7;
      *reinterpret_cast<u32x4 *>(sA + r * G::BK + ((c ^ swz8(r)) << 4)) = ra[set][i];
    }
#pragma unroll
    for (int i = 0; i < G::B_CH; ++i) {
      const int idx = tid + G::NT * i;
      const int r = idx >> 3, c = idx & 7;
      *reinterpret_cast<u32x4 *>(sB + r * G::BK + ((c ^ swz8(r)) << 4)) = rb[set][i];
    }
  };

  const int wm0 = (wave / G::WAVES_N) * WM, wn0 = (wave % G::WAVES_N) * WN;
  const int lrow = lane & 31, lgrp = lane >> 5;
  f32x16 acc[G::FM][G::FN];
#pragma unroll
  for (int i = 0; i < G::FM; ++i)
#pragma unroll
    for (int j = 0; j < G::FN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;

  auto mfma_step = [&](int stage, int ks) {
    const uint8_t *sA = lds + stage * G::STAGE;
    const uint8_t *sB = sA + BM * G::BK;
    // lane holds 32 consecutive k (two 16-byte chunks) of its row / column
    const int c0 = ks * 4 + lgrp * 2;
    i32x8 a[G::FM], b[G::FN];
#pragma unroll
    for (int i = 0; i < G::FM; ++i) {
      const int r = wm0 + i * 32 + lrow;
      const uint4 lo = *reinterpret_cast<const uint4 *>(sA + r * G::BK + ((c0 ^ swz8(r)) << 4));
      const uint4 hi = *reinterpret_cast<const uint4 *>(sA + r * G::BK + (((c0 + 1) ^ swz8(r)) << 4));
      a[i] = i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
    }
#pragma unroll
    for (int j = 0; j < G::FN; ++j) {
      const int r = wn0 + j * 32 + lrow;
      const uint4 lo = *reinterpret_cast<const uint4 *>(sB + r * G::BK + ((c0 ^ swz8(r)) << 4));
      const uint4 hi = *reinterpret_cast<const uint4 *>(sB + r * G::BK + (((c0 + 1) ^ swz8(r)) << 4));
      b[j] = i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
    }
#pragma unroll
    for (int i = 0; i < G::FM; ++i)
#pragma unroll
      for (int j = 0; j < G::FN; ++j)
        // formats: 0 = E4M3 for both operands; no block scaling
        acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a[i], b[j], acc[i][j], 0, 0,
                                                                     0, 0, 0, 0);
  };

  // K loop: slab t multiplied from stage t%2 while slab t+2 is in flight into
  // one register set and slab t+1 (already in the other set) is written to
  // the other stage; one barrier per slab.  Loads past the last slab are
  // clamped to it (in-bounds reads never consumed) so that every iteration
  // issues the same instructions and each wait covers only what it needs.
  using S0 = std::integral_constant<int, 0>;
  using S1 = std::integral_constant<int, 1>;
  const int KT = (int)(Kp / G::BK);
  auto kslab = [&](int sl) { return (sl < KT ? sl : KT - 1) * G::BK; };
  gload(S0{}, 0);
  sstore(S0{}, 0);
  gload(S1{}, kslab(1));
  __syncthreads();
  int t = 0;
  for (; t + 2 <= KT; t += 2) {
    gload(S0{}, kslab(t + 2));
    __builtin_amdgcn_sched_barrier(0);
    mfma_step(0, 0);
    mfma_step(0, 1);
    sstore(S1{}, 1);
    __syncthreads();
    gload(S1{}, kslab(t + 3));
    __builtin_amdgcn_sched_barrier(0);
    mfma_step(1, 0);
    mfma_step(1, 1);
    sstore(S0{}, 0);
    __syncthreads();
  }
  if (t < KT) {
    mfma_step(0, 0);
    mfma_step(0, 1);
  }

  epilogue<G::FM, G::FN, BM, BN, BETA>(acc, Mr, Nr, m0, n0, wm0, wn0, lrow, lgrp, alpha, sa, sb,
                                        beta, C, ldc);
}

// Same tile, MFMA and epilogue, but the operand codes go from HBM straight
// into LDS (buffer_load_dwordx4 ... lds): no register stage, so no VGPRs hold
// slabs in flight and no VALU/LDS-store work sits between load and use.  A
// wave's DMA writes 1024 contiguous LDS bytes (8 rows of 128 bytes, lane l at
// byte 16 l); the swizzle is applied on the global side, i.e. the lane that
// fills physical chunk p of row r fetches logical chunk p ^ swz8(r).  Two
// separate LDS arrays hold the two stages.  Slab t+1 is in flight into one
// stage while slab t is multiplied from the other; one barrier per slab,
// preceded by a wait for the wave's own DMA.
// 16 bytes per lane from a buffer resource into LDS at lds + 16 * lane (lds
// must be wave-uniform).  The LDS address-space cast exists only in the device
// pass; the host pass sees an empty body.
__device__ __forceinline__ void lds_load16(__amdgpu_buffer_rsrc_t rs, uint8_t *lds, int voffset) {
#if defined(__HIP_DEVICE_COMPILE__)
  __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void *)lds, 16,
                                           voffset, 0, 0, 0);
#endif
}

template <int BM, int BN, int WM, int WN, bool BETA>
__global__ __launch_bounds__(64 * (BM / WM) * (BN / WN), 1) void gemm_fp8_dma_kernel(
    int M, int N, int64_t Kp, float alpha, const uint8_t *__restrict__ qa,
    const uint8_t *__restrict__ qbT, const float *__restrict__ sa, const float *__restrict__ sb,
    float beta, float *__restrict__ C, int64_t ldc, int tiles_m, int tiles_n) {
  using G = Fp8Cfg<BM, BN, WM, WN>;
  constexpr int NW = G::NT / 64;
  __shared__ __attribute__((aligned(1024))) uint8_t st0[G::STAGE];
  __shared__ __attribute__((aligned(1024))) uint8_t st1[G::STAGE];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wg = xcd_remap(blockIdx.x, gridDim.x);
  int tm, tn;
  tile_coords(wg, tiles_m, tiles_n, 8, tm, tn);
  const int m0 = tm * BM, n0 = tn * BN;
  const int Mr = M - m0, Nr = N - n0;
  const int rowsA = Mr < BM ? Mr : BM, rowsB = Nr < BN ? Nr : BN;
  // Rows past M (N) read as zero; they feed only C rows (columns) that are
  // never stored.
  const __amdgpu_buffer_rsrc_t rsA = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<uint8_t *>(qa + (int64_t)m0 * Kp), (short)0, (int)(rowsA * Kp), kBufferFlags);
  const __amdgpu_buffer_rsrc_t rsB = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<uint8_t *>(qbT + (int64_t)n0 * Kp), (short)0, (int)(rowsB * Kp), kBufferFlags);
  // DMA block d (1024 bytes) covers stage rows 8d..8d+7; block d of A is
  // issued by wave d % NW as its (d / NW)-th A load.
  int voA[G::A_CH], voB[G::B_CH];
#pragma unroll
  for (int i = 0; i < G::A_CH; ++i) {
    const int r = (i * NW + wave) * 8 + (lane >> 3);
    voA[i] = r * (int)Kp + (((lane & 7) ^ swz8(r)) << 4);
  }
#pragma unroll
  for (int i = 0; i < G::B_CH; ++i) {
    const int r = (i * NW + wave) * 8 + (lane >> 3);
    voB[i] = r * (int)Kp + (((lane & 7) ^ swz8(r)) << 4);
  }
  auto dma = [&](uint8_t *stage, int k0) {
#pragma unroll
    for (int i = 0; i < G::A_CH; ++i) lds_load16(rsA, stage + (i * NW + wave) * 1024, voA[i] + k0);
#pragma unroll
    for (int i = 0; i < G::B_CH; ++i)
      lds_load16(rsB, stage + BM * G::BK + (i * NW + wave) * 1024, voB[i] + k0);
  };

  const int wm0 = (wave / G::WAVES_N) * WM, wn0 = (wave % G::WAVES_N) * WN;
  const int lrow = lane & 31, lgrp = lane >> 5;
  f32x16 acc[G::FM][G::FN];
#pragma unroll
  for (int i = 0; i < G::FM; ++i)
#pragma unroll
    for (int j = 0; j < G::FN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;

  auto mfma_step = [&](const uint8_t *sA, int ks) {
    const uint8_t *sB = sA + BM * G::BK;
    const int c0 = ks * 4 + lgrp * 2;
    i32x8 a[G::FM], b[G::FN];
#pragma unroll
    for (int i = 0; i < G::FM; ++i) {
      const int r = wm0 + i * 32 + lrow;
      const uint4 lo = *reinterpret_cast<const uint4 *>(sA + r * G::BK + ((c0 ^ swz8(r)) << 4));
      const uint4 hi = *reinterpret_cast<const uint4 *>(sA + r * G::BK + (((c0 + 1) ^ swz8(r)) << 4));
      a[i] = i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
    }
#pragma unroll
    for (int j = 0; j < G::FN; ++j) {
      const int r = wn0 + j * 32 + lrow;
      const uint4 lo = *reinterpret_cast<const uint4 *>(sB + r * G::BK + ((c0 ^ swz8(r)) << 4));
      const uint4 hi = *reinterpret_cast<const uint4 *>(sB + r * G::BK + (((c0 + 1) ^ swz8(r)) << 4));
      b[j] = i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
    }
#pragma unroll
    for (int i = 0; i < G::FM; ++i)
#pragma unroll
      for (int j = 0; j < G::FN; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a[i], b[j], acc[i][j], 0, 0,
                                                                     0, 0, 0, 0);
  };

  // Loads past the last slab are clamped to it: in-bounds, never consumed.
  const int KT = (int)(Kp / G::BK);
  auto kslab = [&](int sl) { return (sl < KT ? sl : KT - 1) * G::BK; };
  dma(st0, 0);
  int t = 0;
  for (; t + 2 <= KT; t += 2) {
    __builtin_amdgcn_s_waitcnt(0);  // this wave's DMA of slab t has landed
    __syncthreads();                // ... and every wave's; stage 1 is free
    dma(st1, kslab(t + 1));
    __builtin_amdgcn_sched_barrier(0);  // keep the DMA issue ahead of the MFMAs
    mfma_step(st0, 0);
    mfma_step(st0, 1);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    dma(st0, kslab(t + 2));
    __builtin_amdgcn_sched_barrier(0);
    mfma_step(st1, 0);
    mfma_step(st1, 1);
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (t < KT) {
    mfma_step(st0, 0);
    mfma_step(st0, 1);
  }

  epilogue<G::FM, G::FN, BM, BN, BETA>(acc, Mr, Nr, m0, n0, wm0, wn0, lrow, lgrp, alpha, sa, sb,
                                        beta, C, ldc);
}

// The direct-to-LDS tile with 64-deep slabs in a ring of four LDS stages:
// the DMA of slab t+3 is issued once slab t has landed in every wave, so three
// slabs are in flight while one is multiplied (the two-stage kernel above has
// one).  LDS rows are 64 bytes (64 codes); a wave's DMA fills 1024 contiguous
// bytes, 16 rows, lane l at byte 16 l; the chunk swizzle (r >> 2) & 3 makes each
// group of 16 consecutive rows read at one logical chunk cover the 64 banks
// once.  One MFMA k-step (64 codes) per slab and stage.
__device__ __forceinline__ int swz4(int r) { return (r >> 2) & 3; }

template <int BM, int BN, int WM, int WN, bool BETA>
__global__ __launch_bounds__(64 * (BM / WM) * (BN / WN), 1) void gemm_fp8_ring_kernel(
    int M, int N, int64_t Kp, float alpha, const uint8_t *__restrict__ qa,
    const uint8_t *__restrict__ qbT, const float *__restrict__ sa, const float *__restrict__ sb,
    float beta, float *__restrict__ C, int64_t ldc, int tiles_m, int tiles_n) {
  constexpr int BK = 64, NST = 4;
  constexpr int NT = 64 * (BM / WM) * (BN / WN), NW = NT / 64, WAVES_N = BN / WN;
  constexpr int FM = WM / 32, FN = WN / 32;
  constexpr int STAGE = (BM + BN) * BK;
  constexpr int A_CH = BM * BK / 16 / NT, B_CH = BN * BK / 16 / NT;  // DMA blocks per wave and slab
  static_assert(A_CH * NT * 16 == BM * BK && B_CH * NT * 16 == BN * BK, "whole DMA blocks per wave");
  // four arrays rather than one: the compiler then knows which stage each
  // DMA writes and each fragment read reads, and waits only for the DMA of
  // the stage being read (one array would make every read wait for all)
  __shared__ __attribute__((aligned(1024))) uint8_t st0[STAGE];
  __shared__ __attribute__((aligned(1024))) uint8_t st1[STAGE];
  __shared__ __attribute__((aligned(1024))) uint8_t st2[STAGE];
  __shared__ __attribute__((aligned(1024))) uint8_t st3[STAGE];
  static_assert(NST == 4, "four stage arrays");
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wg = xcd_remap(blockIdx.x, gridDim.x);
  int tm, tn;
  tile_coords(wg, tiles_m, tiles_n, 8, tm, tn);
  const int m0 = tm * BM, n0 = tn * BN;
  const int Mr = M - m0, Nr = N - n0;
  const int rowsA = Mr < BM ? Mr : BM, rowsB = Nr < BN ? Nr : BN;
  const __amdgpu_buffer_rsrc_t rsA = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<uint8_t *>(qa + (int64_t)m0 * Kp), (short)0, (int)(rowsA * Kp), kBufferFlags);
  const __amdgpu_buffer_rsrc_t rsB = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<uint8_t *>(qbT + (int64_t)n0 * Kp), (short)0, (int)(rowsB * Kp), kBufferFlags);
  // DMA block d (1024 bytes) covers stage rows 16d .. 16d+15; block d of A is
  // issued by wave d % NW as its (d / NW)-th A block.  The lane filling
  // physical chunk p of row r fetches logical chunk p ^ swz4(r).
  int voA[A_CH], voB[B_CH];
#pragma unroll
  for (int i = 0; i < A_CH; ++i) {
    const int r = (i * NW + wave) * 16 + (lane >> 2);
    voA[i] = r * (int)Kp + (((lane & 3) ^ swz4(r)) << 4);
  }
#pragma unroll
  for (int i = 0; i < B_CH; ++i) {
    const int r = (i * NW + wave) * 16 + (lane >> 2);
    voB[i] = r * (int)Kp + (((lane & 3) ^ swz4(r)) << 4);
  }
  auto dma = [&](uint8_t *stage, int k0) {
#pragma unroll
    for (int i = 0; i < A_CH; ++i) lds_load16(rsA, stage + (i * NW + wave) * 1024, voA[i] + k0);
#pragma unroll
    for (int i = 0; i < B_CH; ++i)
      lds_load16(rsB, stage + BM * BK + (i * NW + wave) * 1024, voB[i] + k0);
  };
  const int wm0 = (wave / WAVES_N) * WM, wn0 = (wave % WAVES_N) * WN;
  const int lrow = lane & 31, lgrp = lane >> 5;
  f32x16 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;
  auto mfma_slab = [&](const uint8_t *sA) {
    const uint8_t *sB = sA + BM * BK;
    const int c0 = lgrp * 2;  // the lane's 32 codes: logical chunks c0, c0 + 1
    i32x8 a[FM], b[FN];
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      const int r = wm0 + i * 32 + lrow;
      const uint4 lo = *reinterpret_cast<const uint4 *>(sA + r * BK + ((c0 ^ swz4(r)) << 4));
      const uint4 hi = *reinterpret_cast<const uint4 *>(sA + r * BK + (((c0 + 1) ^ swz4(r)) << 4));
      a[i] = i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
    }
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int r = wn0 + j * 32 + lrow;
      const uint4 lo = *reinterpret_cast<const uint4 *>(sB + r * BK + ((c0 ^ swz4(r)) << 4));
      const uint4 hi = *reinterpret_cast<const uint4 *>(sB + r * BK + (((c0 + 1) ^ swz4(r)) << 4));
      b[j] = i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
    }
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a[i], b[j], acc[i][j], 0, 0,
                                                                     0, 0, 0, 0);
  };
  // Kp is a multiple of 128, so KT >= 2.  DMAs past the last slab are clamped
  // to it (in-bounds, never consumed): every iteration issues the same count,
  // and the wait at its top leaves exactly the two later slabs in flight.
  const int KT = (int)(Kp / BK);
  auto kslab = [&](int sl) { return (sl < KT ? sl : KT - 1) * BK; };
  constexpr int kPer = A_CH + B_CH;  // DMA instructions per wave and slab
  // s_waitcnt with vmcnt = the two later slabs' DMAs (gfx9 encoding: vmcnt in
  // bits 3:0 and 15:14), lgkmcnt = 0 (bits 11:8: this wave's LDS reads have
  // completed, so no read of a stage is in flight when the barrier releases
  // its refill), expcnt at its maximum (bits 6:4, no wait)
  constexpr int kWaitTwoLater = ((2 * kPer) & 15) | (((2 * kPer) >> 4) << 14) | (7 << 4);
  static_assert(2 * kPer < 64, "vmcnt range");
  // step of slab t: cur = stage t % 4, prev = stage (t + 3) % 4, which held slab t-1
  // The barrier is the bare instruction: a workgroup fence (as in
  // __syncthreads) would wait for every outstanding load, the two later
  // slabs' DMAs included.  The explicit wait before it covers slab t's DMA,
  // the fragment reads of slab t-1 completed before the MFMAs that consumed
  // them, and the empty asm statements keep the compiler from moving memory
  // accesses across it.  The wait also drains this wave's LDS reads: the
  // compiler may leave the last fragment reads of slab t-1 in flight across
  // the barrier, and the DMA issued after it refills that stage.
  auto step = [&](uint8_t *cur, uint8_t *prev, int t) {
    __builtin_amdgcn_s_waitcnt(kWaitTwoLater);  // this wave's DMA of slab t has landed,
                                                // its LDS reads are complete
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();  // ... and every wave's; every wave is done with slab t-1's stage
    asm volatile("" ::: "memory");
    dma(prev, kslab(t + 3));
    __builtin_amdgcn_sched_barrier(0);
    mfma_slab(cur);
  };
  dma(st0, kslab(0));
  dma(st1, kslab(1));
  dma(st2, kslab(2));
  int t = 0;
  for (; t + 4 <= KT; t += 4) {
    step(st0, st3, t);
    step(st1, st0, t + 1);
    step(st2, st1, t + 2);
    step(st3, st2, t + 3);
  }
  if (t < KT) {  // KT is even: two slabs left
    step(st0, st3, t);
    step(st1, st0, t + 1);
  }
  __builtin_amdgcn_s_waitcnt(0);  // the clamped DMAs have landed before the workgroup ends
  epilogue<FM, FN, BM, BN, BETA>(acc, Mr, Nr, m0, n0, wm0, wn0, lrow, lgrp, alpha, sa, sb, beta,
                                 C, ldc);
}

// Raw conversion, for verification of the encoder.
__global__ __launch_bounds__(256) void encode_kernel(int64_t n, const float *__restrict__ x,
                                                     uint8_t *__restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    out[i] = (uint8_t)e4m3_encode(x[i]);
}

}  // namespace fp8

size_t fp8_ws_bytes(int64_t M, int64_t N, int64_t K) { return fp8::layout(M, N, K).total; }
int64_t fp8_kp(int64_t K) { return fp8::layout(0, 0, K).Kp; }

// Row quantisation: R rows of K binary32 values (row stride ld) -> per-row
// scales and codes in rows of Kp bytes (k contiguous).  zero: nzero words that
// the launch also clears when its grid has a thread for each (for a later
// quant_cols on the same stream); *cleared tells whether it did.
static gemm_status quant_rows(int64_t R, int64_t K, int64_t Kp, const float *P, int64_t ld,
                              uint8_t *q, float *scales, hipStream_t s,
                              uint32_t *zero = nullptr, int64_t nzero = 0,
                              bool *cleared = nullptr) {
  const bool vec = ld % 4 == 0 && ((uintptr_t)P & 15) == 0;
  const int chw = (int)((Kp + 255) / 256);
  const int64_t threads = 256 * (chw <= 2 ? (R + 3) / 4 : R);
  if (zero == nullptr || nzero > threads) nzero = 0;
  if (cleared) *cleared = nzero > 0;
  // Short rows (at most 512 padded elements): one wave per row.  Measured on
  // 4096-row operands, 7 % faster than a workgroup per row at K = 300 and
  // 16 % slower at K = 4096, where four rows per workgroup keep too few bytes
  // in flight per CU.
  if (chw <= 2) {
    const unsigned grid = (unsigned)((R + 3) / 4);
#define MM_QWAVE(CH)                                                                               \
  do {                                                                                             \
    if (vec)                                                                                       \
      hipLaunchKernelGGL((fp8::quant_rows_wave_kernel<CH, true>), dim3(grid), dim3(256), 0, s,      \
                         (int)R, (int)K, Kp, P, ld, q, scales, zero, nzero);                       \
    else                                                                                           \
      hipLaunchKernelGGL((fp8::quant_rows_wave_kernel<CH, false>), dim3(grid), dim3(256), 0, s,     \
                         (int)R, (int)K, Kp, P, ld, q, scales, zero, nzero);                       \
  } while (0)
    if (chw == 1) MM_QWAVE(1);
    else MM_QWAVE(2);
#undef MM_QWAVE
    return check_launch("quant_rows_wave_kernel");
  }
  const int ch = (int)((Kp + 1023) / 1024);
#define MM_QROWS(CH)                                                                             \
  do {                                                                                           \
    if (vec)                                                                                     \
      hipLaunchKernelGGL((fp8::quant_rows_reg_kernel<CH, true>), dim3((unsigned)R), dim3(256), 0, \
                         s, (int)R, (int)K, Kp, P, ld, q, scales, zero, nzero);                  \
    else                                                                                         \
      hipLaunchKernelGGL((fp8::quant_rows_reg_kernel<CH, false>), dim3((unsigned)R), dim3(256),  \
                         0, s, (int)R, (int)K, Kp, P, ld, q, scales, zero, nzero);               \
  } while (0)
  switch (ch) {
    case 1: MM_QROWS(1); break;
    case 2: MM_QROWS(2); break;
    case 3: MM_QROWS(3); break;
    case 4: MM_QROWS(4); break;
    case 5: MM_QROWS(5); break;
    case 6: MM_QROWS(6); break;
    case 7: MM_QROWS(7); break;
    case 8: MM_QROWS(8); break;
    default:
      hipLaunchKernelGGL(fp8::quant_rows_kernel, dim3((unsigned)R), dim3(256), 0, s, (int)R,
                         (int)K, Kp, P, ld, q, scales, zero, nzero);
  }
#undef MM_QROWS
  return check_launch("quant_rows_kernel");
}

// Column quantisation: a K x Nc matrix (row stride ld) -> per-column scales
// and the codes of each column in a row of Kp bytes (transposed, k
// contiguous).  amax: Nc words of scratch, already zero when amax_clear.
static gemm_status quant_cols(int64_t K, int64_t Nc, int64_t Kp, const float *P, int64_t ld,
                              uint32_t *amax, uint8_t *q, float *scales, hipStream_t s,
                              bool amax_clear = false) {
  // up to 4096 rows: one pass, the stripe held in registers
  if (Kp <= 4096) {
    const bool vec1 = ld % 4 == 0 && ((uintptr_t)P & 15) == 0;
    const dim3 grid((unsigned)((Nc + 15) / 16));
#define MM_QCOLS(CQ)                                                                             \
  do {                                                                                           \
    if (vec1)                                                                                    \
      hipLaunchKernelGGL((fp8::quant_cols_reg_kernel<CQ, true>), grid, dim3(1024), 0, s, (int)K, \
                         (int)Nc, Kp, P, ld, q, scales);                                         \
    else                                                                                         \
      hipLaunchKernelGGL((fp8::quant_cols_reg_kernel<CQ, false>), grid, dim3(1024), 0, s,        \
                         (int)K, (int)Nc, Kp, P, ld, q, scales);                                 \
  } while (0)
    if (Kp <= 1024) MM_QCOLS(1);
    else if (Kp <= 2048) MM_QCOLS(2);
    else if (Kp <= 3072) MM_QCOLS(3);
    else MM_QCOLS(4);
#undef MM_QCOLS
    return check_launch("quant_cols_reg_kernel");
  }
  if (!amax_clear) {
    const unsigned fg = (unsigned)std::min<int64_t>((Nc + 255) / 256, 1024);
    hipLaunchKernelGGL(fp8::fill_u32_kernel, dim3(fg), dim3(256), 0, s, amax, Nc);
    if (gemm_status st = check_launch("fill_u32_kernel")) return st;
  }
  const bool vec = ld % 4 == 0 && ((uintptr_t)P & 15) == 0;
  const dim3 ag((unsigned)((Nc + 63) / 64), (unsigned)std::max<int64_t>(1, (K + 255) / 256));
  if (vec)
    hipLaunchKernelGGL(fp8::col_amax4_kernel<true>, ag, dim3(256), 0, s, (int)K, (int)Nc, P, ld, amax);
  else
    hipLaunchKernelGGL(fp8::col_amax4_kernel<false>, ag, dim3(256), 0, s, (int)K, (int)Nc, P, ld, amax);
  if (gemm_status st = check_launch("col_amax4_kernel")) return st;
  hipLaunchKernelGGL(fp8::quant_cols_t_kernel, dim3((unsigned)(Kp / 64), (unsigned)((Nc + 63) / 64)),
                     dim3(256), 0, s, (int)K, (int)Nc, Kp, P, ld, amax, q, scales);
  return check_launch("quant_cols_t_kernel");
}

// op(A) (M x K) by rows and op(B) (K x N) by columns.  A row of op(A) is a
// row of A, or a column of A^T as stored (ta); a column of op(B) is a column
// of B, or a row of B^T as stored (tb).
gemm_status fp8_quantize_run(int64_t M, int64_t N, int64_t K, const float *A, int64_t lda,
                             const float *B, int64_t ldb, void *ws, hipStream_t s, bool ta,
                             bool tb) {
  const fp8::Layout L = fp8::layout(M, N, K);
  uint8_t *base = static_cast<uint8_t *>(ws);
  uint8_t *qa = base + L.qa;
  uint8_t *qb = base + L.qb;
  float *sa = reinterpret_cast<float *>(base + L.sa);
  float *sb = reinterpret_cast<float *>(base + L.sb);
  uint32_t *amax = reinterpret_cast<uint32_t *>(base + L.amax);
  // When A goes by rows and B by columns, A's launch clears B's amax words.
  bool amax_clear = false;
  if (M > 0) {
    gemm_status st = ta ? quant_cols(K, M, L.Kp, A, lda, amax, qa, sa, s)
                        : quant_rows(M, K, L.Kp, A, lda, qa, sa, s, (N > 0 && !tb) ? amax : nullptr,
                                     N, &amax_clear);
    if (st) return st;
  }
  if (N > 0) {
    gemm_status st = tb ? quant_rows(N, K, L.Kp, B, ldb, qb, sb, s)
                        : quant_cols(K, N, L.Kp, B, ldb, amax, qb, sb, s, amax_clear);
    if (st) return st;
  }
  return GEMM_STATUS_OK;
}

template <int BM, int BN, int WM, int WN, bool DMA>
static gemm_status fp8_launch(int64_t M, int64_t N, const fp8::Layout &L, float alpha,
                              const uint8_t *base, float beta, float *C, int64_t ldc,
                              hipStream_t s) {
  if ((int64_t)(BM > BN ? BM : BN) * L.Kp >= ((int64_t)1 << 31)) {
    set_error("gemm_fp8: K too large for 32-bit tile offsets");
    return GEMM_STATUS_UNSUPPORTED;
  }
  const int tiles_m = (int)((M + BM - 1) / BM), tiles_n = (int)((N + BN - 1) / BN);
  const dim3 grid((unsigned)((int64_t)tiles_m * tiles_n)), block(64 * (BM / WM) * (BN / WN));
  const uint8_t *qa = base + L.qa, *qb = base + L.qb;
  const float *sa = reinterpret_cast<const float *>(base + L.sa);
  const float *sb = reinterpret_cast<const float *>(base + L.sb);
  if (DMA) {
    if (beta != 0.0f)
      hipLaunchKernelGGL((fp8::gemm_fp8_dma_kernel<BM, BN, WM, WN, true>), grid, block, 0, s,
                         (int)M, (int)N, L.Kp, alpha, qa, qb, sa, sb, beta, C, ldc, tiles_m, tiles_n);
    else
      hipLaunchKernelGGL((fp8::gemm_fp8_dma_kernel<BM, BN, WM, WN, false>), grid, block, 0, s,
                         (int)M, (int)N, L.Kp, alpha, qa, qb, sa, sb, beta, C, ldc, tiles_m, tiles_n);
    return check_launch("gemm_fp8_dma_kernel");
  }
  if (beta != 0.0f)
    hipLaunchKernelGGL((fp8::gemm_fp8_kernel<BM, BN, WM, WN, true>), grid, block, 0, s, (int)M,
                       (int)N, L.Kp, alpha, qa, qb, sa, sb, beta, C, ldc, tiles_m, tiles_n);
  else
    hipLaunchKernelGGL((fp8::gemm_fp8_kernel<BM, BN, WM, WN, false>), grid, block, 0, s, (int)M,
                       (int)N, L.Kp, alpha, qa, qb, sa, sb, beta, C, ldc, tiles_m, tiles_n);
  return check_launch("gemm_fp8_kernel");
}

template <int BM, int BN, int WM, int WN>
static gemm_status fp8_launch_ring(int64_t M, int64_t N, const fp8::Layout &L, float alpha,
                                   const uint8_t *base, float beta, float *C, int64_t ldc,
                                   hipStream_t s) {
  if ((int64_t)(BM > BN ? BM : BN) * L.Kp >= ((int64_t)1 << 31)) {
    set_error("gemm_fp8: K too large for 32-bit tile offsets");
    return GEMM_STATUS_UNSUPPORTED;
  }
  const int tiles_m = (int)((M + BM - 1) / BM), tiles_n = (int)((N + BN - 1) / BN);
  const dim3 grid((unsigned)((int64_t)tiles_m * tiles_n)), block(64 * (BM / WM) * (BN / WN));
  const uint8_t *qa = base + L.qa, *qb = base + L.qb;
  const float *sa = reinterpret_cast<const float *>(base + L.sa);
  const float *sb = reinterpret_cast<const float *>(base + L.sb);
  if (beta != 0.0f)
    hipLaunchKernelGGL((fp8::gemm_fp8_ring_kernel<BM, BN, WM, WN, true>), grid, block, 0, s,
                       (int)M, (int)N, L.Kp, alpha, qa, qb, sa, sb, beta, C, ldc, tiles_m, tiles_n);
  else
    hipLaunchKernelGGL((fp8::gemm_fp8_ring_kernel<BM, BN, WM, WN, false>), grid, block, 0, s,
                       (int)M, (int)N, L.Kp, alpha, qa, qb, sa, sb, beta, C, ldc, tiles_m, tiles_n);
  return check_launch("gemm_fp8_ring_kernel");
}

int fp8_num_configs() { return 7; }
const char *fp8_config_name(int cfg) {
  switch (cfg) {
    case 0: return "fp8_256x256x128_8w128x64";
    case 1: return "fp8_256x256x128_4w128x128";
    case 3: return "fp8_128x128x128_4w64x64_dma";
    case 4: return "fp8_256x128x128_8w64x64_dma";
    case 5: return "fp8_256x256x128_4w128x128_dma";
    case 6: return "fp8_256x256x64_8w128x64_dma_ring4";
    default: return "fp8_256x256x128_8w128x64_dma";
  }
}

gemm_status fp8_gemm_run_cfg(int64_t M, int64_t N, int64_t K, float alpha, const void *ws,
                             float beta, float *C, int64_t ldc, int cfg, hipStream_t s) {
  const fp8::Layout L = fp8::layout(M, N, K);
  const uint8_t *base = static_cast<const uint8_t *>(ws);
  if (cfg == 1) return fp8_launch<256, 256, 128, 128, false>(M, N, L, alpha, base, beta, C, ldc, s);
  if (cfg == 2) return fp8_launch<256, 256, 128, 64, true>(M, N, L, alpha, base, beta, C, ldc, s);
  if (cfg == 3) return fp8_launch<128, 128, 64, 64, true>(M, N, L, alpha, base, beta, C, ldc, s);
  if (cfg == 4) return fp8_launch<256, 128, 64, 64, true>(M, N, L, alpha, base, beta, C, ldc, s);
  if (cfg == 5) return fp8_launch<256, 256, 128, 128, true>(M, N, L, alpha, base, beta, C, ldc, s);
  if (cfg == 6) return fp8_launch_ring<256, 256, 128, 64>(M, N, L, alpha, base, beta, C, ldc, s);
  return fp8_launch<256, 256, 128, 64, false>(M, N, L, alpha, base, beta, C, ldc, s);
}

// Direct-to-LDS kernels: 256 x 256 tiles while they fill every compute unit
// (measured best at 4096^3 and above), 128 x 128 tiles -- two workgroups per
// compute unit -- below that (1.9x at 2048^3 and at 1024 x 4096 x 4096).
int fp8_default_config(int64_t M, int64_t N, int64_t) {
  const int64_t big = ((M + 255) / 256) * ((N + 255) / 256);
  return big >= num_cus() ? 2 : 3;
}

gemm_status fp8_encode_run(int64_t n, const float *x, uint8_t *out, hipStream_t s) {
  const int64_t want = (n + 255) / 256;
  const unsigned grid = (unsigned)(want < 8192 ? (want > 0 ? want : 1) : 8192);
  hipLaunchKernelGGL(fp8::encode_kernel, dim3(grid), dim3(256), 0, s, n, x, out);
  return check_launch("encode_kernel");
}

}  // namespace mm
