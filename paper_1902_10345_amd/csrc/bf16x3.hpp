// bf16x3.hpp -- tile body of the split-precision bf16 MFMA GEMM (gfx950).
//
// FP32-accurate C <- alpha*A*B + beta*C from bfloat16 matrix-core products.
// Every binary32 element is split while its slab is staged into LDS,
//   x = x0 + x1 (+ x2),  x0 = rne(x), x1 = rne(x - x0), x2 = rne(x - x0 - x1),
// and the kernel accumulates, in binary32 on v_mfma_f32_32x32x16_bf16,
//   NP == 2 (3 products): a0*b0 + a0*b1 + a1*b0
//   NP == 3 (6 products): the above + a0*b2 + a1*b1 + a2*b0.
//
// Structure (the paper's MM transformation chain, Sec. 6.2, on CDNA4):
//   MapTiling       BM x BN workgroup tile over (i, j); 2 x 2 waves, each a
//                   WM x WN wave tile of 32 x 32 MFMA blocks; K in BK slabs.
//   LocalStorage    A slab as [plane][BM][BK] and B slab transposed as
//   DoubleBuffering [plane][BN][BK] bf16 in LDS, two stages, plus two register
//                   sets for the global loads: while slab t is multiplied,
//                   slab t+2 is in flight from HBM and slab t+1 is split and
//                   written to the other LDS stage.
//   Vectorization   128-bit global loads of A rows, 128-bit LDS writes and
//                   ds_read_b128 fragment reads.
//   ReducePeeling   alpha/beta applied once in the epilogue.
// LDS rows are BK bf16 (BK*2 bytes) with an XOR swizzle of the 16-byte chunk
// index, so that 16 consecutive rows read or written at one logical chunk
// fall in distinct banks (for both 32- and 64-bank LDS organisations).
#pragma once

#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"

namespace mm {
namespace bx3 {

typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Word 3 of a raw buffer resource on gfx9-class GPUs: 32-bit data format,
// no swizzle; the hardware range check returns zero for reads past
// num_records.
constexpr int kBufferFlags = 0x00020000;

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// Round-to-nearest-even split of binary32 values into bfloat16 planes, two
// values at a time: v_cvt_pk_bf16_f32 rounds a pair in one instruction, and
// widening a bfloat16 back to binary32 is exact, so x - h is the exact
// remainder.
__device__ __forceinline__ void split2(f32x2 x, bf16x2 &h, bf16x2 &l) {
  h = __builtin_convertvector(x, bf16x2);
  l = __builtin_convertvector(x - __builtin_convertvector(h, f32x2), bf16x2);
}
__device__ __forceinline__ void split3(f32x2 x, bf16x2 &h, bf16x2 &m, bf16x2 &l) {
  h = __builtin_convertvector(x, bf16x2);
  const f32x2 r = x - __builtin_convertvector(h, f32x2);
  m = __builtin_convertvector(r, bf16x2);
  l = __builtin_convertvector(r - __builtin_convertvector(m, f32x2), bf16x2);
}

// f(std::integral_constant<int, i>{}) for i = 0 .. N-1, unrolled at compile
// time (every index is a constant expression inside f).
template <int N, int I = 0, typename F>
__device__ __forceinline__ void static_for(F &&f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<N, I + 1>(f);
  }
}

// XOR swizzle of the 16-byte chunk index of an LDS row holding BK bf16.
template <int BK>
__device__ __forceinline__ int swz(int r) {
  // 64-byte rows: measured on gfx950 with SQ_LDS_BANK_CONFLICT, this form is
  // conflict-free for the fragment reads, the row-major A stores and the
  // transposed B stores; ((r >> 1) ^ (r >> 3)) & 3 conflicts on the reads
  if constexpr (BK == 32) return (r ^ (r >> 2)) & 3;
  else if constexpr (BK == 16) return ((r >> 2) ^ (r >> 3)) & 1;
  else return 0;
}

template <int BM, int BN, int BK, int WM, int WN, int NP, int NW, int ST = 2, int SETS_ = 0>
struct Cfg {
  static constexpr int NT = 64 * NW;          // lanes per workgroup
  static constexpr int WAVES_M = BM / WM;
  static constexpr int WAVES_N = BN / WN;
  static_assert(WAVES_M * WAVES_N == NW, "wave grid must cover the tile");
  static constexpr int FM = WM / 32;          // 32x32 blocks per wave along M
  static constexpr int FN = WN / 32;
  static constexpr int CH = BK / 8;           // 8-element staging items per row
  // LDS row length in bf16 units: BK bf16 per plane, or BK binary32 values
  // (twice the bytes) in the FP32 mode (NP == 1)
  static constexpr int ROW = NP == 1 ? 2 * BK : BK;
  static constexpr int NPL = NP == 1 ? 2 : NP;  // bf16-plane sizes per operand
  // MFMA k-steps per slab: 16 k (bf16 planes) or 8 k (FP32 mode: two 4-k
  // chunks per lane pair, each feeding four 32x32x2 MFMAs)
  static constexpr int KS = NP == 1 ? BK / 8 : BK / 16;
  static constexpr int PLANE_A = BM * BK;     // bf16 elements per A plane
  static constexpr int PLANE_B = BN * BK;
  static constexpr int STAGE = NPL * (PLANE_A + PLANE_B);  // bf16 units per stage
  static constexpr int STAGES = ST;           // LDS stages (2, or a ring of 3)
  static constexpr int LDS_BYTES = ST * STAGE * 2;
  // Register sets for slabs in flight: with BK >= 32 one slab's MFMA work
  // (2 k-steps) already covers the load latency, so one set is kept and the
  // registers go to fragments; BK = 16 keeps two sets.
  static constexpr int SETS = SETS_ ? SETS_ : (BK >= 32 ? 1 : 2);
};

// Staging of one operand slab into LDS: ROWS LDS rows (the rows of A's tile
// or the columns of B's tile), each BK deep in k, moved as items of 8
// consecutive k per lane.
//   KC (k contiguous in memory: row-major A, transposed B): item idx covers
//      LDS row idx / CH, chunk idx % CH; two 128-bit loads when V (row stride
//      a multiple of 4 floats, 16-byte aligned base), else eight 32-bit loads.
//   otherwise (the row index contiguous: row-major B, transposed A): item idx
//      covers LDS row idx % ROWS, chunk idx / ROWS; eight 32-bit loads, one
//      per k, with the lanes of a wave consecutive along the row index.
// Either way the LDS layout is the same ([plane][ROWS][BK], swizzled chunks),
// so the fragment reads and the MFMAs do not depend on the memory layout.
template <int ROWS, int BK, int NT, int SETS, bool KC, bool V>
struct Stage {
  static constexpr int CH = BK / 8;
  static constexpr int ITEMS = ROWS * CH / NT;
  static_assert(ITEMS * NT == ROWS * CH, "even split of the slab over the lanes");
  static_assert(KC || ROWS % 64 == 0 || NT % ROWS == 0, "chunk index must be wave-uniform");
  // global loads per slab and lane
  static constexpr int LOADS = ITEMS * ((KC && V) ? 2 : 8);
  __device__ static __forceinline__ int row_of(int idx) { return KC ? idx / CH : idx % ROWS; }
  __device__ static __forceinline__ int chunk_of(int idx) { return KC ? idx % CH : idx / ROWS; }

  float r[SETS][ITEMS][8];
  // KC: byte offset of the item's (row, chunk) inside the tile's panel at k 0.
  // Otherwise: byte offset of the item's row index inside a k row (rows past
  // the matrix get an offset beyond any slab resource, so they read as zero).
  int voff[ITEMS];
  int soff[ITEMS];  // otherwise: wave-uniform byte offset of the item's first k row
  __amdgpu_buffer_rsrc_t rsrc;  // KC: the tile's panel
  const float *P;
  int64_t ld;
  int r0, nrows, K;
  int tl;  // the lane's index among the threads that share this staging

  // P: the operand as stored; ld: its row stride; r0: the tile's first LDS
  // row (output row of A / column of B); total: rows (KC) or row-index extent.
  __device__ __forceinline__ void init(const float *P_, int64_t ld_, int r0_, int total, int K_,
                                       int tid) {
    P = P_; ld = ld_; r0 = r0_; K = K_; tl = tid;
    nrows = total - r0 < ROWS ? total - r0 : ROWS;
    if constexpr (KC) {
      // valid bytes end with the last valid row's K elements: reads past the
      // matrix (rows beyond it, k beyond K of the last row) return zero
      rsrc = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<float *>(P + (int64_t)r0 * ld), (short)0,
          nrows > 0 ? (int)(((int64_t)(nrows - 1) * ld + K) * 4) : 0, kBufferFlags);
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        const int idx = tid + NT * i;
        voff[i] = (row_of(idx) * (int)ld + chunk_of(idx) * 8) * 4;
      }
    } else {
      const int ld4 = (int)ld * 4;
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        const int idx = tid + NT * i;
        const int n = row_of(idx);
        voff[i] = n < nrows ? n * 4 : (int)0x80000000;
        soff[i] = __builtin_amdgcn_readfirstlane(8 * chunk_of(idx)) * ld4;
      }
    }
  }

  // Item i of a full slab (every k of the slab in [0, K)), on its own: the
  // pieces a software-pipelined loop places between its MFMAs.
  template <int SET>
  __device__ __forceinline__ void load_item(int i, int k0) {
    if constexpr (KC) {
      const int off = voff[i] + k0 * 4;
      if constexpr (V) {
        const float4 v0 =
            __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rsrc, off, 0, 0));
        const float4 v1 =
            __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rsrc, off + 16, 0, 0));
        r[SET][i][0] = v0.x; r[SET][i][1] = v0.y; r[SET][i][2] = v0.z; r[SET][i][3] = v0.w;
        r[SET][i][4] = v1.x; r[SET][i][5] = v1.y; r[SET][i][6] = v1.z; r[SET][i][7] = v1.w;
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e)
          r[SET][i][e] = __builtin_bit_cast(
              float, __builtin_amdgcn_raw_buffer_load_b32(rsrc, off + 4 * e, 0, 0));
      }
    } else {
      const int ld4 = (int)ld * 4;
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<float *>(P + (int64_t)(k0 > 0 ? k0 : 0) * ld + r0), (short)0,
          k0 >= 0 ? (int)(((int64_t)(BK - 1) * ld + nrows) * 4) : 0, kBufferFlags);
#pragma unroll
      for (int e = 0; e < 8; ++e)
        r[SET][i][e] = __builtin_bit_cast(
            float, __builtin_amdgcn_raw_buffer_load_b32(rs, voff[i], soff[i] + e * ld4, 0));
    }
  }

  // FAST: every k of the slab lies in [0, K) (or the data is never consumed).
  // Otherwise k outside [0, K) read as zero.
  template <int SET, bool FAST>
  __device__ __forceinline__ void load(int k0) {
    if constexpr (KC) {
      if constexpr (FAST) {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
          const int off = voff[i] + k0 * 4;
          if constexpr (V) {
            // (bit-cast whole vectors: a bit_cast of a vector element is not
            // element-indexed in this compiler)
            const float4 v0 =
                __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rsrc, off, 0, 0));
            const float4 v1 =
                __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rsrc, off + 16, 0, 0));
            r[SET][i][0] = v0.x; r[SET][i][1] = v0.y; r[SET][i][2] = v0.z; r[SET][i][3] = v0.w;
            r[SET][i][4] = v1.x; r[SET][i][5] = v1.y; r[SET][i][6] = v1.z; r[SET][i][7] = v1.w;
          } else {
#pragma unroll
            for (int e = 0; e < 8; ++e)
              r[SET][i][e] = __builtin_bit_cast(
                  float, __builtin_amdgcn_raw_buffer_load_b32(rsrc, off + 4 * e, 0, 0));
          }
        }
      } else {  // partial slab: per-element offsets, invalid ones pushed out of range
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
          const int k = k0 + chunk_of(tl + NT * i) * 8;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const int off = (k + e >= 0 && k + e < K) ? voff[i] + (k0 + e) * 4 : (int)0x80000000;
            r[SET][i][e] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rsrc, off, 0, 0));
          }
        }
      }
    } else {
      const int ld4 = (int)ld * 4;
      if constexpr (FAST) {
        // one resource for the whole slab; per-lane offsets select the rows
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<float *>(P + (int64_t)(k0 > 0 ? k0 : 0) * ld + r0), (short)0,
            k0 >= 0 ? (int)(((int64_t)(BK - 1) * ld + nrows) * 4) : 0, kBufferFlags);
#pragma unroll
        for (int i = 0; i < ITEMS; ++i)
#pragma unroll
          for (int e = 0; e < 8; ++e)
            r[SET][i][e] = __builtin_bit_cast(
                float, __builtin_amdgcn_raw_buffer_load_b32(rs, voff[i], soff[i] + e * ld4, 0));
      } else {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
          const int idx = tl + NT * i;
          const int n = row_of(idx);
          const int c = __builtin_amdgcn_readfirstlane(chunk_of(idx));  // wave-uniform
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            // one resource per k row: rows outside [0, K) have no valid bytes,
            // row indices at or past the extent fall beyond the row's valid bytes
            const int k = k0 + 8 * c + e;
            const bool kin = k >= 0 && k < K;
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<float *>(P + (int64_t)(kin ? k : 0) * ld + r0), (short)0,
                kin ? nrows * 4 : 0, kBufferFlags);
            r[SET][i][e] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, n * 4, 0, 0));
          }
        }
      }
    }
  }
};

// One output tile.  lds must hold Cfg::LDS_BYTES bytes (16-byte aligned).
// TA / TB: A / B are given transposed (A stored K x M with row stride lda,
// B stored N x K with row stride ldb); op(A) op(B) is computed either way.
// VEC: every operand stored with k contiguous (A unless TA, B if TB) has a
// row stride that is a multiple of 4 floats and a 16-byte aligned base
// (128-bit loads), and K % 4 == 0.
// Interior slabs (tile fully inside M x N and a whole BK slab of K) take an
// unpredicated load path; edge slabs take a guarded path that reads zeros
// outside the matrices.  The choice is uniform across the workgroup.
template <int BM, int BN, int BK, int WM, int WN, int NP, int NW, bool VEC, bool BETA,
          bool TA = false, bool TB = false, int ST = 2, int SETS_ = 0, int KG = 1>
__device__ __forceinline__ void tile(int M, int N, int K, float alpha,
                                     const float *__restrict__ A, int64_t lda,
                                     const float *__restrict__ B, int64_t ldb, float beta,
                                     float *__restrict__ C, int64_t ldc, int m0, int n0,
                                     __bf16 *lds) {
  using G = Cfg<BM, BN, BK, WM, WN, NP, NW, ST, SETS_>;
  static_assert(ST == 2 || (ST == 3 && NP == 2 && BK == 16),
                "the three-stage ring is built for 16-deep slabs of three products");
  constexpr int NT = G::NT;
  // KG > 1: the workgroup holds KG groups of NW waves; group g multiplies the
  // g-th of KG equal k ranges (the caller guarantees K % KG == 0) into the
  // same output tile with its own LDS stages (lds + g * LDS_BYTES), and the
  // partial tiles are summed in group order before the epilogue.
  static_assert(KG == 1 || (KG == 2 && !TA && !TB && ST == 2),
                "k-groups: two groups, operands not transposed, two LDS stages");
  const int grp = KG > 1 ? __builtin_amdgcn_readfirstlane((int)threadIdx.x / NT) : 0;
  const int tid = (int)threadIdx.x - grp * NT;
  if constexpr (KG > 1) {
    K /= KG;
    A += (int64_t)grp * K;
    B += (int64_t)grp * K * ldb;
    lds += grp * (G::LDS_BYTES / 2);
  }
  const int lane = tid & 63, wave = tid >> 6;
  const int Mr = M - m0, Nr = N - n0;
  const bool interior = Mr >= BM && Nr >= BN;
  // Staging loads are raw buffer loads: the resource holds the tile's base
  // address and the number of valid bytes, so reads past the matrix return
  // zero in hardware and lane addresses stay 32-bit offsets (no 64-bit VALU
  // address arithmetic).  The launcher guarantees that every panel's and
  // slab's byte extent stays below 2^31.
  using SA = Stage<BM, BK, NT, G::SETS, !TA, VEC && !TA>;
  using SB = Stage<BN, BK, NT, G::SETS, TB, VEC && TB>;
  SA sa;
  SB sb;
  sa.init(A, lda, m0, M, K, tid);
  sb.init(B, ldb, n0, N, K, tid);

  // ---- global -> registers (register sets selected at compile time) --------
  auto gload = [&](auto S, auto F, int k0) {
    constexpr int set = decltype(S)::value;
    constexpr bool FAST = decltype(F)::value;
    sa.template load<set, FAST>(k0);
    sb.template load<set, FAST>(k0);
  };

  // ---- split + registers -> LDS --------------------------------------------
  auto split8 = [&](const float (&x)[8], bf16x8 &h, bf16x8 &m, bf16x8 &l) {
#pragma unroll
    for (int e = 0; e < 8; e += 2) {
      bf16x2 x0, x1, x2;
      if constexpr (NP == 2) split2(f32x2{x[e], x[e + 1]}, x0, x1);
      else split3(f32x2{x[e], x[e + 1]}, x0, x1, x2);
      h[e] = x0.x; h[e + 1] = x0.y;
      m[e] = x1.x; m[e + 1] = x1.y;
      if constexpr (NP == 3) { l[e] = x2.x; l[e + 1] = x2.y; }
    }
  };
  // One operand's items into its LDS planes (row-major [plane][ROWS][ROW]).
  auto store_op = [&](auto &op, auto S, __bf16 *base, auto PL) {
    using Op = std::remove_reference_t<decltype(op)>;
    constexpr int set = decltype(S)::value;
    constexpr int PLANE = decltype(PL)::value;
#pragma unroll
    for (int i = 0; i < Op::ITEMS; ++i) {
      const int idx = tid + NT * i;
      const int r = Op::row_of(idx), c = Op::chunk_of(idx);
      const float *x = op.r[set][i];
      if constexpr (NP == 1) {  // FP32 mode: the item's 8 values as two 16-byte chunks
        *reinterpret_cast<f32x4 *>(base + r * G::ROW + (((2 * c) ^ swz<G::ROW>(r)) << 3)) =
            f32x4{x[0], x[1], x[2], x[3]};
        *reinterpret_cast<f32x4 *>(base + r * G::ROW + (((2 * c + 1) ^ swz<G::ROW>(r)) << 3)) =
            f32x4{x[4], x[5], x[6], x[7]};
      } else {
        bf16x8 h, m, l;
        split8(op.r[set][i], h, m, l);
        const int off = r * BK + ((c ^ swz<BK>(r)) << 3);
        *reinterpret_cast<bf16x8 *>(base + off) = h;
        *reinterpret_cast<bf16x8 *>(base + PLANE + off) = m;
        if constexpr (NP == 3) *reinterpret_cast<bf16x8 *>(base + 2 * PLANE + off) = l;
      }
    }
  };
  auto sstore = [&](auto S, int stage) {
    __bf16 *sA = lds + stage * G::STAGE;
    __bf16 *sB = sA + G::NPL * G::PLANE_A;
    store_op(sa, S, sA, std::integral_constant<int, G::PLANE_A>{});
    store_op(sb, S, sB, std::integral_constant<int, G::PLANE_B>{});
  };

  // ---- MFMA over one slab ------------------------------------------------
  const int wm0 = (wave / G::WAVES_N) * WM;
  const int wn0 = (wave % G::WAVES_N) * WN;
  const int lrow = lane & 31, lgrp = lane >> 5;
  f32x16 acc[G::FM][G::FN];
#pragma unroll
  for (int i = 0; i < G::FM; ++i)
#pragma unroll
    for (int j = 0; j < G::FN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;

  // Fragments of one 16-deep k-step: the lane's 8 consecutive k of its A row
  // (per block i and plane p) and of its B column (per block j and plane p).
  using FragT = std::conditional_t<NP == 1, f32x4, bf16x8>;
  struct Frags {
    FragT a[NP][G::FM], b[NP][G::FN];
  };
  // Reads in the order the products consume them (b0 and a1 first).
  auto frag_read = [&](Frags &f, int stage, int ks) {
    const __bf16 *sA = lds + stage * G::STAGE;
    const __bf16 *sB = sA + G::NPL * G::PLANE_A;
    const int c = ks * 2 + lgrp;  // logical 16-byte chunk of this lane
    if constexpr (NP == 1) {  // FP32 mode: 4 consecutive k per lane and block
#pragma unroll
      for (int j = 0; j < G::FN; ++j) {
        const int n = wn0 + j * 32 + lrow;
        f.b[0][j] = *reinterpret_cast<const f32x4 *>(sB + n * G::ROW + ((c ^ swz<G::ROW>(n)) << 3));
      }
#pragma unroll
      for (int i = 0; i < G::FM; ++i) {
        const int r = wm0 + i * 32 + lrow;
        f.a[0][i] = *reinterpret_cast<const f32x4 *>(sA + r * G::ROW + ((c ^ swz<G::ROW>(r)) << 3));
      }
    } else {
      auto rd_b = [&](int p) {
#pragma unroll
        for (int j = 0; j < G::FN; ++j) {
          const int n = wn0 + j * 32 + lrow;
          f.b[p][j] = *reinterpret_cast<const bf16x8 *>(sB + p * G::PLANE_B + n * BK +
                                                        ((c ^ swz<BK>(n)) << 3));
        }
      };
      auto rd_a = [&](int p) {
#pragma unroll
        for (int i = 0; i < G::FM; ++i) {
          const int r = wm0 + i * 32 + lrow;
          f.a[p][i] = *reinterpret_cast<const bf16x8 *>(sA + p * G::PLANE_A + r * BK +
                                                        ((c ^ swz<BK>(r)) << 3));
        }
      };
      rd_b(0);
      if constexpr (NP == 3) rd_a(2);
      rd_a(1);
      rd_b(1);
      if constexpr (NP == 3) rd_b(2);
      rd_a(0);
    }
  };
  // Small products first, the leading product last; consecutive MFMAs go to
  // different accumulator blocks.
  auto frag_mfma = [&](const Frags &f) {
    if constexpr (NP == 1) {
      // MFMA q sums k = 4c + q of the lower half-wave's chunk and of the
      // upper half-wave's chunk: every k of the two chunks exactly once
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int i = 0; i < G::FM; ++i)
#pragma unroll
          for (int j = 0; j < G::FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(f.a[0][i][q], f.b[0][j][q], acc[i][j],
                                                             0, 0, 0);
    } else {
      auto prod = [&](int pa, int pb) {
#pragma unroll
        for (int i = 0; i < G::FM; ++i)
#pragma unroll
          for (int j = 0; j < G::FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[pa][i], f.b[pb][j], acc[i][j],
                                                                0, 0, 0);
      };
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
  // All MFMAs of one LDS stage.  With one k-step per stage every fragment
  // read is issued before the first MFMA (a scheduling barrier stops the
  // compiler from re-reading fragments in small groups, each waiting out the
  // LDS latency).  With two k-steps the registers do not allow both steps'
  // fragments at once; each step reads, then multiplies, and the compiler
  // overlaps the second step's reads with the first step's MFMAs.
  auto mfma_stage = [&](int stage) {
    if constexpr (G::KS == 1) {
      Frags f0;
      frag_read(f0, stage, 0);
      __builtin_amdgcn_sched_barrier(0);
      frag_mfma(f0);
    } else {
#pragma unroll
      for (int ks = 0; ks < G::KS; ++ks) {
        Frags f;
        frag_read(f, stage, ks);
        frag_mfma(f);
      }
    }
  };

  // ---- K loop ---------------------------------------------------------------
  // Two register sets (BK = 16): slab t is multiplied from LDS stage t%2 while
  // (a) the global loads of slab t+2 are in flight into one register set and
  // (b) slab t+1, loaded during slab t-1 into the other set, is split and
  // written to stage (t+1)%2.  One register set (BK >= 32): slab t+1 is
  // loaded at the top of slab t's step and split and written at its end.
  // Either way the loads are issued ahead of the MFMAs (a scheduling barrier
  // keeps the compiler from sinking them) and one barrier per slab separates
  // the LDS stages.
  // The slab grid ends exactly at K (slab s covers [kbase + s*BK, +BK) with
  // kbase = K - KT*BK <= 0), so only slab 0 can be partial; it is loaded with
  // masking in the prologue when it is.  Loads past the last slab are clamped to it
  // (in-bounds reads whose data is never consumed), so both halves of the loop
  // issue the same instructions on every iteration and each wait covers only
  // the loads it needs.
  using S0 = std::integral_constant<int, 0>;
  using S1 = std::integral_constant<int, 1>;
  // one wave per SIMD with 128 x 128 wave tiles: the deeply pipelined loop
  constexpr bool kDeep = NP >= 2 && NW == 4 && WM == 128 && WN == 128 && BK == 16;
  using Fast = std::true_type;
  using Masked = std::false_type;
  const int KT = (K + BK - 1) / BK;
  const int kbase = K - KT * BK;
  auto kslab = [&](int sl) { return kbase + (sl < KT ? sl : KT - 1) * BK; };
  // slab 0 is partial unless K is a multiple of BK (then kbase == 0)
  if (kbase == 0) gload(S0{}, Fast{}, 0);
  else gload(S0{}, Masked{}, kbase);
  sstore(S0{}, 0);
  int t = 0;
  if constexpr (G::SETS == 1) {
    // One register set: slab t+1 is loaded at the top of the step that
    // multiplies slab t and written to the other stage at its end.
    __syncthreads();
    for (; t + 2 <= KT; t += 2) {
      gload(S0{}, Fast{}, kslab(t + 1));
      __builtin_amdgcn_sched_barrier(0);
      mfma_stage(0);
      sstore(S0{}, 1);
      __syncthreads();
      gload(S0{}, Fast{}, kslab(t + 2));
      __builtin_amdgcn_sched_barrier(0);
      mfma_stage(1);
      sstore(S0{}, 0);
      __syncthreads();
    }
  } else if constexpr (ST == 3) {
    // Three LDS stages in a ring, two register sets, one 16-deep k-step per
    // slab.  Step s multiplies slab s from stage s%3.  The fragments of its
    // first product (a1 * b0) were read during step s-1, so its MFMAs issue
    // right after the barrier while the reads of a0 and b1 are in flight.
    // In the same step slab s+2 (loaded from global memory in step s-1, in
    // register set s%2) is split and written to stage (s+2)%3, the loads of
    // slab s+3 go to the other set, and the first-product fragments of slab
    // s+1 are read from stage (s+1)%3 into the other fragment set.  One
    // barrier per step: it orders the writes of slab s+2 before their first
    // reads (step s+1) and the last reads of stage s%3 (this step) before it
    // is rewritten with slab s+3 (step s+1).
    using Fr = Frags;
    using First = std::true_type;
    using Rest = std::false_type;
    auto rd = [&](Fr &f, int stage, auto FIRST) {
      const __bf16 *sA = lds + stage * G::STAGE;
      const __bf16 *sB = sA + G::NPL * G::PLANE_A;
      const int c = lgrp;
      constexpr int pa = decltype(FIRST)::value ? 1 : 0, pb = decltype(FIRST)::value ? 0 : 1;
#pragma unroll
      for (int j = 0; j < G::FN; ++j) {
        const int n = wn0 + j * 32 + lrow;
        f.b[pb][j] = *reinterpret_cast<const bf16x8 *>(sB + pb * G::PLANE_B + n * BK +
                                                       ((c ^ swz<BK>(n)) << 3));
      }
#pragma unroll
      for (int i = 0; i < G::FM; ++i) {
        const int r = wm0 + i * 32 + lrow;
        f.a[pa][i] = *reinterpret_cast<const bf16x8 *>(sA + pa * G::PLANE_A + r * BK +
                                                       ((c ^ swz<BK>(r)) << 3));
      }
    };
    auto prod = [&](const Fr &f, int pa, int pb) {
#pragma unroll
      for (int i = 0; i < G::FM; ++i)
#pragma unroll
        for (int j = 0; j < G::FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[pa][i], f.b[pb][j], acc[i][j],
                                                              0, 0, 0);
    };
    // One fragment of a set: idx < FN the B block idx, else the A block
    // idx - FN, of the planes of the first product (a1, b0) or of the rest
    // (a0, b1).
    auto rd_one = [&](Fr &f, int stage, auto FIRST, auto IDX) {
      constexpr int idx = decltype(IDX)::value;
      constexpr int pa = decltype(FIRST)::value ? 1 : 0, pb = decltype(FIRST)::value ? 0 : 1;
      const __bf16 *sA = lds + stage * G::STAGE;
      const __bf16 *sB = sA + G::NPL * G::PLANE_A;
      const int c = lgrp;
      if constexpr (idx < G::FN) {
        const int n = wn0 + idx * 32 + lrow;
        f.b[pb][idx] = *reinterpret_cast<const bf16x8 *>(sB + pb * G::PLANE_B + n * BK +
                                                         ((c ^ swz<BK>(n)) << 3));
      } else {
        const int r = wm0 + (idx - G::FN) * 32 + lrow;
        f.a[pa][idx - G::FN] = *reinterpret_cast<const bf16x8 *>(sA + pa * G::PLANE_A + r * BK +
                                                                 ((c ^ swz<BK>(r)) << 3));
      }
    };
    constexpr int kBlk = G::FM * G::FN;
    constexpr int kMfma = 3 * kBlk;               // a1*b0, a0*b1, a0*b0
    constexpr int kHalf = G::FM + G::FN;          // fragments per plane pair
    constexpr int kItems = SA::ITEMS + SB::ITEMS;
    static_assert(kHalf <= 2 * kBlk && 4 * kItems <= kBlk, "the step's work fits its MFMA slots");
    // MFMA q of a step: product q / kBlk, block q % kBlk
    auto mfma_one = [&](const Fr &f, auto Q) {
      constexpr int q = decltype(Q)::value;
      constexpr int pr = q / kBlk, bi = (q % kBlk) / G::FN, bj = q % G::FN;
      constexpr int pa = pr == 0 ? 1 : 0, pb = pr == 1 ? 1 : 0;
      acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[pa][bi], f.b[pb][bj], acc[bi][bj],
                                                            0, 0, 0);
    };
    // split of value pair E of item IT (A items first) from register set SS,
    // and the item's LDS writes with its last pair
    bf16x8 sp0, sp1;
    auto split_pair = [&](auto SS, int stage, auto IT, auto E) {
      constexpr int set = decltype(SS)::value;
      constexpr int it = decltype(IT)::value, e = 2 * decltype(E)::value;
      const float *x;
      if constexpr (it < SA::ITEMS) x = sa.r[set][it];
      else x = sb.r[set][it - SA::ITEMS];
      bf16x2 x0, x1;
      split2(f32x2{x[e], x[e + 1]}, x0, x1);
      sp0[e] = x0.x; sp0[e + 1] = x0.y;
      sp1[e] = x1.x; sp1[e + 1] = x1.y;
      if constexpr (e == 6) {
        __bf16 *sA = lds + stage * G::STAGE;
        __bf16 *base = it < SA::ITEMS ? sA : sA + G::NPL * G::PLANE_A;
        constexpr int PLANE = it < SA::ITEMS ? G::PLANE_A : G::PLANE_B;
        const int idx = tid + NT * (it < SA::ITEMS ? it : it - SA::ITEMS);
        const int rr = it < SA::ITEMS ? SA::row_of(idx) : SB::row_of(idx);
        const int cc = it < SA::ITEMS ? SA::chunk_of(idx) : SB::chunk_of(idx);
        const int off = rr * BK + ((cc ^ swz<BK>(rr)) << 3);
        *reinterpret_cast<bf16x8 *>(base + off) = sp0;
        *reinterpret_cast<bf16x8 *>(base + PLANE + off) = sp1;
      }
    };
    // LS: register set receiving slab s+3; SS: set holding slab s+2; fc:
    // fragments of slab s (a1, b0 already read); fn: receives the a1, b0
    // fragments of slab s+1 (after a0 * b1, while a0 * b0 still needs fc.b0).
    // The step's other work sits between its MFMAs in a fixed order (a
    // scheduling barrier after each slot): the reads of a0 and b1 first, the
    // global loads, the split and LDS writes of slab s+2 during a0 * b1's
    // predecessor slots, the first-product reads of slab s+1 last.
    auto step = [&](auto LS, auto SS, int kload, int st, Fr &fc, Fr &fn) {
      const int st1 = st == 2 ? 0 : st + 1, st2 = st1 == 2 ? 0 : st1 + 1;
      __builtin_amdgcn_sched_barrier(0);
      static_for<kMfma>([&](auto Q) {
        constexpr int m = decltype(Q)::value;
        if constexpr (2 * m < kHalf) {
          rd_one(fc, st, Rest{}, std::integral_constant<int, 2 * m>{});
          if constexpr (2 * m + 1 < kHalf) rd_one(fc, st, Rest{}, std::integral_constant<int, 2 * m + 1>{});
        }
        mfma_one(fc, Q);
        constexpr int kLoad0 = (kHalf + 1) / 2;
        if constexpr (m >= kLoad0 && m < kLoad0 + SA::ITEMS)
          sa.template load_item<decltype(LS)::value>(m - kLoad0, kload);
        else if constexpr (m >= kLoad0 + SA::ITEMS && m < kLoad0 + kItems)
          sb.template load_item<decltype(LS)::value>(m - kLoad0 - SA::ITEMS, kload);
        constexpr int kSplit0 = kBlk;
        if constexpr (m >= kSplit0 && m < kSplit0 + 4 * kItems)
          split_pair(SS, st2, std::integral_constant<int, (m - kSplit0) / 4>{},
                     std::integral_constant<int, (m - kSplit0) % 4>{});
        constexpr int kEarly0 = 2 * kBlk;
        if constexpr (m >= kEarly0 && 2 * (m - kEarly0) < kHalf) {
          rd_one(fn, st1, First{}, std::integral_constant<int, 2 * (m - kEarly0)>{});
          if constexpr (2 * (m - kEarly0) + 1 < kHalf)
            rd_one(fn, st1, First{}, std::integral_constant<int, 2 * (m - kEarly0) + 1>{});
        }
        __builtin_amdgcn_sched_barrier(0);
      });
      __syncthreads();
    };
    Fr f0, f1;
    // prologue: slab 0 is in stage 0 (above); slab 1 to stage 1, slab 2 in
    // flight in set 0, the first-product fragments of slab 0 in registers
    if (KT > 1) gload(S1{}, Fast{}, kslab(1));
    else gload(S1{}, Masked{}, kbase);
    sstore(S1{}, 1);
    if (KT > 1) gload(S0{}, Fast{}, kslab(2));
    else gload(S0{}, Masked{}, kbase);
    __syncthreads();
    rd(f0, 0, First{});
    int st = 0;
    for (; t + 2 <= KT; t += 2) {
      step(S1{}, S0{}, kslab(t + 3), st, f0, f1);
      st = st == 2 ? 0 : st + 1;
      step(S0{}, S1{}, kslab(t + 4), st, f1, f0);
      st = st == 2 ? 0 : st + 1;
    }
    if (t < KT) {  // odd slab count: the last slab, in stage st, a1 and b0 in f0
      rd(f0, st, Rest{});
      prod(f0, 1, 0);
      prod(f0, 0, 1);
      prod(f0, 0, 0);
    }
  } else if constexpr (kDeep) {
    // One wave per SIMD (4 waves of 128 x 128): no other wave hides a stall,
    // so every latency is covered inside the wave.  Slab s is loaded from
    // global memory in step s-3 (register set s%2), split and written to LDS
    // stage s%2 in step s-2, read into fragment set s%2 in step s-1 and
    // multiplied in step s.  The MFMAs of a step depend on nothing issued in
    // that step; the barrier at its end orders the writes of slab s+2 before
    // their reads (next step) and the reads of slab s+1 before stage (s+1)%2
    // is overwritten (next step).  The other work of a step is placed between
    // its MFMAs in a fixed order (scheduling barriers keep the compiler from
    // regrouping it): the global loads first, then the fragment reads, then
    // the split and LDS writes one item at a time.
    constexpr int kProd = NP == 2 ? 3 : 6;
    constexpr int kBlk = G::FM * G::FN;
    constexpr int kMfma = kBlk * kProd;
    constexpr int kReads = (G::FM + G::FN) * NP;
    constexpr int kItems = SA::ITEMS + SB::ITEMS;
    constexpr int kRead0 = kItems;                 // first MFMA slot with fragment reads
    constexpr int kSplit0 = kRead0 + (kReads + 1) / 2;  // first slot of the split
    static_assert(kSplit0 + 4 * kItems <= kMfma, "the step's work fits between its MFMAs");
    // product q of the step: planes (pa, pb), small products first
    auto mfma_one = [&](const Frags &f, auto Q) {
      constexpr int q = decltype(Q)::value;
      constexpr int pr = q / kBlk, bi = (q % kBlk) / G::FN, bj = q % G::FN;
      constexpr int pa = NP == 2 ? (pr == 0 ? 1 : 0) : (pr < 3 ? 2 - pr : (pr == 3 ? 1 : 0));
      constexpr int pb = NP == 2 ? (pr == 1 ? 1 : 0) : (pr < 3 ? pr : (pr == 4 ? 1 : 0));
      acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[pa][bi], f.b[pb][bj], acc[bi][bj],
                                                            0, 0, 0);
    };
    // fragment read r of a slab: B planes then A planes, one 32-row block each
    auto read_one = [&](Frags &f, int stage, auto R) {
      constexpr int r = decltype(R)::value;
      const __bf16 *sA = lds + stage * G::STAGE;
      const __bf16 *sB = sA + G::NPL * G::PLANE_A;
      const int c = lgrp;  // one k-step per slab: logical chunk 0 or 1
      if constexpr (r < NP * G::FN) {
        constexpr int p = r / G::FN, j = r % G::FN;
        const int n = wn0 + j * 32 + lrow;
        f.b[p][j] = *reinterpret_cast<const bf16x8 *>(sB + p * G::PLANE_B + n * BK +
                                                      ((c ^ swz<BK>(n)) << 3));
      } else {
        constexpr int p = (r - NP * G::FN) / G::FM, i = (r - NP * G::FN) % G::FM;
        const int rr = wm0 + i * 32 + lrow;
        f.a[p][i] = *reinterpret_cast<const bf16x8 *>(sA + p * G::PLANE_A + rr * BK +
                                                      ((c ^ swz<BK>(rr)) << 3));
      }
    };
    // the split of item it (A items first, then B items), one value pair at a
    // time, and its LDS writes with the last pair
    bf16x8 sp[NP];
    auto split_pair = [&](auto S, int stage, auto IT, auto E) {
      constexpr int set = decltype(S)::value;
      constexpr int it = decltype(IT)::value, e = 2 * decltype(E)::value;
      const float *x;
      if constexpr (it < SA::ITEMS) x = sa.r[set][it];
      else x = sb.r[set][it - SA::ITEMS];
      bf16x2 x0, x1, x2;
      if constexpr (NP == 2) split2(f32x2{x[e], x[e + 1]}, x0, x1);
      else split3(f32x2{x[e], x[e + 1]}, x0, x1, x2);
      sp[0][e] = x0.x; sp[0][e + 1] = x0.y;
      sp[1][e] = x1.x; sp[1][e + 1] = x1.y;
      if constexpr (NP == 3) { sp[2][e] = x2.x; sp[2][e + 1] = x2.y; }
      if constexpr (e == 6) {
        __bf16 *sA = lds + stage * G::STAGE;
        __bf16 *base = it < SA::ITEMS ? sA : sA + G::NPL * G::PLANE_A;
        constexpr int PLANE = it < SA::ITEMS ? G::PLANE_A : G::PLANE_B;
        const int idx = tid + NT * (it < SA::ITEMS ? it : it - SA::ITEMS);
        const int rr = it < SA::ITEMS ? SA::row_of(idx) : SB::row_of(idx);
        const int cc = it < SA::ITEMS ? SA::chunk_of(idx) : SB::chunk_of(idx);
        const int off = rr * BK + ((cc ^ swz<BK>(rr)) << 3);
#pragma unroll
        for (int p = 0; p < NP; ++p) *reinterpret_cast<bf16x8 *>(base + p * PLANE + off) = sp[p];
      }
    };
    auto step = [&](auto LS, int kload, auto SS, int wstage, Frags &fn, int rstage,
                    const Frags &fc) {
      constexpr int lset = decltype(LS)::value;
      __builtin_amdgcn_sched_barrier(0);
      static_for<kMfma>([&](auto Q) {
        constexpr int m = decltype(Q)::value;
        mfma_one(fc, Q);
        if constexpr (m < SA::ITEMS) sa.template load_item<lset>(m, kload);
        else if constexpr (m < kItems) sb.template load_item<lset>(m - SA::ITEMS, kload);
        if constexpr (m >= kRead0 && 2 * (m - kRead0) < kReads) {
          read_one(fn, rstage, std::integral_constant<int, 2 * (m - kRead0)>{});
          if constexpr (2 * (m - kRead0) + 1 < kReads)
            read_one(fn, rstage, std::integral_constant<int, 2 * (m - kRead0) + 1>{});
        }
        if constexpr (m >= kSplit0 && m < kSplit0 + 4 * kItems)
          split_pair(SS, wstage, std::integral_constant<int, (m - kSplit0) / 4>{},
                     std::integral_constant<int, (m - kSplit0) % 4>{});
        __builtin_amdgcn_sched_barrier(0);
      });
    };
    Frags f0, f1;
    if (KT > 1) gload(S1{}, Fast{}, kslab(1));
    else gload(S1{}, Masked{}, kbase);
    sstore(S1{}, 1);
    if (KT > 1) gload(S0{}, Fast{}, kslab(2));
    else gload(S0{}, Masked{}, kbase);
    __syncthreads();
    frag_read(f0, 0, 0);
    __syncthreads();
    for (; t + 2 <= KT; t += 2) {
      step(S1{}, kslab(t + 3), S0{}, 0, f1, 1, f0);
      __syncthreads();
      step(S0{}, kslab(t + 4), S1{}, 1, f0, 0, f1);
      __syncthreads();
    }
    if (t < KT) frag_mfma(f0);  // odd slab count: the last slab is in f0
  } else if constexpr (NP == 1 || G::KS == 2) {
    // Two register sets with two k-steps per slab (the FP32 mode, whose 64
    // MFMAs per wave and slab leave the loads and stores plenty of room, and
    // 32-deep split slabs with their loads issued two slabs ahead): the
    // compiler schedules the loads and stores around the MFMAs.
    if (KT > 1) gload(S1{}, Fast{}, kslab(1));
    else gload(S1{}, Masked{}, kbase);
    __syncthreads();
    for (; t + 2 <= KT; t += 2) {
      gload(S0{}, Fast{}, kslab(t + 2));
      __builtin_amdgcn_sched_barrier(0);
      mfma_stage(0);
      sstore(S1{}, 1);
      __syncthreads();
      gload(S1{}, Fast{}, kslab(t + 3));
      __builtin_amdgcn_sched_barrier(0);
      mfma_stage(1);
      sstore(S0{}, 0);
      __syncthreads();
    }
  } else {
    // Two register sets, one k-step per stage: each step's instructions are
    // interleaved one by one with its MFMAs -- all fragment reads first, then
    // one global load after each of the first MFMAs, then the split's VALU
    // work three instructions per MFMA (measured against 2, 4 and 6: 1 %
    // faster than 4, the other two slower), the LDS writes last.  Issued in
    // clusters, the loads and the split stall the wave between MFMAs (both
    // waves of a SIMD reach them together, so neither feeds the pipe).
    static_assert(G::KS == 1, "two register sets are used with 16-deep slabs");
    constexpr int kMfma = G::FM * G::FN * (NP == 2 ? 3 : 6);
    constexpr int kReads = (G::FM + G::FN) * NP;
    constexpr int kLoads = SA::LOADS + SB::LOADS;
    constexpr int kWrites = (SA::ITEMS + SB::ITEMS) * NP;
    constexpr int kLoadSlots = kLoads < kMfma ? kLoads : kMfma;
    auto step = [&](auto LS, int kload, int mstage, auto SS, int sstage) {
      gload(LS, Fast{}, kload);
      Frags f;
      frag_read(f, mstage, 0);
      frag_mfma(f);
      sstore(SS, sstage);
      __builtin_amdgcn_sched_group_barrier(0x100, kReads, 0);   // DS read
#pragma unroll
      for (int i = 0; i < kLoadSlots; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);      // MFMA
        __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);      // VMEM read
      }
#pragma unroll
      for (int i = kLoadSlots; i < kMfma; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);      // MFMA
        __builtin_amdgcn_sched_group_barrier(0x002, 3, 0);      // VALU
      }
      __builtin_amdgcn_sched_group_barrier(0x200, kWrites, 0);  // DS write
    };
    if (KT > 1) gload(S1{}, Fast{}, kslab(1));
    else gload(S1{}, Masked{}, kbase);
    __syncthreads();
    for (; t + 2 <= KT; t += 2) {
      step(S0{}, kslab(t + 2), 0, S1{}, 1);
      __syncthreads();
      step(S1{}, kslab(t + 3), 1, S0{}, 0);
      __syncthreads();
    }
  }
  if constexpr (!kDeep && ST == 2) {
    if (t < KT) {  // odd slab count: the last slab sits in stage 0
      mfma_stage(0);
    }
  }

  // ---- sum of the k-groups' partial tiles (group order) --------------------
  if constexpr (KG > 1) {
    // every fragment read of both groups is done before their stages are
    // reused; group 1 leaves its partial tile in LDS lane-contiguous (the
    // two groups' stages together hold exactly one group's accumulators)
    float *red = reinterpret_cast<float *>(lds - grp * (G::LDS_BYTES / 2));
    static_assert(G::NT * G::FM * G::FN * 16 * 4 <= KG * G::LDS_BYTES, "partial tile fits");
    __syncthreads();
    if (grp == 1) {
#pragma unroll
      for (int i = 0; i < G::FM; ++i)
#pragma unroll
        for (int j = 0; j < G::FN; ++j)
#pragma unroll
          for (int e = 0; e < 16; ++e)
            red[(((wave * G::FM + i) * G::FN + j) * 16 + e) * 64 + lane] = acc[i][j][e];
    }
    __syncthreads();
    if (grp == 1) return;
#pragma unroll
    for (int i = 0; i < G::FM; ++i)
#pragma unroll
      for (int j = 0; j < G::FN; ++j)
#pragma unroll
        for (int e = 0; e < 16; ++e)
          acc[i][j][e] += red[(((wave * G::FM + i) * G::FN + j) * 16 + e) * 64 + lane];
  }

  // ---- peeled epilogue ----------------------------------------------------
  // 32x32 block layout: lane l, element e -> row 8*(e/4) + 4*(l/32) + e%4,
  // column l%32.
  const int rowsC = Mr < BM ? Mr : BM, colsC = Nr < BN ? Nr : BN;
  if ((int64_t)BM * ldc * 4 < ((int64_t)1 << 31)) {
    // Buffer stores with 32-bit offsets: the resource covers the tile's valid
    // part of C (rows past M fall beyond it and are dropped), columns past N
    // get an out-of-range lane offset, and the row step of element e is a
    // wave-uniform scalar offset -- no per-element address arithmetic.
    const __amdgpu_buffer_rsrc_t rC = __builtin_amdgcn_make_buffer_rsrc(
        C + (int64_t)m0 * ldc + n0, (short)0, (int)(((int64_t)(rowsC - 1) * ldc + colsC) * 4),
        kBufferFlags);
    const int ldc4 = (int)ldc * 4;
    // With beta != 0 the reads of C for a group of blocks are all issued
    // before the group's first store: a buffer load is never moved above a
    // buffer store through the same resource, so a read-modify-write per
    // element would wait out one memory round trip per element.
    constexpr int kBlk = G::FM * G::FN;
    constexpr int kGrp = kBlk < 4 ? kBlk : 4;
    static_assert(kBlk % kGrp == 0, "whole groups of accumulator blocks");
#pragma unroll
    for (int g0 = 0; g0 < kBlk; g0 += kGrp) {
      float cold[kGrp][16];
      int vb[kGrp];
#pragma unroll
      for (int q = 0; q < kGrp; ++q) {
        const int i = (g0 + q) / G::FN, j = (g0 + q) % G::FN;
        const int col = wn0 + j * 32 + lrow;
        vb[q] = col < colsC ? (wm0 + i * 32 + 4 * lgrp) * ldc4 + col * 4 : (int)0x80000000;
        if (BETA) {
#pragma unroll
          for (int e = 0; e < 16; ++e)
            cold[q][e] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                                       rC, vb[q], (8 * (e >> 2) + (e & 3)) * ldc4, 0));
        }
      }
#pragma unroll
      for (int q = 0; q < kGrp; ++q) {
        const int i = (g0 + q) / G::FN, j = (g0 + q) % G::FN;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          float v = alpha * acc[i][j][e];
          if (BETA) v = fmaf(beta, cold[q][e], v);
          __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), rC, vb[q],
                                                (8 * (e >> 2) + (e & 3)) * ldc4, 0);
        }
      }
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < G::FM; ++i)
#pragma unroll
    for (int j = 0; j < G::FN; ++j) {
      const int col = wn0 + j * 32 + lrow;
      if (!interior && col >= Nr) continue;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int row = wm0 + i * 32 + 8 * (e >> 2) + 4 * lgrp + (e & 3);
        if (interior || row < Mr) {
          float *p = C + (int64_t)(m0 + row) * ldc + (n0 + col);
          const float v = alpha * acc[i][j][e];
          *p = BETA ? fmaf(beta, *p, v) : v;
        }
      }
    }
}

}  // namespace bx3
}  // namespace mm
