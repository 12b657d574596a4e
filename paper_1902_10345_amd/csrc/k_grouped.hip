// k_grouped.hip -- one persistent launch for a batch of independent GEMMs of
// uneven sizes on the 3xBF16 split-precision MFMA path.
//
// The batch is flattened into one list of output tiles (problem p owns tiles
// [start[p], start[p+1])).  A grid sized to the machine's resident capacity
// takes tile indices from an atomic counter -- the mechanism behind the
// paper's consume scopes (Sec. 3.3), where workers take elements off a shared
// stream with atomic operations -- finds the
// owning problem by binary search over the prefix of tile counts and runs the
// same tile body as the single-GEMM kernel.  Each problem carries its own tile
// shape, chosen per problem (library heuristic or the autotuner).
//
// The counter lives in the caller's workspace and is cleared by a fill kernel
// launched before the persistent kernel on the same stream, so the pair can be
// captured into a HIP graph and replayed (no memset nodes).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "bf16x3.hpp"
#include "grouped.hpp"
#include "kernels.hpp"

namespace mm {
namespace grp {

// Tile variants of the grouped kernel (all 256 lanes, 2 bf16 planes, BK 32).
//   0: 128 x 128 (2 x 2 waves of 64 x 64)     1: 64 x 64 (2 x 2 waves of 32 x 32)
constexpr int kVariants = 2;
constexpr int kBM[kVariants] = {128, 64};
constexpr int kBN[kVariants] = {128, 64};
using G0 = bx3::Cfg<128, 128, 32, 64, 64, 2, 4>;
using G1 = bx3::Cfg<64, 64, 32, 32, 32, 2, 4>;
constexpr int kLdsBytes = G0::LDS_BYTES > G1::LDS_BYTES ? G0::LDS_BYTES : G1::LDS_BYTES;

template <int V, bool VEC, bool BETA>
__device__ __forceinline__ void run_tile(const Desc &d, int m0, int n0, __bf16 *lds) {
  if constexpr (V == 0)
    bx3::tile<128, 128, 32, 64, 64, 2, 4, VEC, BETA>(d.M, d.N, d.K, d.alpha, d.A, d.lda, d.B,
                                                     d.ldb, d.beta, d.C, d.ldc, m0, n0, lds);
  else
    bx3::tile<64, 64, 32, 32, 32, 2, 4, VEC, BETA>(d.M, d.N, d.K, d.alpha, d.A, d.lda, d.B, d.ldb,
                                                   d.beta, d.C, d.ldc, m0, n0, lds);
}

__device__ __forceinline__ int starts_at(bool in_lds, const int *s_starts, const int *starts,
                                         int p) {
  return in_lds ? s_starts[p] : starts[p];
}

__global__ __launch_bounds__(64) void clear_counter_kernel(unsigned *counter) {
  if (threadIdx.x == 0) counter[0] = 0u;
}

// Tile prefixes of batches up to this size are searched in LDS.
constexpr int kLdsStarts = 3072;

__global__ __launch_bounds__(256, 2) void grouped_kernel(const Desc *__restrict__ descs,
                                                         const int *__restrict__ starts, int count,
                                                         int total_tiles, int static_tiles,
                                                         unsigned *__restrict__ counter) {
  __shared__ __attribute__((aligned(16))) __bf16 lds[kLdsBytes / 2];
  __shared__ int s_starts[kLdsStarts];
  __shared__ int s_tile[2];
  const bool in_lds = count < kLdsStarts;
  if (in_lds)
    for (int i = threadIdx.x; i <= count; i += 256) s_starts[i] = starts[i];
  // Tiles [0, static_tiles) are dealt round-robin (tile t to slot t mod G):
  // the list is sorted longest first, so each round hands every
  // workgroup a tile of similar cost and needs no atomics.  The remaining
  // tiles are dequeued from the counter (first come, first served), which
  // evens out the tail; a whole grid's worth of simultaneous same-address
  // atomics would otherwise serialise at the start of every launch.
  // Workgroup ids are dispatched round robin over the 8 XCDs; the slot
  // permutation hands each XCD a run of G/8 consecutive tiles per round, so
  // neighbouring tiles of a problem -- which share A row panels and B column
  // panels -- run on one XCD and meet in its L2 instead of being fetched from
  // HBM once per XCD.
  const int G = gridDim.x;
  const int w = (int)blockIdx.x;
  const int slot = G % 8 == 0 ? (w % 8) * (G / 8) + w / 8 : w;
  if (threadIdx.x == 0)
    s_tile[0] = slot < static_tiles ? slot : static_tiles + (int)atomicAdd(counter, 1u);
  __syncthreads();
  // Values read from LDS are per-lane to the compiler; the tile index is
  // wave-uniform by construction, and saying so keeps everything derived
  // from it (tile origin, buffer resources) in scalar registers -- a per-lane
  // buffer resource turns every buffer load into a readfirstlane loop.
  int t = __builtin_amdgcn_readfirstlane(s_tile[0]);
  for (int it = 1; t < total_tiles; ++it) {
    // Dequeue the next tile now: the atomic's round trip overlaps this tile's
    // work, and its result is only read after the tile.
    unsigned next = 0u;
    if (threadIdx.x == 0)
      next = (t + G < static_tiles || static_tiles >= total_tiles)
                 ? (unsigned)(t + G)
                 : (unsigned)static_tiles + atomicAdd(counter, 1u);
    // owning problem: the last p with starts[p] <= t
    int lo = 0, hi = count - 1;
    if (in_lds) {
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_starts[mid] <= t) lo = mid;
        else hi = mid - 1;
      }
    } else {
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (starts[mid] <= t) lo = mid;
        else hi = mid - 1;
      }
    }
    lo = __builtin_amdgcn_readfirstlane(lo);
    const Desc d = descs[lo];
    const int local = t - __builtin_amdgcn_readfirstlane(starts_at(in_lds, s_starts, starts, lo));
    const int bm = d.variant == 0 ? 128 : 64, bn = bm;
    // tiles of a problem in groups of 8 tile rows, as in the single-GEMM
    // kernels: consecutive dequeues share A row panels and B column panels
    int tm, tn;
    tile_coords(local, (d.M + bm - 1) / bm, d.tiles_n, 8, tm, tn);
    const int m0 = tm * bm, n0 = tn * bn;
    const int sel = d.variant * 4 + (d.vec ? 2 : 0) + (d.beta != 0.0f ? 1 : 0);
    switch (sel) {
      case 0: run_tile<0, false, false>(d, m0, n0, lds); break;
      case 1: run_tile<0, false, true>(d, m0, n0, lds); break;
      case 2: run_tile<0, true, false>(d, m0, n0, lds); break;
      case 3: run_tile<0, true, true>(d, m0, n0, lds); break;
      case 4: run_tile<1, false, false>(d, m0, n0, lds); break;
      case 5: run_tile<1, false, true>(d, m0, n0, lds); break;
      case 6: run_tile<1, true, false>(d, m0, n0, lds); break;
      default: run_tile<1, true, true>(d, m0, n0, lds); break;
    }
    // One barrier per tile: publishes the next index (alternate slots, so no
    // thread can still be reading the slot being written) and separates this
    // tile's last LDS reads from the next tile's first LDS writes.
    if (threadIdx.x == 0) s_tile[it & 1] = (int)next;
    __syncthreads();
    t = __builtin_amdgcn_readfirstlane(s_tile[it & 1]);
  }
}

}  // namespace grp

int grouped_num_variants() { return grp::kVariants; }
int grouped_variant_bm(int v) { return grp::kBM[v]; }

// Library heuristic: the variant with the smaller padded work, where a 64 x 64
// tile is charged `small_cost` times a 128 x 128 tile's work per output
// element (it re-reads its operands twice as often).
int grouped_pick_variant(int64_t M, int64_t N, double small_cost) {
  const double w0 = (double)((M + 127) / 128) * ((N + 127) / 128) * 128.0 * 128.0;
  const double w1 = (double)((M + 63) / 64) * ((N + 63) / 64) * 64.0 * 64.0 * small_cost;
  return w1 < w0 ? 1 : 0;
}

size_t grouped_ws_bytes(int count) {
  const size_t head = 256;
  const size_t descs = ((sizeof(Desc) * (size_t)count + 255) / 256) * 256;
  const size_t starts = sizeof(int) * ((size_t)count + 1);
  return head + descs + starts;
}

gemm_status grouped_build(const gemm_problem *probs, int count, const int *variant,
                          std::vector<Desc> &descs, std::vector<int> &starts, int &total) {
  descs.resize(count);
  starts.resize((size_t)count + 1);
  const double small_cost = tuned_small_cost();
  // Longest tiles first: a tile's time grows with K, so handing out the
  // deepest problems' tiles first keeps the end of the queue short.  The
  // table order changes only the schedule, never a problem's result.
  std::vector<int> order(count);
  for (int p = 0; p < count; ++p) order[p] = p;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return probs[a].K > probs[b].K; });
  int64_t t = 0;
  for (int slot = 0; slot < count; ++slot) {
    const int p = order[slot];
    const gemm_problem &q = probs[p];
    Desc &d = descs[slot];
    d.A = q.A; d.B = q.B; d.C = q.C;
    d.lda = q.lda; d.ldb = q.ldb; d.ldc = q.ldc;
    d.M = (int)q.M; d.N = (int)q.N; d.K = (int)q.K;
    d.alpha = q.alpha; d.beta = q.beta;
    d.variant = variant ? variant[p] : grouped_pick_variant(q.M, q.N, small_cost);
    const int bm = grp::kBM[d.variant], bn = grp::kBN[d.variant];
    d.vec = (q.lda % 4 == 0 && q.K % 4 == 0 && ((uintptr_t)q.A & 15) == 0) ? 1 : 0;
    // problems that need no MFMA work contribute no tiles; the host handles
    // them (no-op or C <- beta*C) before the launch
    const bool work = q.M > 0 && q.N > 0 && q.K > 0 && q.alpha != 0.0f;
    d.tiles_n = work ? (int)((q.N + bn - 1) / bn) : 0;
    const int64_t tiles = work ? ((q.M + bm - 1) / bm) * (int64_t)d.tiles_n : 0;
    starts[slot] = (int)t;
    t += tiles;
    if (t > 0x7fffffff) { set_error("grouped_gemm: too many tiles"); return GEMM_STATUS_UNSUPPORTED; }
  }
  starts[count] = (int)t;
  total = (int)t;
  return GEMM_STATUS_OK;
}

gemm_status grouped_enqueue(void *ws, int count, int total, int grid, hipStream_t s) {
  uint8_t *base = static_cast<uint8_t *>(ws);
  unsigned *counter = reinterpret_cast<unsigned *>(base);
  const Desc *descs = reinterpret_cast<const Desc *>(base + 256);
  const int *starts = reinterpret_cast<const int *>(
      base + 256 + ((sizeof(Desc) * (size_t)count + 255) / 256) * 256);
  hipLaunchKernelGGL(grp::clear_counter_kernel, dim3(1), dim3(64), 0, s, counter);
  if (gemm_status st = check_launch("clear_counter_kernel")) return st;
  if (total == 0) return GEMM_STATUS_OK;
  // all but the last two rounds are dealt statically, and at least the first
  // round (a batch of at most one round needs no atomics at all)
  const int rounds = total / grid;
  const int static_tiles = rounds > 2 ? (rounds - 2) * grid : std::min(total, grid);
  hipLaunchKernelGGL(grp::grouped_kernel, dim3(grid), dim3(256), 0, s, descs, starts, count, total,
                     static_tiles, counter);
  return check_launch("grouped_kernel");
}

gemm_status grouped_upload(void *ws, const std::vector<Desc> &descs, const std::vector<int> &starts,
                           hipStream_t s) {
  uint8_t *base = static_cast<uint8_t *>(ws);
  const size_t dbytes = sizeof(Desc) * descs.size();
  const size_t soff = 256 + ((dbytes + 255) / 256) * 256;
  hipError_t e = hipMemcpyAsync(base + 256, descs.data(), dbytes, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail("grouped_gemm: descriptor upload", e);
  e = hipMemcpyAsync(base + soff, starts.data(), sizeof(int) * starts.size(), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail("grouped_gemm: tile-prefix upload", e);
  // the host vectors are freed on return: make sure the copies have consumed them
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail("grouped_gemm: upload sync", e);
  return GEMM_STATUS_OK;
}

gemm_status grouped_upload_pinned(void *ws, void *pinned, const std::vector<Desc> &descs,
                                  const std::vector<int> &starts, hipStream_t s) {
  // the pinned staging buffer mirrors the workspace from byte 256 on; the
  // caller guarantees it is not rewritten before this copy has executed
  const size_t dbytes = sizeof(Desc) * descs.size();
  const size_t soff = ((dbytes + 255) / 256) * 256;
  uint8_t *h = static_cast<uint8_t *>(pinned);
  std::memcpy(h, descs.data(), dbytes);
  std::memcpy(h + soff, starts.data(), sizeof(int) * starts.size());
  hipError_t e = hipMemcpyAsync(static_cast<uint8_t *>(ws) + 256, h, soff + sizeof(int) * starts.size(),
                                hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail("grouped: descriptor upload", e);
  return GEMM_STATUS_OK;
}

int grouped_grid(int total) {
  const int resident = num_cus() * 2;  // two 256-lane workgroups per CU
  return std::max(1, std::min(total, resident));
}

}  // namespace mm
