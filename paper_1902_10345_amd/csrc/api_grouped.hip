// api_grouped.hip -- C-ABI of the grouped launch and its HIP-graph form.
#include <string>
#include <vector>

#include "common.hpp"
#include "grouped.hpp"
#include "kernels.hpp"

namespace mm {

// Per-problem checks (the same rules as a single call); on failure the message
// names the problem index and the status points at argument 1 (problems).
static gemm_status check_problems(const char *fn, const gemm_problem *probs, int count,
                                  const int *variant) {
  for (int p = 0; p < count; ++p) {
    const gemm_problem &q = probs[p];
    const char *why = nullptr;
    if (q.M < 0 || q.N < 0 || q.K < 0) why = "negative size";
    else if (q.M > 0x7fffffffLL || q.N > 0x7fffffffLL || q.K > 0x7fffffffLL) why = "size exceeds 2^31-1";
    else if (q.lda < (q.K > 1 ? q.K : 1)) why = "lda < max(1,K)";
    else if (q.ldb < (q.N > 1 ? q.N : 1)) why = "ldb < max(1,N)";
    else if (q.ldc < (q.N > 1 ? q.N : 1)) why = "ldc < max(1,N)";
    else if (q.M > 0 && q.N > 0 && !q.C) why = "C is NULL";
    else if (q.M > 0 && q.N > 0 && q.K > 0 && q.alpha != 0.0f && (!q.A || !q.B)) why = "A or B is NULL";
    else if ((128 * q.lda + q.K) * 4 >= ((int64_t)1 << 31) || (32 * q.ldb + q.N) * 4 >= ((int64_t)1 << 31))
      why = "leading dimension too large for 32-bit tile offsets";
    else if (variant && (variant[p] < 0 || variant[p] >= grouped_num_variants())) {
      set_error(std::string(fn) + ": tile_variant[" + std::to_string(p) + "] out of range");
      return -4;
    }
    if (why) {
      set_error(std::string(fn) + ": argument 1 (problems[" + std::to_string(p) + "]): " + why);
      return -1;
    }
  }
  return GEMM_STATUS_OK;
}

static gemm_status check_common(const char *fn, const gemm_problem *probs, int count, int path,
                                const int *variant, void *ws, size_t ws_bytes) {
  if (count < 0) return bad_arg(2, fn, "(count) must be >= 0");
  if (count > 0 && !probs) return bad_arg(1, fn, "(problems) is NULL");
  if (path != GEMM_PATH_3XBF16) return bad_arg(3, fn, "(path) must be GEMM_PATH_3XBF16");
  gemm_status st = check_problems(fn, probs, count, variant);
  if (st) return st;
  if (!ws) return bad_arg(5, fn, "(workspace) is NULL");
  if (((uintptr_t)ws & 255) != 0) return bad_arg(5, fn, "(workspace) must be 256-byte aligned");
  if (ws_bytes < grouped_ws_bytes(count)) return bad_arg(6, fn, "(ws_bytes) too small");
  return GEMM_STATUS_OK;
}

// C <- beta*C for the problems that need no matrix-core work.
static gemm_status enqueue_scale_only(const gemm_problem *probs, int count, hipStream_t s) {
  for (int p = 0; p < count; ++p) {
    const gemm_problem &q = probs[p];
    if (q.M > 0 && q.N > 0 && (q.K == 0 || q.alpha == 0.0f)) {
      gemm_status st = scale_c(q.M, q.N, q.beta, q.C, q.ldc, s);
      if (st) return st;
    }
  }
  return GEMM_STATUS_OK;
}

struct GroupedGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

}  // namespace mm

using namespace mm;

extern "C" {

size_t grouped_gemm_workspace_bytes(int count) { return count < 0 ? 0 : grouped_ws_bytes(count); }

int grouped_default_variant(int64_t M, int64_t N, int64_t K) {
  (void)K;
  return grouped_pick_variant(M, N, tuned_small_cost());
}

gemm_status grouped_gemm(const gemm_problem *problems, int count, int path,
                         const int *tile_variant, void *workspace, size_t ws_bytes,
                         hipStream_t stream) {
  clear_error();
  const char *fn = "grouped_gemm";
  gemm_status st = check_common(fn, problems, count, path, tile_variant, workspace, ws_bytes);
  if (st) return st;
  std::vector<Desc> descs;
  std::vector<int> starts;
  int total = 0;
  if ((st = grouped_build(problems, count, tile_variant, descs, starts, total))) return st;
  if ((st = enqueue_scale_only(problems, count, stream))) return st;
  if (count == 0) return GEMM_STATUS_OK;
  if ((st = grouped_upload(workspace, descs, starts, stream))) return st;
  return grouped_enqueue(workspace, count, total, grouped_grid(total), stream);
}

gemm_status grouped_graph_create(const gemm_problem *problems, int count, int path,
                                 const int *tile_variant, void *workspace, size_t ws_bytes,
                                 hipStream_t stream, void **graph) {
  clear_error();
  const char *fn = "grouped_graph_create";
  if (!graph) return bad_arg(8, fn, "(graph) is NULL");
  *graph = nullptr;
  gemm_status st = check_common(fn, problems, count, path, tile_variant, workspace, ws_bytes);
  if (st) return st;
  std::vector<Desc> descs;
  std::vector<int> starts;
  int total = 0;
  if ((st = grouped_build(problems, count, tile_variant, descs, starts, total))) return st;
  if (count > 0 && (st = grouped_upload(workspace, descs, starts, stream))) return st;

  hipStream_t cap = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail("grouped_graph_create: stream", e);
  auto *g = new GroupedGraph();
  e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    hipStreamDestroy(cap);
    delete g;
    return hip_fail("grouped_graph_create: begin capture", e);
  }
  st = enqueue_scale_only(problems, count, cap);
  if (!st && count > 0) st = grouped_enqueue(workspace, count, total, grouped_grid(total), cap);
  e = hipStreamEndCapture(cap, &g->graph);
  hipStreamDestroy(cap);
  if (st || e != hipSuccess) {
    if (g->graph) hipGraphDestroy(g->graph);
    delete g;
    return st ? st : hip_fail("grouped_graph_create: end capture", e);
  }
  e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    hipGraphDestroy(g->graph);
    delete g;
    return hip_fail("grouped_graph_create: instantiate", e);
  }
  *graph = g;
  return GEMM_STATUS_OK;
}

gemm_status grouped_graph_launch(void *graph, hipStream_t stream) {
  clear_error();
  if (!graph) return bad_arg(1, "grouped_graph_launch", "(graph) is NULL");
  hipError_t e = hipGraphLaunch(static_cast<GroupedGraph *>(graph)->exec, stream);
  if (e != hipSuccess) return hip_fail("grouped_graph_launch", e);
  return GEMM_STATUS_OK;
}

gemm_status grouped_graph_destroy(void *graph) {
  clear_error();
  if (!graph) return GEMM_STATUS_OK;
  auto *g = static_cast<GroupedGraph *>(graph);
  if (g->exec) hipGraphExecDestroy(g->exec);
  if (g->graph) hipGraphDestroy(g->graph);
  delete g;
  return GEMM_STATUS_OK;
}

}  // extern "C"
