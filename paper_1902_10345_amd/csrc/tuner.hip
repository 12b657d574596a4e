// tuner.hip -- size-specific tile-configuration autotuner and its JSON cache.
//
// The paper reaches its best matrix-multiplication performance by tuning the
// transformation parameters for one size after the transformation chain
// (Sec. 6.2), and its IDE saves transformation chains to files (Sec. 4.2).
// Here the tunable parameter is the tile configuration: gemm_autotune times
// every configuration of a path on real operands and records the fastest per
// power-of-two size bucket; grouped_autotune picks the per-problem tile
// shapes of a grouped batch.  The table persists as a small JSON file.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "common.hpp"
#include "grouped.hpp"
#include "kernels.hpp"

namespace mm {

namespace {
using Key = std::tuple<int, int, int, int, int>;  // path, n_products, log2 buckets of M, N, K
std::mutex g_mu;
std::map<Key, int> g_table;
double g_small_cost = kDefaultSmallCost;

int bucket(int64_t x) {
  int b = 0;
  while (((int64_t)1 << b) < x) ++b;
  return b;
}
Key key(int path, int np, int64_t M, int64_t N, int64_t K) {
  if (path == GEMM_PATH_FP8_PREQUANTIZED) path = GEMM_PATH_FP8;  // same kernels
  return Key(path, path == GEMM_PATH_3XBF16 ? np : 0, bucket(M), bucket(N), bucket(K));
}
const char *cfg_name(int path, int cfg) {
  switch (path) {
    case GEMM_PATH_F32: return f32_config(cfg).name;
    case GEMM_PATH_3XBF16: return bx3_config(cfg).name;
    default: return fp8_config_name(cfg);
  }
}
int cfg_count(int path) {
  switch (path) {
    case GEMM_PATH_F32: return f32_num_configs();
    case GEMM_PATH_3XBF16: return bx3_num_configs();
    default: return fp8_num_configs();
  }
}
}  // namespace

int tuned_config(int path, int n_products, int64_t M, int64_t N, int64_t K) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_table.find(key(path, n_products, M, N, K));
  return it == g_table.end() ? -1 : it->second;
}

double tuned_small_cost() {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_small_cost;
}

}  // namespace mm

using namespace mm;

extern "C" {

gemm_status gemm_run_config(int path, int cfg, int64_t M, int64_t N, int64_t K, float alpha,
                            const float *A, int64_t lda, const float *B, int64_t ldb, float beta,
                            float *C, int64_t ldc, int n_products, void *workspace,
                            size_t ws_bytes, hipStream_t stream);

gemm_status gemm_autotune(int path, int64_t M, int64_t N, int64_t K, float alpha, const float *A,
                          int64_t lda, const float *B, int64_t ldb, float beta, float *C,
                          int64_t ldc, int n_products, void *workspace, size_t ws_bytes, int reps,
                          hipStream_t stream, int *best_cfg) {
  clear_error();
  const char *fn = "gemm_autotune";
  if (path < GEMM_PATH_F32 || path > GEMM_PATH_FP8_PREQUANTIZED) return bad_arg(1, fn, "(path) unknown");
  if (reps < 1) return bad_arg(16, fn, "(reps) must be >= 1");
  if (!best_cfg) return bad_arg(18, fn, "(best_cfg) is NULL");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  if (he != hipSuccess) {
    if (e0) hipEventDestroy(e0);
    return hip_fail("gemm_autotune: event", he);
  }
  int best = -1;
  float best_ms = 0.0f;
  gemm_status last = GEMM_STATUS_OK;
  for (int c = 0; c < cfg_count(path); ++c) {
    if (path == GEMM_PATH_3XBF16 && bx3_config_products(c) != n_products) continue;
    gemm_status st = gemm_run_config(path, c, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
                                     n_products, workspace, ws_bytes, stream);
    if (st < 0) { hipEventDestroy(e0); hipEventDestroy(e1); return st; }  // bad arguments
    if (st) { last = st; continue; }                                      // config unusable here
    he = hipEventRecord(e0, stream);
    for (int r = 0; !st && he == hipSuccess && r < reps; ++r)
      st = gemm_run_config(path, c, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, n_products,
                           workspace, ws_bytes, stream);
    if (!st && he == hipSuccess) he = hipEventRecord(e1, stream);
    if (!st && he == hipSuccess) he = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (!st && he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
    if (st || he != hipSuccess) {
      hipEventDestroy(e0);
      hipEventDestroy(e1);
      return st ? st : hip_fail("gemm_autotune: timing", he);
    }
    if (best < 0 || ms < best_ms) { best = c; best_ms = ms; }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (best < 0) {
    if (!last) set_error(std::string(fn) + ": no configuration for this path/n_products");
    return last ? last : GEMM_STATUS_UNSUPPORTED;
  }
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_table[key(path, n_products, M, N, K)] = best;
  }
  *best_cfg = best;
  return GEMM_STATUS_OK;
}

gemm_status grouped_autotune(const gemm_problem *problems, int count, int path, void *workspace,
                             size_t ws_bytes, int reps, hipStream_t stream, int *variants_out) {
  clear_error();
  const char *fn = "grouped_autotune";
  if (count < 1) return bad_arg(2, fn, "(count) must be >= 1");
  if (!problems) return bad_arg(1, fn, "(problems) is NULL");
  if (path != GEMM_PATH_3XBF16) return bad_arg(3, fn, "(path) must be GEMM_PATH_3XBF16");
  if (!workspace || ((uintptr_t)workspace & 255)) return bad_arg(4, fn, "(workspace) NULL or unaligned");
  if (ws_bytes < grouped_ws_bytes(count)) return bad_arg(5, fn, "(ws_bytes) too small");
  if (reps < 1) return bad_arg(6, fn, "(reps) must be >= 1");
  if (!variants_out) return bad_arg(8, fn, "(variants_out) is NULL");
  // validate the problems once through the public entry point's checks
  gemm_status st = grouped_gemm(problems, count, path, nullptr, workspace, ws_bytes, stream);
  if (st) return st;
  // Candidate policies, all expressed as the padded-work rule's relative cost
  // of a 64 x 64 tile element: 0 makes every tile 64 x 64, kNeverSmall every
  // tile 128 x 128, the others weigh padding against the small tile's extra
  // operand traffic.  The winner becomes the library's rule, so later
  // grouped_default_variant choices reproduce the returned variants.
  constexpr double kNeverSmall = 1e30;
  const double costs[] = {kNeverSmall, 0.0, 1.0, 1.3, 1.6, 2.0, 2.6};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  if (he != hipSuccess) {
    if (e0) hipEventDestroy(e0);
    return hip_fail("grouped_autotune: event", he);
  }
  float best_ms = 0.0f;
  double best_cost = kDefaultSmallCost;
  bool have_best = false;
  std::vector<int> var(count), best_var(count);
  for (double cost : costs) {
    for (int p = 0; p < count; ++p) var[p] = grouped_pick_variant(problems[p].M, problems[p].N, cost);
    std::vector<Desc> descs;
    std::vector<int> starts;
    int total = 0;
    if ((st = grouped_build(problems, count, var.data(), descs, starts, total))) break;
    if ((st = grouped_upload(workspace, descs, starts, stream))) break;
    const int grid = grouped_grid(total);
    if ((st = grouped_enqueue(workspace, count, total, grid, stream))) break;  // warm-up
    he = hipEventRecord(e0, stream);
    for (int r = 0; !st && he == hipSuccess && r < reps; ++r)
      st = grouped_enqueue(workspace, count, total, grid, stream);
    if (!st && he == hipSuccess) he = hipEventRecord(e1, stream);
    if (!st && he == hipSuccess) he = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (!st && he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
    if (st) break;
    if (he != hipSuccess) {
      st = hip_fail("grouped_autotune: timing", he);
      break;
    }
    if (!have_best || ms < best_ms) {
      have_best = true;
      best_ms = ms;
      best_cost = cost;
      best_var = var;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st) return st;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_small_cost = best_cost;
  }
  std::memcpy(variants_out, best_var.data(), sizeof(int) * (size_t)count);
  return GEMM_STATUS_OK;
}

gemm_status gemm_tuner_save(const char *json_path) {
  clear_error();
  if (!json_path) return bad_arg(1, "gemm_tuner_save", "(json_path) is NULL");
  FILE *f = std::fopen(json_path, "w");
  if (!f) {
    set_error(std::string("gemm_tuner_save: cannot open ") + json_path);
    return GEMM_STATUS_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  std::fprintf(f, "{\"arch\": \"gfx950\", \"grouped_small_cost\": %.6g, \"entries\": [\n", g_small_cost);
  size_t i = 0;
  for (const auto &kv : g_table) {
    int path, np, bm, bn, bk;
    std::tie(path, np, bm, bn, bk) = kv.first;
    std::fprintf(f, "{\"path\": %d, \"n_products\": %d, \"log2_m\": %d, \"log2_n\": %d, \"log2_k\": %d, \"config\": \"%s\"}%s\n",
                 path, np, bm, bn, bk, cfg_name(path, kv.second), ++i < g_table.size() ? "," : "");
  }
  std::fprintf(f, "]}\n");
  std::fclose(f);
  return GEMM_STATUS_OK;
}

gemm_status gemm_tuner_load(const char *json_path) {
  clear_error();
  if (!json_path) return bad_arg(1, "gemm_tuner_load", "(json_path) is NULL");
  FILE *f = std::fopen(json_path, "r");
  if (!f) {
    set_error(std::string("gemm_tuner_load: cannot open ") + json_path);
    return GEMM_STATUS_UNSUPPORTED;
  }
  char line[512];
  std::map<Key, int> table;
  double small = kDefaultSmallCost;
  while (std::fgets(line, sizeof line, f)) {
    const char *g = std::strstr(line, "\"grouped_small_cost\":");
    if (g) std::sscanf(g, "\"grouped_small_cost\": %lf", &small);
    int path, np, bm, bn, bk;
    char name[128];
    if (std::sscanf(line, " {\"path\": %d, \"n_products\": %d, \"log2_m\": %d, \"log2_n\": %d, \"log2_k\": %d, \"config\": \"%127[^\"]\"",
                    &path, &np, &bm, &bn, &bk, name) == 6) {
      if (path < GEMM_PATH_F32 || path > GEMM_PATH_FP8) continue;
      for (int c = 0; c < cfg_count(path); ++c)
        if (std::strcmp(cfg_name(path, c), name) == 0) table[Key(path, np, bm, bn, bk)] = c;
    }
  }
  std::fclose(f);
  std::lock_guard<std::mutex> lk(g_mu);
  g_table = table;
  g_small_cost = small;
  return GEMM_STATUS_OK;
}

void gemm_tuner_clear(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_table.clear();
  g_small_cost = kDefaultSmallCost;
}

}  // extern "C"
