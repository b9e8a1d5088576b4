// Autotuner of the level kernel's launch configuration (slimsell_autotune).
//
// The search space is the SlimChunk split length (Section III-D) and the
// MI355X launch shape.  Every configuration computes identical results, so
// the tuner only times them: BFS calls through the public entry points with
// event timing, median of a few repetitions, coordinate descent in two passes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "internal.h"

namespace ss {

namespace {

using ClassKey = std::tuple<int, int, int, int, int>;
std::mutex g_cache_mu;
std::map<ClassKey, ss_tune> g_cache;

ClassKey class_of(const Graph& g, int semiring, int batched) {
  const double n = (double)g.n;
  const double mean = g.n ? (double)g.entries / n : 0.0;
  const int log_n = (int)std::ceil(std::log2(std::max(2.0, n)));
  const int mean_b = (int)std::lround(2.0 * std::log2(std::max(1.0, mean)));
  const int skew_b = (int)std::lround(std::log2(std::max(1.0, (double)g.max_cl / std::max(1.0, mean))));
  return ClassKey(batched ? -1 : semiring, batched, log_n, mean_b, skew_b);
}

}  // namespace

// Time one configuration: median over repeats of the summed per-root BFS time.
static int time_config(ss_graph* gp, const ss_autotune_opts& o, const ss_tune& t, int32_t* dist,
                       int32_t* parent, float* rv, float* out_ms) {
  int rc = slimsell_tune_set(gp, &t);
  if (rc) return rc;
  const int reps = o.repeats > 0 ? o.repeats : 3;
  std::vector<ss_run_stats> rs((size_t)o.num_roots);
  std::vector<float> samples;
  ss_bfs_opts bo;
  std::memset(&bo, 0, sizeof(bo));
  bo.size = sizeof(bo);
  bo.slimwork = 2;
  bo.split_len = -1;
  bo.stream = o.stream;
  bo.flags = SS_STATS_TIME;
  bo.run_stats_out = rs.data();
  for (int r = -1; r < reps; ++r) {  // r = -1 warms up
    if (o.batched)
      rc = slimsell_bfs_batch(gp, o.roots, o.num_roots, &bo, dist);
    else
      rc = slimsell_bfs(gp, o.roots, o.num_roots, (ss_semiring)o.semiring, &bo, dist, parent, rv);
    if (rc) return rc;
    if (r < 0) continue;
    float sum = 0.f;
    for (const auto& x : rs) sum += x.bfs_ms;
    samples.push_back(sum);
  }
  std::sort(samples.begin(), samples.end());
  *out_ms = samples[samples.size() / 2];
  return SS_OK;
}

}  // namespace ss

using namespace ss;

extern "C" int slimsell_autotune(ss_graph* gp, const ss_autotune_opts* o, ss_autotune_result* res) {
  if (!gp || !o || !res) return set_error(SS_EINVAL, "NULL argument");
  if (o->size != sizeof(ss_autotune_opts)) return set_error(SS_EINVAL, "opts->size mismatch");
  if (o->num_roots < 1 || !o->roots) return set_error(SS_EINVAL, "need at least one root");
  if (!o->batched && (o->semiring < 0 || o->semiring > 3))
    return set_error(SS_EINVAL, "unknown semiring");
  if (o->batched && o->num_roots > 64) return set_error(SS_EINVAL, "batched: at most 64 roots");
  Graph& g = *gp;
  std::memset(res, 0, sizeof(*res));
  const ClassKey key = class_of(g, o->semiring, o->batched);
  if (!o->force) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
      int rc = slimsell_tune_set(gp, &it->second);
      if (rc) return rc;
      res->best = it->second;
      res->from_cache = 1;
      return SS_OK;
    }
  }
  (void)hipSetDevice(g.device);
  int32_t* dist = nullptr;
  int32_t* parent = nullptr;
  float* rv = nullptr;
  const size_t cells = (size_t)o->num_roots * (size_t)g.n;
  if (hipMalloc(&dist, sizeof(int32_t) * cells) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(SS_ENOMEM, "autotune: no device memory for outputs");
  }
  const ss_tune before = g.tune;
  int rc = SS_OK;
  float before_ms = 0.f;
  rc = time_config(gp, *o, before, dist, parent, rv, &before_ms);
  ss_tune best = before;
  float best_ms = before_ms;
  int evaluated = 1;
  // Coordinate descent stalls where two dimensions only pay together (no
  // SlimChunk split pays only with one workgroup per unit and no LDS
  // prefix on a union of small graphs), so it starts from the best of the
  // current configuration and a few seeds that differ in several at once.
  const ss_tune seeds[] = {
      {0, 16, 8, 0, 0, 0},     // whole chunks, a wavefront per chunk, no prefix
      {0, 4, 8, 0, 0, 0},      // the same in 4-wavefront workgroups
      {256, 16, 8, 0, 0, 64},  // 256-column pieces, a wavefront per piece
  };
  for (const ss_tune& t : seeds) {
    if (rc != SS_OK) break;
    if (std::memcmp(&t, &best, sizeof(ss_tune)) == 0) continue;
    float ms = 0.f;
    rc = time_config(gp, *o, t, dist, parent, rv, &ms);
    if (rc) break;
    ++evaluated;
    if (ms < best_ms) {
      best_ms = ms;
      best = t;
    }
  }
  const std::vector<int32_t> splits = {0, 64, 128, 256, 512, 1024, 2048, 4096};
  const std::vector<int32_t> waves = {1, 2, 4, 8, 16};
  const std::vector<int32_t> unrolls = {4, 8, 16};
  const std::vector<int32_t> groups = {0, 1024, 4096};
  const std::vector<int32_t> packs = {0, 32, 128};
  const std::vector<int32_t> stages = {0, 32, 64};
  for (int pass = 0; pass < 2 && rc == SS_OK; ++pass) {
    for (int dim = 0; dim < 6 && rc == SS_OK; ++dim) {
      const std::vector<int32_t>& vals = dim == 0   ? splits
                                         : dim == 1 ? waves
                                         : dim == 2 ? unrolls
                                         : dim == 3 ? groups
                                         : dim == 4 ? packs
                                                    : stages;
      for (int32_t v : vals) {
        ss_tune t = best;
        int32_t* field = dim == 0   ? &t.split_len
                         : dim == 1 ? &t.waves_per_group
                         : dim == 2 ? &t.unroll
                         : dim == 3 ? &t.max_groups
                         : dim == 4 ? &t.pack_cols
                                    : &t.lds_kib;
        if (*field == v) continue;
        *field = v;
        float ms = 0.f;
        rc = time_config(gp, *o, t, dist, parent, rv, &ms);
        if (rc) break;
        ++evaluated;
        if (ms < best_ms) {
          best_ms = ms;
          best = t;
        }
      }
    }
  }
  (void)hipFree(dist);
  if (rc) {
    (void)slimsell_tune_set(gp, &before);
    return rc;
  }
  rc = slimsell_tune_set(gp, &best);
  if (rc) return rc;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_cache[key] = best;
  }
  res->best = best;
  res->best_ms = best_ms;
  res->before_ms = before_ms;
  res->evaluated = evaluated;
  res->from_cache = 0;
  return SS_OK;
}
