// C ABI of libslimsell: graph construction/upload and the per-root BFS driver.
//
// The level loop runs on the host with a short look-ahead: level kernels are
// enqueued ahead of the one being waited on, and each level kernel reports
// the previous level's outcome to a host-mapped ring, so the host never
// waits for the stream to drain between levels.  A kernel launched past the
// last level sees that the level before it found nothing and exits at once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <immintrin.h>
#include <new>
#include <numeric>
#include <queue>
#include <string>
#include <thread>
#include <tuple>

#include "internal.h"

namespace ss {

static thread_local std::string g_last_error;

int set_error(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

static std::mutex g_model_mu;
static std::vector<float> g_model;
static uint64_t g_model_version = 0;  // 0 = no model
static uint64_t g_model_counter = 0;

bool sched_model(std::vector<float>* out, uint64_t* version) {
  std::lock_guard<std::mutex> lk(g_model_mu);
  if (g_model_version == 0) return false;
  *out = g_model;
  *version = g_model_version;
  return true;
}

static int hip_fail(hipError_t e, const char* what) {
  return set_error(SS_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define SS_HIP(call)                                   \
  do {                                                 \
    hipError_t _e = (call);                            \
    if (_e != hipSuccess) return hip_fail(_e, #call);  \
  } while (0)

template <class T>
static int dalloc(T** p, int64_t count) {
  *p = nullptr;
  if (count <= 0) count = 1;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * (size_t)count);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return set_error(SS_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  }
  return SS_OK;
}

static void release_units(UnitList& u) {
  if (u.d_units) (void)hipFree(u.d_units);
  if (u.d_pieces) (void)hipFree(u.d_pieces);
  if (u.d_bundle) (void)hipFree(u.d_bundle);
  if (u.d_arrive2) (void)hipFree(u.d_arrive2);
  for (auto& kv : u.assign) {
    if (kv.second.d_units) (void)hipFree(kv.second.d_units);
    if (kv.second.d_off) (void)hipFree(kv.second.d_off);
  }
  u.assign.clear();
  u.d_units = nullptr;
  u.d_pieces = nullptr;
  u.d_bundle = nullptr;
  u.d_arrive2 = nullptr;
}

static void release_graph(Graph* g) {
  if (!g) return;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(g->device);
  void* ptrs[] = {g->d_col,     g->d_cs,   g->d_cl,    g->d_v,     g->d_perm, g->d_deg,
                  g->d_scol,    g->d_sval,
                  g->ws.vec_a,  g->ws.vec_b, g->ws.state, g->ws.g, g->ws.d,
                  g->ws.rv,     g->ws.acc, g->ws.arrive, g->ws.done, g->ws.any, g->ws.counters,
                  g->d_voff,    g->bw.vis, g->bw.fa,   g->bw.fb,   g->bw.acc64,
                  g->bw.lvl,    g->bw.full, g->bw.root_rows, g->bw.slots,
                  g->ws.q[0],   g->ws.q[1], g->ws.qn,   g->ws.variant, g->ws.decided, g->ws.ring_ctr,
                  g->ws.sched_sums, g->ws.model, g->ws.sched_log, g->ws.bar, g->ws.pstatus,
                  g->ws.segs,   g->ws.seg_n, g->ws.summ};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  for (void* ev : g->ev_pool)
    if (ev) (void)hipEventDestroy(static_cast<hipEvent_t>(ev));
  if (g->ws.h_report) (void)hipHostFree(const_cast<uint64_t*>(g->ws.h_report));
  for (auto& kv : g->units) release_units(kv.second);
  (void)hipSetDevice(prev);
  delete g;
}

// Work units for split length `split` (0 = never split) with small chunks
// packed into runs of at most `pack` columns (0 = one chunk per unit).
// Chunks without columns are left out: their rows have no neighbours, so no
// product can change them and no gather reads them.  Built and uploaded on
// first use; with `lookup_only` a missing list is an error instead.
static int get_units(Graph& g, int32_t split, int32_t pack, UnitList** out,
                     bool lookup_only = false) {
  auto key = std::make_pair(split, pack);
  auto it = g.units.find(key);
  if (it != g.units.end()) {
    *out = &it->second;
    return SS_OK;
  }
  if (lookup_only)
    return set_error(SS_EINVAL, "no work units prepared for split_len " + std::to_string(split) +
                                    ", pack_cols " + std::to_string(pack) +
                                    " (slimsell_tune_set prepares the graph's configuration)");
  constexpr int32_t kMaxRun = 64;
  std::vector<Unit> units;
  std::vector<int32_t> pieces((size_t)g.n_chunks, 1);
  int64_t split_chunks = 0;
  const int64_t nc = g.n_chunks;
  int64_t i = 0;
  while (i < nc) {
    const int32_t len = g.h_cl[i];
    if (len == 0) { ++i; continue; }
    if (split > 0 && len > split) {
      const int32_t np = (len + split - 1) / split;
      for (int32_t q = 0; q < np; ++q)
        units.push_back(Unit{(int32_t)i, (int32_t)i + 1, q * split, std::min(len, (q + 1) * split)});
      pieces[i] = np;
      ++split_chunks;
      ++i;
    } else if (pack > 0) {
      const int64_t start = i;
      int64_t cols = 0;
      while (i < nc && g.h_cl[i] > 0 && (split <= 0 || g.h_cl[i] <= split) &&
             (i == start || cols + g.h_cl[i] <= pack) && i - start < kMaxRun) {
        cols += g.h_cl[i];
        ++i;
      }
      if (i - start == 1)
        units.push_back(Unit{(int32_t)start, (int32_t)start + 1, 0, g.h_cl[start]});
      else
        units.push_back(Unit{(int32_t)start, (int32_t)i, 0, 0});
    } else {
      units.push_back(Unit{(int32_t)i, (int32_t)i + 1, 0, len});
      ++i;
    }
  }
  // Longest units first, by powers of two: a level hands units to its
  // wavefronts round-robin (or the per-wavefront assignment takes them in
  // this order), so the long ones spread evenly over the grid and start
  // first, and the short ones fill in.  Within one power of two the units
  // keep chunk order, so neighbouring wavefronts work on neighbouring
  // chunks (the pieces of one chunk stay together, and in a union of graphs
  // a workgroup stays within one graph's vertices).
  auto cost = [&](const Unit& w) -> int64_t {
    if (w.c1 == w.c0 + 1) return (int64_t)w.j1 - w.j0;
    int64_t cols = 0;
    for (int32_t c = w.c0; c < w.c1; ++c) cols += g.h_cl[c];
    return cols;
  };
  auto octave = [&](const Unit& w) -> int {
    const int64_t c = cost(w);
    return c > 0 ? 63 - __builtin_clzll((unsigned long long)c) : -1;
  };
  std::stable_sort(units.begin(), units.end(),
                   [&](const Unit& x, const Unit& y) { return octave(x) > octave(y); });
  UnitList ul;
  ul.split_len = split;
  ul.pack_cols = pack;
  ul.h_units = units;
  ul.h_cols.resize(units.size());
  for (size_t i = 0; i < units.size(); ++i) ul.h_cols[i] = cost(units[i]);
  ul.count = (int64_t)units.size();
  ul.split_chunks = split_chunks;
  int rc = dalloc(&ul.d_units, std::max<int64_t>(1, ul.count));
  if (rc) return rc;
  rc = dalloc(&ul.d_pieces, std::max<int64_t>(1, nc));
  if (rc) { release_units(ul); return rc; }
  if (ul.count > 0) {
    hipError_t e = hipMemcpy(ul.d_units, units.data(), sizeof(Unit) * units.size(),
                             hipMemcpyHostToDevice);
    if (e != hipSuccess) { release_units(ul); return hip_fail(e, "upload units"); }
  }
  if (nc > 0) {
    hipError_t e = hipMemcpy(ul.d_pieces, pieces.data(), sizeof(int32_t) * (size_t)nc,
                             hipMemcpyHostToDevice);
    if (e != hipSuccess) { release_units(ul); return hip_fail(e, "upload pieces"); }
  }
  // arrival bundles of the split chunks
  std::vector<int32_t> bundle((size_t)std::max<int64_t>(nc, 1), 0);
  int64_t bundles = 0;
  for (int64_t c = 0; c < nc; ++c) {
    bundle[(size_t)c] = (int32_t)bundles;
    if (pieces[(size_t)c] > 1) bundles += (pieces[(size_t)c] + kBundle - 1) / kBundle;
  }
  ul.bundles = bundles;
  rc = dalloc(&ul.d_bundle, std::max<int64_t>(1, nc));
  if (!rc) rc = dalloc(&ul.d_arrive2, std::max<int64_t>(1, bundles));
  if (rc) { release_units(ul); return rc; }
  {
    hipError_t e = hipMemcpy(ul.d_bundle, bundle.data(), sizeof(int32_t) * bundle.size(),
                             hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemset(ul.d_arrive2, 0, sizeof(int32_t) * (size_t)std::max<int64_t>(1, bundles));
    if (e != hipSuccess) { release_units(ul); return hip_fail(e, "upload arrival bundles"); }
  }
  auto res = g.units.emplace(key, ul);
  *out = &res.first->second;
  return SS_OK;
}

// A unit's cost for the assignment: its columns plus a fixed per-unit cost
// (reading its descriptor, chunk extent and row states before the first
// column, and post-processing its rows), in columns: measured on R-MAT s22,
// a unit of a few columns keeps a wavefront about as long as ten columns of a
// long piece do.
constexpr int64_t kUnitCost = 12;

// Relative streaming speed of wavefront w of a grid whose workgroups of 16
// wavefronts run two per compute unit (n_cu compute units): a SIMD issues
// the memory instructions of its older wavefronts first, so the workgroups
// dispatched first, and inside a workgroup the wavefronts created first,
// progress faster while all compete.  Per-wavefront end times of the
// full-sweep levels on MI355X (R-MAT s22), measured with equal work and then
// twice again with the work weighted, gave these speeds, by dispatch round of the
// workgroup and the wavefront's rank on its SIMD; the sparser levels follow
// the same pattern.
static double slot_speed(int64_t w, int waves, int64_t n_cu) {
  static const double kSpeed[2][4] = {{1.0, 0.964, 0.925, 0.866}, {0.80, 0.702, 0.609, 0.516}};
  if (waves != 16 || n_cu <= 0) return 1.0;
  const int64_t round = (w / waves) / n_cu;
  const int rank = (int)(w % waves) / 4;
  return round < 2 ? kSpeed[round][rank] : kSpeed[1][3];
}

// The per-wavefront assignment of a unit list for a grid of W wavefronts in
// workgroups of `waves`: units, longest first, each to the wavefront that
// would finish it first given its work so far and its speed (the
// longest-processing-time rule for machines of different speeds).
static int get_assignment(UnitList& ul, int64_t W, int waves, int64_t n_cu,
                          const UnitList::Assignment** out, bool lookup_only) {
  *out = nullptr;
  const int64_t key = W * 32 + waves;
  auto it = ul.assign.find(key);
  if (it != ul.assign.end()) {
    *out = &it->second;
    return SS_OK;
  }
  if (lookup_only || W < 1 || W > INT32_MAX) return SS_OK;  // round-robin instead
  const std::vector<Unit>& units = ul.h_units;
  const int64_t n = (int64_t)units.size();
  // One heap of (work so far, tie order, wavefront) per speed class.  Ties
  // are broken by a multiplicative permutation of the wavefronts, so that
  // units of one kind (the long pieces come first) spread over the grid.
  int64_t mult = (int64_t)(0.6180339887 * (double)W) | 1;
  while (std::gcd(mult, W) != 1) mult += 2;
  using Load = std::tuple<int64_t, int64_t, int64_t>;
  using Heap = std::priority_queue<Load, std::vector<Load>, std::greater<Load>>;
  std::vector<double> speeds;
  std::vector<Heap> heaps;
  for (int64_t w = 0; w < W; ++w) {
    const double sp = slot_speed(w, waves, n_cu);
    size_t c = 0;
    while (c < speeds.size() && speeds[c] != sp) ++c;
    if (c == speeds.size()) {
      speeds.push_back(sp);
      heaps.emplace_back();
    }
    heaps[c].push({0, (int64_t)(((__int128)w * mult) % W), w});
  }
  std::vector<int32_t> owner((size_t)n);
  std::vector<int64_t> per((size_t)W + 1, 0);
  for (int64_t i = 0; i < n; ++i) {
    const int64_t cost = ul.h_cols[(size_t)i] + kUnitCost;
    size_t best = 0;
    double best_t = INFINITY;
    for (size_t c = 0; c < heaps.size(); ++c) {
      const double t = (double)(std::get<0>(heaps[c].top()) + cost) / speeds[c];
      if (t < best_t) {
        best_t = t;
        best = c;
      }
    }
    Load top = heaps[best].top();
    heaps[best].pop();
    owner[(size_t)i] = (int32_t)std::get<2>(top);
    ++per[(size_t)std::get<2>(top) + 1];
    heaps[best].push({std::get<0>(top) + cost, std::get<1>(top), std::get<2>(top)});
  }
  for (int64_t w = 0; w < W; ++w) per[(size_t)w + 1] += per[(size_t)w];
  std::vector<Unit> order((size_t)std::max<int64_t>(n, 1));
  std::vector<int64_t> fill(per.begin(), per.end() - 1);
  for (int64_t i = 0; i < n; ++i) order[(size_t)fill[(size_t)owner[(size_t)i]]++] = units[(size_t)i];
  std::vector<int32_t> off(per.begin(), per.end());
  UnitList::Assignment as;
  int rc = dalloc(&as.d_units, (int64_t)order.size());
  if (!rc) rc = dalloc(&as.d_off, W + 1);
  if (!rc && (hipMemcpy(as.d_units, order.data(), sizeof(Unit) * order.size(),
                        hipMemcpyHostToDevice) != hipSuccess ||
              hipMemcpy(as.d_off, off.data(), sizeof(int32_t) * off.size(),
                        hipMemcpyHostToDevice) != hipSuccess))
    rc = set_error(SS_EHIP, "upload of the unit assignment failed");
  if (rc) {
    if (as.d_units) (void)hipFree(as.d_units);
    if (as.d_off) (void)hipFree(as.d_off);
    return rc;
  }
  *out = &ul.assign.emplace(key, as).first->second;
  return SS_OK;
}

static int ensure_counters(Graph& g, int64_t words) {
  if (words <= g.ws.counter_words) return SS_OK;
  if (g.ws.counters) (void)hipFree(g.ws.counters);
  g.ws.counters = nullptr;
  g.ws.counter_words = 0;
  int rc = dalloc(&g.ws.counters, words);
  if (rc) return rc;
  g.ws.counter_words = words;
  return SS_OK;
}

// Events for SS_STATS_TIME come from a per-graph pool that grows on demand.
static int pool_event(Graph& g, size_t idx, hipEvent_t* out) {
  while (g.ev_pool.size() <= idx) {
    hipEvent_t ev = nullptr;
    SS_HIP(hipEventCreate(&ev));
    g.ev_pool.push_back(ev);
  }
  *out = static_cast<hipEvent_t>(g.ev_pool[idx]);
  return SS_OK;
}

static int alloc_workspace(Graph& g) {
  Workspace& ws = g.ws;
  ws.n_pad = g.n_pad;
  int rc;
  if ((rc = dalloc(reinterpret_cast<int32_t**>(&ws.vec_a), g.n_pad))) return rc;
  if ((rc = dalloc(reinterpret_cast<int32_t**>(&ws.vec_b), g.n_pad))) return rc;
  if ((rc = dalloc(&ws.state, g.n_pad))) return rc;
  if ((rc = dalloc(&ws.g, g.n_pad))) return rc;
  if ((rc = dalloc(&ws.d, g.n_pad))) return rc;
  if ((rc = dalloc(&ws.rv, g.n_pad))) return rc;
  if ((rc = dalloc(&ws.acc, g.n_pad))) return rc;
  if ((rc = dalloc(&ws.arrive, g.n_chunks))) return rc;
  SS_HIP(hipMemset(ws.arrive, 0, sizeof(int32_t) * (size_t)std::max<int64_t>(1, g.n_chunks)));
  if ((rc = dalloc(&ws.done, g.n_chunks))) return rc;
  if ((rc = dalloc(&ws.q[0], g.n_pad))) return rc;
  if ((rc = dalloc(&ws.q[1], g.n_pad))) return rc;
  if ((rc = dalloc(&ws.qn, kRing))) return rc;
  if ((rc = dalloc(&ws.variant, kRing))) return rc;
  if ((rc = dalloc(&ws.decided, kRing))) return rc;
  SS_HIP(hipMemset(ws.decided, 0, sizeof(uint64_t) * kRing));
  if ((rc = dalloc(&ws.ring_ctr, (int64_t)kRing * kRingSlots * kCountFields))) return rc;
  if ((rc = dalloc(&ws.sched_sums, 8))) return rc;
  if ((rc = dalloc(&ws.model, kModelCap))) return rc;
  ws.sched_log_cap = std::min<int64_t>((int64_t)g.n + 2, 65536);
  if ((rc = dalloc(&ws.sched_log, ws.sched_log_cap * 12))) return rc;
  // segments of long frontier rows: at most one per frontier row plus one per
  // 1024 cells of the graph
  ws.seg_cap = (int64_t)g.n_pad + g.entries / 1024 + 64;
  if ((rc = dalloc(&ws.segs, ws.seg_cap))) return rc;
  if ((rc = dalloc(&ws.seg_n, 2))) return rc;
  SS_HIP(hipMemset(ws.seg_n, 0, sizeof(int32_t) * 2));
  if ((rc = dalloc(&ws.bar, 2))) return rc;
  if ((rc = dalloc(&ws.pstatus, 4))) return rc;
  if ((rc = dalloc(&ws.any, kRing))) return rc;
  SS_HIP(hipMemset(ws.any, 0, sizeof(uint64_t) * kRing));
  // frontier summaries (one bit per chunk, three buffers) where they are small
  // enough to sit in LDS beside the staged prefix
  const int64_t summ_words = (g.n_chunks + 31) / 32;
  if (summ_words * 4 <= kSummMaxBytes) {
    // three summaries, then one word per summary: whether its level wrote it
    if ((rc = dalloc(&ws.summ, 3 * summ_words + 4))) return rc;
    ws.summ_words = (int32_t)summ_words;
  }
  void* h = nullptr;
  hipError_t e = hipHostMalloc(&h, sizeof(uint64_t) * (kRing + 1),
                               hipHostMallocMapped | hipHostMallocCoherent);
  if (e != hipSuccess) return hip_fail(e, "hipHostMalloc(report ring)");
  std::memset(h, 0, sizeof(uint64_t) * kRing);
  static_cast<uint64_t*>(h)[kRing] = 1;  // a graph's first learned run stages its model up front
  ws.h_report = static_cast<volatile uint64_t*>(h);
  void* dptr = nullptr;
  SS_HIP(hipHostGetDevicePointer(&dptr, h, 0));
  ws.d_report = static_cast<uint64_t*>(dptr);
  return SS_OK;
}

// Wait until the level kernel after `level` has reported `level`'s outcome.
static int wait_report(Graph& g, int32_t level, uint32_t run_id, hipStream_t st, bool* found) {
  const uint64_t tag = ((uint64_t)run_id << 32) | (uint32_t)level;
  volatile uint64_t* slot = &g.ws.h_report[level % kRing];
  uint64_t spins = 0;
  for (;;) {
    uint64_t v = *slot;
    if ((v >> 1) == tag) {
      *found = (v & 1) != 0;
      return SS_OK;
    }
    if ((++spins & 1023) == 0) {
      hipError_t e = hipStreamQuery(st);
      if (e == hipSuccess) {
        v = *slot;
        if ((v >> 1) == tag) {
          *found = (v & 1) != 0;
          return SS_OK;
        }
        return set_error(SS_EHIP, "level report missing after the stream drained");
      }
      if (e != hipErrorNotReady) return hip_fail(e, "level kernel");
    }
    _mm_pause();
  }
}


ss_bfs_opts default_opts() {
  ss_bfs_opts d;
  std::memset(&d, 0, sizeof(d));
  d.size = sizeof(d);
  d.slimwork = 2;
  d.split_len = -1;
  return d;
}

uint32_t next_run_id(Graph& g) {
  g.run_id = (g.run_id >= 0x7FFFFFF0u) ? 1u : g.run_id + 1;
  return g.run_id;
}

// Validated launch parameters of one call (shared by single-root and batched BFS).
struct RunPlan {
  int waves = 4, unroll = 8;
  int64_t max_groups = 0, cap = 0, lcap = 0, words_per_run = 0;
  bool timing = false, counting = false, persistent = false, sell = false;
  bool level_events = false;  // timing: events around every level launch too
  bool summ = false;          // frontier summaries filter the gathers (plain runs)
  int32_t filter_limit = 0;   // most flagged chunks for which a level filters
  int32_t prefix_words = 0;   // summary words covering the chunks of the LDS prefix
  int32_t slimwork = 2;
  int32_t schedule = 0;
  bool sched_lazy = false;    // the learned schedule stages its model only inside the box
  uint32_t lds_bytes = 0;
  UnitList* ul = nullptr;
  const UnitList::Assignment* as = nullptr;  // per-wavefront units of the level launch
  UnitList* vul[kPullVariants] = {nullptr, nullptr, nullptr};  // pull variants
  const UnitList::Assignment* vas[kPullVariants] = {nullptr, nullptr, nullptr};
  bool has_model = false;
  int32_t n_anchors = 0;  // training-domain anchors carried by the model
  float tau = 0.f;
};

// Per-call record of what was launched, for the statistics epilogue.
struct RunLog {
  explicit RunLog(size_t runs)
      : ev_first(runs, 0), ev_last(runs, 0), ev_dp(runs, 0), dp(runs, 0), launches(runs, 0),
        iters(runs, 0) {}
  size_t next_ev = 0;
  std::vector<size_t> ev_first;  // event before the run's first kernel
  std::vector<size_t> ev_last;   // event after its last kernel
  std::vector<size_t> ev_dp;     // first of the two events around its DP sweep (timing)
  std::vector<char> dp;          // whether the run ended with the DP transformation
  std::vector<int32_t> launches;
  std::vector<int32_t> iters;
};

// With `no_alloc`, only what allocates nothing is accepted: no statistics,
// schedule, persistent launch or Sell-C-sigma comparator, and work units that
// already exist.
static int plan_run(Graph& g, const ss_bfs_opts* o, int policy, int32_t runs,
                    int64_t default_cap, hipStream_t st, RunPlan* p, bool no_alloc = false) {
  if (o->size != sizeof(ss_bfs_opts)) return set_error(SS_EINVAL, "opts->size mismatch");
  if (no_alloc && ((o->flags & ~SS_NO_SUMMARY) || o->schedule || o->level_stats_out ||
                   o->run_stats_out))
    return set_error(SS_EINVAL,
                     "the allocation-free BFS takes no statistics, schedule, persistent launch "
                     "or comparator (flags may hold SS_NO_SUMMARY only)");
  if (o->slimwork < 0 || o->slimwork > 2) return set_error(SS_EINVAL, "slimwork must be 0, 1 or 2");
  p->waves = o->waves_per_group ? o->waves_per_group : g.tune.waves_per_group;
  if (p->waves != 1 && p->waves != 2 && p->waves != 4 && p->waves != 8 && p->waves != 16)
    return set_error(SS_EINVAL, "waves_per_group must be 1, 2, 4, 8 or 16");
  int32_t split = o->split_len;
  if (split < -1) return set_error(SS_EINVAL, "split_len must be >= -1");
  if (split == -1) split = g.tune.split_len;
  const int32_t pack = g.tune.pack_cols < 0 ? (split > 0 ? split : 0) : g.tune.pack_cols;
  p->unroll = g.tune.unroll;
  p->max_groups = g.tune.max_groups;
  p->cap = (o->max_levels > 0) ? std::min<int64_t>(o->max_levels, default_cap) : default_cap;
  if (o->level_cap < 0) return set_error(SS_EINVAL, "level_cap < 0");
  if (o->flags &
      ~(SS_STATS_TIME | SS_STATS_COUNTERS | SS_RUN_PERSISTENT | SS_SELL_VAL | SS_STATS_TIME_BFS |
        SS_NO_SUMMARY | SS_SCHED_LAZY))
    return set_error(SS_EINVAL, "bad flags");
  p->sched_lazy = (o->flags & SS_SCHED_LAZY) != 0;
  p->persistent = (o->flags & SS_RUN_PERSISTENT) != 0;
  p->sell = (o->flags & SS_SELL_VAL) != 0;
  if (p->sell && (p->persistent || o->schedule || policy == kBatchSemiring))
    return set_error(SS_EINVAL, "SS_SELL_VAL runs plain single-root levels only");
  if (p->sell && !g.d_scol) {
    // Sell-C-sigma arrays, built once per graph
    SS_HIP(hipMalloc(&g.d_scol, sizeof(int32_t) * std::max<int64_t>(g.cells, 1)));
    SS_HIP(hipMalloc(&g.d_sval, sizeof(int32_t) * std::max<int64_t>(g.cells, 1)));
    int brc = launch_sell_build(g.d_col, g.cells, g.d_scol, g.d_sval, st);
    if (brc) return brc;
  }
  p->slimwork = o->slimwork;
  p->lds_bytes = 0;
  if (g.tune.lds_kib > 0) {
    // bytes of the gathered vector each policy reads, rounded down to 16
    const int64_t used = policy == SS_BOOLEAN     ? g.n_pad
                         : policy == SS_SELMAX    ? g.n_pad / 8
                         : policy == kBatchSemiring ? g.n_pad * 8
                                                  : g.n_pad * 4;
    p->lds_bytes = (uint32_t)(std::min<int64_t>(used, (int64_t)g.tune.lds_kib * 1024) / 16 * 16);
  }
  if (o->schedule < 0 || o->schedule > 3 + kVariants - 1)
    return set_error(SS_EINVAL, "schedule must be 0..6");
  // Plain runs (single-root and batched) keep one summary bit per chunk of
  // each level's frontier and skip the gathers of chunks without frontier
  // rows.  Push levels of a scheduled run do not maintain it.
  p->summ = g.ws.summ && !o->schedule &&
            !(o->flags & SS_NO_SUMMARY) &&
            (int64_t)p->lds_bytes + 4 * (int64_t)g.ws.summ_words <= g.lds_dev;
  if (p->summ) {
    // The filter skips the memory gathers of unflagged chunks but puts an
    // LDS round trip before the others, so it pays while the terms it can
    // skip are many: (share of terms outside the LDS prefix) x (share of
    // unflagged chunks) at least kFilterTau.  The first share follows from
    // the row degrees (a symmetric matrix: row r is the column of deg(r)
    // cells) and the rows the prefix holds for this semiring's element size.
    constexpr double kFilterTau = 1.0 / 16;
    const int64_t rows = policy == SS_SELMAX    ? (int64_t)p->lds_bytes * 8
                         : policy == SS_BOOLEAN ? (int64_t)p->lds_bytes
                         : policy == kBatchSemiring ? (int64_t)p->lds_bytes / 8
                                                    : (int64_t)p->lds_bytes / 4;
    const int64_t nc = g.n_chunks;
    const int64_t in_chunks = std::min<int64_t>(rows / kC, nc);
    // chunks with rows in the prefix (a partly covered one included)
    const int64_t cover = std::min<int64_t>((rows + kC - 1) / kC, nc);
    p->prefix_words = (int32_t)((cover + 31) / 32);
    const double total = nc > 0 ? (double)g.h_chunk_deg[(size_t)nc] : 0.0;
    const double outside = total > 0 ? 1.0 - (double)g.h_chunk_deg[(size_t)in_chunks] / total : 0.0;
    const double frac = outside > kFilterTau ? 1.0 - kFilterTau / outside : 0.0;
    // the share of unflagged chunks counts chunks that have rows with
    // neighbours (a chunk of isolated rows is never flagged)
    int64_t nonempty = 0;
    for (int32_t len : g.h_cl) nonempty += len > 0 ? 1 : 0;
    p->filter_limit = (int32_t)std::floor(frac * (double)nonempty);
  }
  if (o->schedule && o->slimwork != 2) return set_error(SS_EINVAL, "scheduling needs slimwork = 2");
  p->schedule = o->schedule;
  int rc = get_units(g, split, pack, &p->ul, no_alloc);
  if (rc) return rc;
  // the level launch's grid, and its per-wavefront assignment of the units
  // (an allocation-free call uses a prepared one or none)
  {
    const int64_t W = level_groups(p->ul->count, p->waves, p->max_groups) * p->waves;
    // with no more units than wavefronts each takes one (or none): no table
    if (W < p->ul->count &&
        (rc = get_assignment(*p->ul, W, p->waves, g.n_cu, &p->as, no_alloc)))
      return rc;
  }
  if (p->schedule) {
    const int32_t vsplit[kPullVariants] = {0, 256, 1024};
    int64_t most = 0;
    for (int v = 0; v < kPullVariants; ++v) {
      if ((rc = get_units(g, vsplit[v], 0, &p->vul[v]))) return rc;
      most = std::max(most, p->vul[v]->count);
    }
    // the scheduled level's grid serves the variant with the most units;
    // each variant's units get their assignment for that grid
    const int64_t Ws = level_groups(most, p->waves, p->max_groups) * p->waves;
    for (int v = 0; v < kPullVariants; ++v)
      if (Ws < p->vul[v]->count &&
          (rc = get_assignment(*p->vul[v], Ws, p->waves, g.n_cu, &p->vas[v], false)))
        return rc;
    std::vector<float> host;
    uint64_t version = 0;
    p->has_model = (p->schedule == 1) && sched_model(&host, &version);
    if (p->has_model && g.ws.model_version != version) {
      SS_HIP(hipMemcpy(g.ws.model, host.data(), sizeof(float) * host.size(),
                       hipMemcpyHostToDevice));
      g.ws.model_version = version;
    }
    p->n_anchors = p->has_model && (int64_t)host.size() > kModelSize
                       ? (int32_t)host[kModelSize + 1] : 0;
    p->tau = p->n_anchors ? host[kModelSize] : 0.f;
  }
  p->timing = (o->flags & (SS_STATS_TIME | SS_STATS_TIME_BFS)) != 0;
  p->level_events = (o->flags & SS_STATS_TIME) && !(o->flags & SS_STATS_TIME_BFS);
  p->lcap = o->level_cap;
  p->counting = (o->flags & SS_STATS_COUNTERS) && p->lcap > 0 && o->level_stats_out;
  // levels 0..lcap, then one block for the DP transformation's sweep
  p->words_per_run = (p->lcap + 2) * kCountSlots * kCountFields;
  if (p->counting) {
    rc = ensure_counters(g, p->words_per_run * runs);
    if (rc) return rc;
    rc = launch_fill_u64(g.ws.counters, 0ull, p->words_per_run * runs, st);
    if (rc) return rc;
  }
  return SS_OK;
}

static int mark_event(Graph& g, const RunPlan& p, size_t& next_ev, hipStream_t st,
                      size_t* first) {
  if (!p.timing) return SS_OK;
  if (first) *first = next_ev;
  hipEvent_t ev;
  int rc = pool_event(g, next_ev++, &ev);
  if (rc) return rc;
  SS_HIP(hipEventRecord(ev, st));
  return SS_OK;
}

static LevelArgs base_args(Graph& g, const Workspace& ws, const RunPlan& p, const ss_bfs_opts* o,
                           uint32_t run, int32_t run_idx) {
  LevelArgs a;
  std::memset(&a, 0, sizeof(a));
  a.col = p.sell ? g.d_scol : g.d_col;
  a.val = p.sell ? g.d_sval : nullptr;
  a.cs = g.d_cs;
  a.cl = g.d_cl;
  a.v = g.d_v;
  a.deg = g.d_deg;
  a.units = p.ul->d_units;
  a.pieces = p.ul->d_pieces;
  a.n_units = p.ul->count;
  a.bundle = p.ul->d_bundle;
  a.arrive2 = p.ul->d_arrive2;
  a.piece_cols = p.ul->split_len;
  if (p.as) {
    a.units = p.as->d_units;
    a.wave_off = p.as->d_off;
  }
  a.state = ws.state;
  a.g = ws.g;
  a.d = ws.d;
  a.rv = ws.rv;
  a.acc = ws.acc;
  a.arrive = ws.arrive;
  a.done = ws.done;
  a.any = ws.any;
  a.counters = p.counting ? g.ws.counters + p.words_per_run * run_idx : nullptr;
  a.report = g.ws.d_report;
  a.run_id = run;
  a.n_pad = (uint32_t)g.n_pad;
  a.slimwork = p.slimwork;
  a.lds_bytes = p.lds_bytes;
  a.summ = p.summ ? ws.summ : nullptr;
  a.summ_words = ws.summ_words;
  a.filter_limit = p.filter_limit;
  a.prefix_words = p.prefix_words;
  if (p.schedule) {
    a.variant = g.ws.variant;
    for (int v = 0; v < kPullVariants; ++v) {
      a.vunits[v] = p.vas[v] ? p.vas[v]->d_units : p.vul[v]->d_units;
      a.vwave_off[v] = p.vas[v] ? p.vas[v]->d_off : nullptr;
      a.vpieces[v] = p.vul[v]->d_pieces;
      a.vn_units[v] = p.vul[v]->count;
      a.vbundle[v] = p.vul[v]->d_bundle;
      a.varrive2[v] = p.vul[v]->d_arrive2;
      a.vpiece_cols[v] = p.vul[v]->split_len;
    }
    a.qn = g.ws.qn;
    a.ring_ctr = g.ws.ring_ctr;
    a.segs = g.ws.segs;
    a.seg_n = g.ws.seg_n;
  }
  (void)o;
  return a;
}

// A scheduled run writes frontier queues, queue lengths, push segments and
// ring counters: refuse to launch one with any of them missing.
static int check_sched_args(const LevelArgs& a) {
  if (!a.variant || !a.qn || !a.ring_ctr || !a.segs || !a.seg_n)
    return set_error(SS_EHIP, "internal: scheduled run without its queue buffers");
  for (int v = 0; v < kPullVariants; ++v)
    if (!a.vunits[v] || !a.vpieces[v] || !a.vbundle[v] || !a.varrive2[v])
      return set_error(SS_EHIP, "internal: scheduled run without its work units");
  return SS_OK;
}

// The level loop of one BFS run: level kernels are enqueued kLookahead ahead
// of the level being waited on; the run ends at the first level that
// discovers nothing.
// Schedule parameters that stay fixed over one run.
static SchedLaunch sched_launch(const Graph& g, const RunPlan& p) {
  SchedLaunch sl;
  std::memset(&sl, 0, sizeof(sl));
  sl.any = g.ws.any;
  sl.report = g.ws.d_report;
  sl.variant = g.ws.variant;
  sl.decided = g.ws.decided;
  // The learned schedule stages its model in every workgroup before it
  // knows whether the level needs it; on a graph whose levels all fell
  // outside the model's domain last time, it stages it only for a level
  // inside the domain.  The word is read and cleared between runs: the
  // levels of the previous run have all finished by then (the host saw its
  // last report).
  if (p.schedule == 1 && p.has_model) {
    sl.eager = (!p.sched_lazy && g.ws.h_report[kRing] != 0) ? 1 : 0;
    g.ws.h_report[kRing] = 0;
    sl.in_box = g.ws.d_report + kRing;
  }
  sl.qn = g.ws.qn;
  sl.seg_n = g.ws.seg_n;
  sl.ring_ctr = g.ws.ring_ctr;
  sl.sums = g.ws.sched_sums;
  sl.model = p.has_model ? g.ws.model : nullptr;
  sl.anchors = p.n_anchors ? g.ws.model + kModelSize + 2 : nullptr;
  sl.box = p.n_anchors ? g.ws.model + kModelSize + 2 + (int64_t)p.n_anchors * kFeatures : nullptr;
  sl.cells = sl.box ? sl.box + 2 * kFeatures : nullptr;
  sl.n_anchors = p.n_anchors;
  sl.tau2 = p.tau * p.tau;
  sl.log = g.ws.sched_log;
  sl.log_cap = (int32_t)g.ws.sched_log_cap;
  sl.mode = p.schedule;
  sl.heuristic_pull = g.tune.split_len == 0 ? 0 : (g.tune.split_len <= 512 ? 1 : 2);
  sl.n = (double)g.n;
  sl.two_m = (double)g.entries;
  return sl;
}

static int run_persistent(Graph& g, const RunPlan& p, int policy, LevelArgs a, void* buf_a,
                          void* buf_b, hipStream_t st, RunLog* log, int32_t run_idx) {
  int rc;
  if ((rc = launch_fill_i32(reinterpret_cast<int32_t*>(g.ws.bar), 0, 2, st))) return rc;
  if ((rc = launch_fill_i32(g.ws.pstatus, 0, 4, st))) return rc;
  const int32_t lcap = (int32_t)std::min<int64_t>(p.lcap, INT32_MAX);
  if ((rc = launch_fill_i32(g.ws.pstatus + 2, lcap, 1, st))) return rc;
  int rate_khz = 0;
  if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, g.device) != hipSuccess ||
      rate_khz <= 0)
    rate_khz = 100000;
  const uint64_t limit = (uint64_t)rate_khz * 1000ull * 5ull;  // 5 s per barrier wait
  a.count_stats = p.counting ? 1 : 0;
  a.wave_off = nullptr;  // the persistent grid deals the units round-robin
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (p.level_events) {
    if ((rc = pool_event(g, log->next_ev++, &e0))) return rc;
    if ((rc = pool_event(g, log->next_ev++, &e1))) return rc;
    SS_HIP(hipEventRecord(e0, st));
  }
  if (p.schedule && (rc = check_sched_args(a))) return rc;
  const SchedLaunch sl = sched_launch(g, p);
  if (p.schedule && (!sl.sums || !sl.seg_n || !g.ws.q[0] || !g.ws.q[1]))
    return set_error(SS_EHIP, "internal: scheduled run without its queue buffers");
  PersistentRun pr;
  pr.cap = (int32_t)std::min<int64_t>(p.cap, INT32_MAX);
  pr.max_groups = p.max_groups;
  pr.bar = g.ws.bar;
  pr.status = g.ws.pstatus;
  pr.limit = limit;
  pr.sched = p.schedule ? &sl : nullptr;
  pr.q0 = g.ws.q[0];
  pr.q1 = g.ws.q[1];
  rc = launch_persistent(policy, p.unroll, a, buf_a, buf_b, pr, st);
  if (rc) return rc;
  if (p.level_events) SS_HIP(hipEventRecord(e1, st));
  int32_t status[4] = {0, 0, 0, 0};
  SS_HIP(hipMemcpyAsync(status, g.ws.pstatus, sizeof(status), hipMemcpyDeviceToHost, st));
  SS_HIP(hipStreamSynchronize(st));
  if (status[1]) return set_error(SS_EHIP, "persistent kernel: a level barrier timed out");
  if (status[0] < 0) return set_error(SS_EITER, "level cap reached before the BFS finished");
  log->iters[run_idx] = status[0];
  log->launches[run_idx] = 1;
  return SS_OK;
}

static int run_levels(Graph& g, const RunPlan& p, int policy, LevelArgs a, void* buf_a,
                      void* buf_b, hipStream_t st, RunLog* log, int32_t run_idx) {
  if (p.persistent) return run_persistent(g, p, policy, a, buf_a, buf_b, st, log, run_idx);
  constexpr int kLookahead = 2;
  int32_t launched = 0;
  const SchedLaunch sl = sched_launch(g, p);
  if (p.schedule) {
    int rc = check_sched_args(a);
    if (rc) return rc;
  }
  auto launch = [&](int32_t k) -> int {
    a.level = k;
    a.vin = (k & 1) ? buf_a : buf_b;
    a.vout = (k & 1) ? buf_b : buf_a;
    a.q_in = g.ws.q[(k - 1) & 1];
    a.q_out = g.ws.q[k & 1];
    a.segs = g.ws.segs;
    a.seg_n = g.ws.seg_n + (k & 1);
    a.count_stats = (p.counting && k <= p.lcap) ? 1 : 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (p.level_events) {
      int pr;
      if ((pr = pool_event(g, log->next_ev++, &e0))) return pr;
      if ((pr = pool_event(g, log->next_ev++, &e1))) return pr;
      SS_HIP(hipEventRecord(e0, st));
    }
    int lr;
    if (p.schedule) {
      LevelArgs pa = a;
      int64_t most = 0;
      for (int v = 0; v < kPullVariants; ++v) most = std::max(most, pa.vn_units[v]);
      pa.n_units = most;  // grid size only: the kernel uses its variant's units
      if ((lr = launch_sched_level(policy, p.waves, p.unroll, p.max_groups, pa, sl, st)))
        return lr;
      if ((lr = launch_push(policy, a, g.max_cl > kPushLaneMax, st))) return lr;
    } else {
      if ((lr = launch_level(policy, p.waves, p.unroll, p.max_groups, a, st))) return lr;
    }
    if (p.level_events) SS_HIP(hipEventRecord(e1, st));
    return SS_OK;
  };
  for (int32_t j = 1;; ++j) {
    while (launched < j + kLookahead && launched <= p.cap) {
      int rc = launch(++launched);
      if (rc) return rc;
    }
    bool found = false;
    int rc = wait_report(g, j, a.run_id, st, &found);
    if (rc) return rc;
    if (!found) {
      log->iters[run_idx] = j;
      break;
    }
    if (j >= p.cap) {
      (void)hipStreamSynchronize(st);
      return set_error(SS_EITER, "level cap reached before the BFS finished");
    }
  }
  log->launches[run_idx] = launched;
  return SS_OK;
}

// Statistics epilogue: wait for the stream, then fill run and level records.
static int collect_stats(Graph& g, const ss_bfs_opts* o, const RunPlan& p, int32_t runs,
                         const RunLog& log, hipStream_t st) {
  const bool want_levels = o->level_stats_out && p.lcap > 0;
  if (!(p.timing || p.counting || o->run_stats_out || want_levels)) return SS_OK;
  SS_HIP(hipStreamSynchronize(st));
  std::vector<unsigned long long> h;
  if (p.counting) {
    h.resize((size_t)(p.words_per_run * runs));
    SS_HIP(hipMemcpy(h.data(), g.ws.counters, sizeof(unsigned long long) * h.size(),
                     hipMemcpyDeviceToHost));
  }
  auto ev = [&](size_t i) { return static_cast<hipEvent_t>(g.ev_pool[i]); };
  std::vector<float> hlog;  // schedule log of the last run (variants per level)
  if (p.schedule && want_levels && runs == 1) {
    const int64_t nl = std::min<int64_t>(std::min<int64_t>(p.lcap, log.iters[0]), g.ws.sched_log_cap);
    hlog.resize((size_t)nl * 12);
    if (nl > 0)
      SS_HIP(hipMemcpy(hlog.data(), g.ws.sched_log, sizeof(float) * hlog.size(),
                       hipMemcpyDeviceToHost));
  }
  for (int32_t r = 0; r < runs; ++r) {
    float kernel_ms = 0.f, bfs_ms = 0.f;
    std::vector<float> lvl_ms((size_t)log.launches[r], 0.f);
    float dp_ms = 0.f;
    if (p.timing) {
      const size_t e = log.ev_first[r];
      if (p.level_events) {
        for (int32_t k = 0; k < log.launches[r]; ++k) {
          float ms = 0.f;
          SS_HIP(hipEventElapsedTime(&ms, ev(e + 1 + 2 * k), ev(e + 2 + 2 * k)));
          lvl_ms[k] = ms;
          kernel_ms += ms;
        }
        if (p.persistent) std::fill(lvl_ms.begin(), lvl_ms.end(), 0.f);  // one launch, all levels
      }
      SS_HIP(hipEventElapsedTime(&bfs_ms, ev(e), ev(log.ev_last[r])));
      if (log.dp[r])
        SS_HIP(hipEventElapsedTime(&dp_ms, ev(log.ev_dp[r]), ev(log.ev_dp[r] + 1)));
    }
    if (o->run_stats_out) {
      ss_run_stats& rs = o->run_stats_out[r];
      std::memset(&rs, 0, sizeof(rs));
      rs.iterations = log.iters[r];
      rs.launches = log.launches[r];
      rs.kernel_ms = kernel_ms;
      rs.bfs_ms = bfs_ms;
      rs.dp_ms = dp_ms;
      if (p.counting && log.dp[r]) {
        // the DP sweep's block sits behind the levels (see words_per_run)
        const unsigned long long* base =
            h.data() + p.words_per_run * r + (p.lcap + 1) * kCountSlots * kCountFields;
        for (int q = 0; q < kCountSlots; ++q) {
          rs.dp_chunks += (int64_t)base[q * kCountFields + 1];
          rs.dp_cells += (int64_t)base[q * kCountFields + 2];
        }
      }
    }
    if (want_levels) {
      for (int64_t k = 1; k <= p.lcap; ++k) {
        ss_level_stats& ls = o->level_stats_out[r * p.lcap + (k - 1)];
        std::memset(&ls, 0, sizeof(ls));
        if (k > log.iters[r]) continue;
        ls.ms = (p.level_events && k - 1 < (int64_t)lvl_ms.size()) ? lvl_ms[k - 1] : 0.f;
        ls.variant = -1;
        if (p.schedule && k <= (int64_t)hlog.size() / 12) ls.variant = (int32_t)hlog[(k - 1) * 12 + 10];
        if (p.counting) {
          const unsigned long long* base = h.data() + p.words_per_run * r;
          for (int q = 0; q < kCountSlots; ++q) {
            const unsigned long long* f = base + (k * kCountSlots + q) * kCountFields;
            ls.discovered += (int64_t)f[0];
            ls.active_chunks += (int64_t)f[1];
            ls.active_cells += (int64_t)f[2];
            ls.max_active_cl = std::max<int64_t>(ls.max_active_cl, (int64_t)f[3]);
            ls.frontier_edges += (int64_t)f[4];
          }
        }
      }
    }
  }
  return SS_OK;
}

static int ensure_batch_workspace(Graph& g, int64_t roots,
                                  const std::vector<unsigned long long>& full_per_graph,
                                  hipStream_t st) {
  BatchWorkspace& b = g.bw;
  int rc;
  if (!b.vis) {
    b.n_pad = g.n_pad;
    if ((rc = dalloc(&b.vis, g.n_pad))) return rc;
    if ((rc = dalloc(&b.fa, g.n_pad))) return rc;
    if ((rc = dalloc(&b.fb, g.n_pad))) return rc;
    if ((rc = dalloc(&b.acc64, g.n_pad))) return rc;
    if ((rc = dalloc(&b.lvl, g.n_pad * 64))) return rc;
    if ((rc = dalloc(&b.full, g.n_chunks))) return rc;
  }
  if (roots > b.root_cap) {
    if (b.root_rows) (void)hipFree(b.root_rows);
    if (b.slots) (void)hipFree(b.slots);
    b.root_rows = b.slots = nullptr;
    b.root_cap = 0;
    if ((rc = dalloc(&b.root_rows, roots))) return rc;
    if ((rc = dalloc(&b.slots, roots))) return rc;
    b.root_cap = roots;
  }
  std::vector<unsigned long long> full((size_t)g.n_chunks, 0ull);
  for (int32_t i = 0; i < g.num_graphs; ++i)
    for (int64_t c = g.h_roff[i] / kC; c < g.h_roff[i + 1] / kC; ++c) full[c] = full_per_graph[i];
  SS_HIP(hipMemcpyAsync(b.full, full.data(), sizeof(unsigned long long) * full.size(),
                        hipMemcpyHostToDevice, st));
  // the host vector must outlive the copy
  SS_HIP(hipStreamSynchronize(st));
  return SS_OK;
}


// ------------------------------------------------ allocation-free BFS state
//
// slimsell_bfs_noalloc keeps the per-call BFS workspace (frontier vectors,
// row states, distances, SlimChunk combine buffers, level tags, frontier
// summaries) in one file-scope device array instead of the graph's
// workspace, so a call allocates nothing.  Every GPU the library runs on
// holds its own copy for the life of the process; host code uses only the
// address hipGetSymbolAddress returns for the current device, never the
// array's name (which is a host-side stand-in).
constexpr int64_t kScratchBytes = 64ll << 20;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kScratchDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kScratchDevices];

// Address of this device's scratch, looked up once per device (the device
// must be current).
static int scratch_address(int device, uint8_t** out) {
  if (device < 0 || device >= kScratchDevices)
    return set_error(SS_EUNSUP, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return set_error(SS_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[device] = ptr;
  }
  *out = static_cast<uint8_t*>(g_scratch_ptr[device]);
  return SS_OK;
}

// The workspace of one allocation-free call on graph g, carved from `base` in
// 256-byte aligned pieces (base == nullptr: sizes only).  Only the buffers
// the semiring touches are carved (the DP transformation adds distances and
// their codes); returns the bytes used.
static int64_t carve_workspace(const Graph& g, int semiring, bool dp, uint8_t* base,
                               Workspace* w) {
  int64_t off = 0;
  auto take = [&](int64_t bytes) -> void* {
    void* p = base ? base + off : nullptr;
    off += (std::max<int64_t>(bytes, 1) + 255) / 256 * 256;
    return p;
  };
  const int64_t n = g.n_pad, nc = std::max<int64_t>(g.n_chunks, 1);
  *w = Workspace();
  w->n_pad = n;
  w->any = static_cast<uint64_t*>(take(8 * (int64_t)kRing));
  w->arrive = static_cast<int32_t*>(take(4 * nc));
  w->done = static_cast<uint8_t*>(take(nc));
  if (g.ws.summ) {
    w->summ = static_cast<uint32_t*>(take(4 * (3 * (int64_t)g.ws.summ_words + 4)));
    w->summ_words = g.ws.summ_words;
  }
  w->acc = static_cast<int32_t*>(take(4 * n));
  switch (semiring) {
    case SS_TROPICAL:
      w->state = static_cast<int32_t*>(take(4 * n));
      break;
    case SS_REAL:
      w->vec_a = take(4 * n);
      w->vec_b = take(4 * n);
      w->g = static_cast<uint8_t*>(take(n));
      w->d = static_cast<int32_t*>(take(4 * n));
      w->rv = static_cast<float*>(take(4 * n));
      break;
    case SS_BOOLEAN:
      w->vec_a = take(n);
      w->vec_b = take(n);
      w->g = static_cast<uint8_t*>(take(n));
      w->d = static_cast<int32_t*>(take(4 * n));
      break;
    default:  // SS_SELMAX: one 64-bit frontier word per chunk
      w->vec_a = take(8 * nc);
      w->vec_b = take(8 * nc);
      w->state = static_cast<int32_t*>(take(4 * n));
      w->g = static_cast<uint8_t*>(take(n));
      w->d = static_cast<int32_t*>(take(4 * n));
      break;
  }
  if (dp && semiring == SS_TROPICAL) {
    // row distances and their 2-bit codes (n / 4 bytes); the other
    // semirings have both buffers already
    w->d = static_cast<int32_t*>(take(4 * n));
    w->g = static_cast<uint8_t*>(take(n / 4));
  }
  if (dp && !w->state) w->state = static_cast<int32_t*>(take(4 * n));  // best v per row
  // the graph's host-mapped report ring (part of the graph, not scratch)
  w->h_report = g.ws.h_report;
  w->d_report = g.ws.d_report;
  return off;
}

}  // namespace ss

using namespace ss;


extern "C" {

const char* slimsell_last_error(void) { return g_last_error.c_str(); }

const char* slimsell_version(void) { return "slimsell-mi355x 0.1 (gfx950)"; }

int slimsell_sched_load(const float* w, int64_t count) {
  if (!w || count < kModelSize)
    return set_error(SS_EINVAL, "the scheduler model has 1412 parameters");
  if (count > kModelSize) {
    // training domain: tau, K, K anchors of 6 features
    const float tau = count >= kModelSize + 2 ? w[kModelSize] : -1.f;
    const float kf = count >= kModelSize + 2 ? w[kModelSize + 1] : -1.f;
    if (!(tau > 0.f) || !std::isfinite(tau) || !(kf >= 1.f) || kf > (float)kMaxAnchors ||
        kf != std::floor(kf) || count != kModelSize + 2 + (int64_t)kf * kFeatures)
      return set_error(SS_EINVAL,
                       "model domain must be tau > 0, K in 1..1024, then K x 6 features");
    for (int64_t i = kModelSize + 2; i < count; ++i)
      if (!std::isfinite(w[i])) return set_error(SS_EINVAL, "model anchors must be finite");
  }
  std::vector<float> m(w, w + count);
  if (count > kModelSize) {
    // the anchors' box widened by tau, plus a relative margin that keeps
    // the float distance of any level outside it above tau^2 after rounding
    const float tau = w[kModelSize];
    const int64_t K = (count - kModelSize - 2) / kFeatures;
    float lo[kFeatures], hi[kFeatures];
    for (int f = 0; f < kFeatures; ++f) {
      lo[f] = INFINITY;
      hi[f] = -INFINITY;
      for (int64_t a = 0; a < K; ++a) {
        const float x = w[kModelSize + 2 + a * kFeatures + f];
        lo[f] = std::min(lo[f], x);
        hi[f] = std::max(hi[f], x);
      }
      const float r = tau * 1.001f + 1e-6f * std::max(std::fabs(lo[f]), std::fabs(hi[f]));
      lo[f] -= r;
      hi[f] += r;
    }
    m.insert(m.end(), lo, lo + kFeatures);
    m.insert(m.end(), hi, hi + kFeatures);
    // the cell map: a level's cell is floor((x - lo) * scale) per feature,
    // clamped to the bins, in single precision on the device; the cells an
    // anchor's cube touches are taken a thousandth of a bin wider on each
    // side, so no rounding of that product can put a level within tau of
    // the anchor into a cell left clear
    float scale[kFeatures];
    for (int f = 0; f < kFeatures; ++f) scale[f] = (float)kCellBins / (hi[f] - lo[f]);
    uint32_t bits[kCellWords] = {};
    for (int64_t a = 0; a < K; ++a) {
      int b0[kFeatures], b1[kFeatures];
      for (int f = 0; f < kFeatures; ++f) {
        const double x = w[kModelSize + 2 + a * kFeatures + f];
        const double r = (double)tau * 1.001 + 1e-6 * std::max(std::fabs(lo[f]), std::fabs(hi[f]));
        const double u0 = (x - r - lo[f]) * scale[f] - 1e-3, u1 = (x + r - lo[f]) * scale[f] + 1e-3;
        b0[f] = (int)std::min<double>(std::max<double>(std::floor(u0), 0.0), kCellBins - 1);
        b1[f] = (int)std::min<double>(std::max<double>(std::floor(u1), 0.0), kCellBins - 1);
      }
      int q[kFeatures];
      for (int f = 0; f < kFeatures; ++f) q[f] = b0[f];
      for (;;) {  // every cell of the product of the ranges
        int idx = 0;
        for (int f = kFeatures - 1; f >= 0; --f) idx = idx * kCellBins + q[f];
        bits[idx >> 5] |= 1u << (idx & 31);
        int f = 0;
        while (f < kFeatures && q[f] == b1[f]) q[f] = b0[f], ++f;
        if (f == kFeatures) break;
        ++q[f];
      }
    }
    m.insert(m.end(), scale, scale + kFeatures);
    for (int i = 0; i < kCellWords; ++i) {
      float v;
      std::memcpy(&v, &bits[i], sizeof(v));  // the words travel as raw bits
      m.push_back(v);
    }
  }
  std::lock_guard<std::mutex> lk(g_model_mu);
  g_model.swap(m);
  g_model_version = ++g_model_counter;
  return SS_OK;
}

int slimsell_sched_clear(void) {
  std::lock_guard<std::mutex> lk(g_model_mu);
  g_model.clear();
  g_model_version = 0;
  return SS_OK;
}

int slimsell_layout_build(const int32_t* src, const int32_t* dst, int64_t m, int32_t n, int32_t C,
                          int32_t sigma, ss_layout** out) {
  if (!out) return set_error(SS_EINVAL, "out is NULL");
  *out = nullptr;
  Layout* L = nullptr;
  int rc = build_layout(src, dst, m, n, C, sigma, &L);
  if (rc) return rc;
  // ss_layout adds nothing to Layout; move the contents into the ABI type
  ss_layout* h = new (std::nothrow) ss_layout();
  if (!h) { delete L; return set_error(SS_ENOMEM, "host allocation failed"); }
  static_cast<Layout&>(*h) = std::move(*L);
  delete L;
  *out = h;
  return SS_OK;
}

int slimsell_layout_view(const ss_layout* L, ss_layout_view* v) {
  if (!L || !v) return set_error(SS_EINVAL, "NULL argument");
  v->n = L->n;
  v->n_pad = L->n_pad;
  v->C = kC;
  v->sigma = L->sigma;
  v->n_chunks = L->n_chunks;
  v->entries = L->entries;
  v->cells = L->cells;
  v->max_cl = L->max_cl;
  v->pad0 = 0;
  v->col = L->col.data();
  v->cs = L->cs.data();
  v->cl = L->cl.data();
  v->v = L->v.data();
  v->perm = L->perm.data();
  v->degree = L->degree.data();
  return SS_OK;
}

void slimsell_layout_free(ss_layout* L) { delete L; }

int slimsell_build_from_layout(const ss_layout* L, void* stream, ss_graph** out) {
  if (!L || !out) return set_error(SS_EINVAL, "NULL argument");
  *out = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev < 1) {
    (void)hipGetLastError();
    return set_error(SS_EUNSUP, "no HIP device available");
  }
  ss_graph* g = new (std::nothrow) ss_graph();
  if (!g) return set_error(SS_ENOMEM, "host allocation failed");
  (void)hipGetDevice(&g->device);
  {
    // dynamic LDS a kernel may ask for: the device's limit, at most 64 KiB
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, g->device) !=
            hipSuccess ||
        lds < 0)
      lds = 0;
    g->lds_cap = std::min(lds, 64 * 1024);
    g->lds_dev = lds;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g->device) != hipSuccess)
      cus = 0;
    g->n_cu = cus;  // 0: the unit assignment treats every wavefront alike
  }
  g->n = L->n;
  g->n_pad = L->n_pad;
  g->sigma = L->sigma;
  g->n_chunks = L->n_chunks;
  g->entries = L->entries;
  g->cells = L->cells;
  g->max_cl = L->max_cl;
  g->h_perm = L->perm;
  g->h_cl = L->cl;
  g->num_graphs = 1;
  g->h_voff = {0, (int64_t)L->n};
  g->h_roff = {0, (int64_t)L->n_pad};
  g->h_degree.resize((size_t)L->n);
  for (int32_t o = 0; o < L->n; ++o) g->h_degree[o] = L->degree[L->perm[o]];
  g->h_chunk_deg.assign((size_t)L->n_chunks + 1, 0);
  for (int64_t c = 0; c < L->n_chunks; ++c) {
    int64_t sum = 0;
    for (int64_t r = c * kC; r < (c + 1) * kC && r < (int64_t)L->degree.size(); ++r)
      sum += L->degree[(size_t)r];
    g->h_chunk_deg[(size_t)c + 1] = g->h_chunk_deg[(size_t)c] + sum;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  int rc = SS_OK;
  auto up = [&](auto** dst, const auto& vec) -> int {
    using T = std::remove_reference_t<decltype(vec[0])>;
    int r = dalloc(reinterpret_cast<std::remove_const_t<T>**>(dst), (int64_t)vec.size());
    if (r) return r;
    if (!vec.empty()) {
      hipError_t ee = hipMemcpyAsync(*dst, vec.data(), sizeof(T) * vec.size(),
                                     hipMemcpyHostToDevice, st);
      if (ee != hipSuccess) return hip_fail(ee, "upload layout");
    }
    return SS_OK;
  };
  if (!rc) rc = up(&g->d_col, L->col);
  if (!rc) rc = up(&g->d_cs, L->cs);
  if (!rc) rc = up(&g->d_cl, L->cl);
  if (!rc) rc = up(&g->d_v, L->v);
  if (!rc) rc = up(&g->d_perm, L->perm);
  if (!rc) rc = up(&g->d_deg, L->degree);
  if (!rc) {
    hipError_t ee = hipStreamSynchronize(st);
    if (ee != hipSuccess) rc = hip_fail(ee, "upload layout");
  }
  if (!rc) rc = alloc_workspace(*g);
  if (!rc) {
    // the default configuration's work units (the allocation-free BFS needs them)
    UnitList* ul = nullptr;
    const int32_t sp = g->tune.split_len;
    const int32_t pack = g->tune.pack_cols < 0 ? (sp > 0 ? sp : 0) : g->tune.pack_cols;
    rc = get_units(*g, g->tune.split_len, pack, &ul);
    const UnitList::Assignment* as = nullptr;
    const int w = g->tune.waves_per_group;
    const int64_t W = level_groups(ul ? ul->count : 0, w, g->tune.max_groups) * w;
    if (!rc && W < ul->count) rc = get_assignment(*ul, W, w, g->n_cu, &as, false);
  }
  if (!rc) rc = dalloc(&g->d_voff, 2);
  if (!rc && hipMemcpy(g->d_voff, g->h_voff.data(), sizeof(int64_t) * 2, hipMemcpyHostToDevice) !=
                 hipSuccess)
    rc = set_error(SS_EHIP, "upload graph offsets");
  if (rc) {
    release_graph(g);
    return rc;
  }
  *out = g;
  return SS_OK;
}

int slimsell_build(const int32_t* src, const int32_t* dst, int64_t m, int32_t n, int32_t C,
                   int32_t sigma, void* stream, ss_graph** out) {
  if (!out) return set_error(SS_EINVAL, "out is NULL");
  *out = nullptr;
  ss_layout* L = nullptr;
  int rc = slimsell_layout_build(src, dst, m, n, C, sigma, &L);
  if (rc) return rc;
  rc = slimsell_build_from_layout(L, stream, out);
  slimsell_layout_free(L);
  return rc;
}

int slimsell_graph_info(const ss_graph* g, int64_t* n, int64_t* entries, int64_t* padding,
                        int64_t* chunks, int64_t* max_cl) {
  if (!g) return set_error(SS_EINVAL, "graph is NULL");
  if (n) *n = g->n;
  if (entries) *entries = g->entries;
  if (padding) *padding = g->cells - g->entries;
  if (chunks) *chunks = g->n_chunks;
  if (max_cl) *max_cl = g->max_cl;
  return SS_OK;
}

int slimsell_tune_set(ss_graph* g, const ss_tune* t) {
  if (!g || !t) return set_error(SS_EINVAL, "NULL argument");
  const int w = t->waves_per_group;
  if (t->split_len < 0) return set_error(SS_EINVAL, "split_len must be >= 0");
  if (w != 1 && w != 2 && w != 4 && w != 8 && w != 16)
    return set_error(SS_EINVAL, "waves_per_group must be 1, 2, 4, 8 or 16");
  if (t->unroll != 4 && t->unroll != 8 && t->unroll != 16)
    return set_error(SS_EINVAL, "unroll must be 4, 8 or 16");
  if (t->max_groups < 0) return set_error(SS_EINVAL, "max_groups must be >= 0");
  if (t->pack_cols < -1) return set_error(SS_EINVAL, "pack_cols must be >= -1");
  if (t->lds_kib != 0 && t->lds_kib != 16 && t->lds_kib != 32 && t->lds_kib != 64)
    return set_error(SS_EINVAL, "lds_kib must be 0, 16, 32 or 64");
  std::lock_guard<std::mutex> lock(g->mu);
  g->tune = *t;
  // the work units of the configuration, so that the allocation-free BFS
  // finds them
  SS_HIP(hipSetDevice(g->device));
  UnitList* ul = nullptr;
  const int32_t sp = t->split_len;
  int rc = get_units(*g, sp, t->pack_cols < 0 ? (sp > 0 ? sp : 0) : t->pack_cols, &ul);
  const UnitList::Assignment* as = nullptr;
  if (!rc) {
    const int64_t W = level_groups(ul->count, w, t->max_groups) * w;
    if (W < ul->count) rc = get_assignment(*ul, W, w, g->n_cu, &as, false);
  }
  return rc;
}

int slimsell_tune_get(const ss_graph* g, ss_tune* t) {
  if (!g || !t) return set_error(SS_EINVAL, "NULL argument");
  *t = g->tune;
  return SS_OK;
}

int slimsell_graph_degrees(const ss_graph* g, int32_t* degree) {
  if (!g || !degree) return set_error(SS_EINVAL, "NULL argument");
  std::memcpy(degree, g->h_degree.data(), sizeof(int32_t) * g->h_degree.size());
  return SS_OK;
}

void slimsell_free(ss_graph* g) { release_graph(g); }

int slimsell_sync(void* stream) {
  hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  return SS_OK;
}

int slimsell_bfs(ss_graph* gp, const int32_t* roots, int32_t num_roots, ss_semiring s,
                 const ss_bfs_opts* o, int32_t* dist, int32_t* parent, float* real_val) {
  if (!gp) return set_error(SS_EINVAL, "graph is NULL");
  Graph& g = *gp;
  if (num_roots < 0) return set_error(SS_EINVAL, "num_roots < 0");
  if (num_roots == 0) return SS_OK;
  if (!roots || !dist) return set_error(SS_EINVAL, "roots and dist are required");
  if ((int)s < 0 || (int)s > 3) return set_error(SS_EINVAL, "unknown semiring");
  if (real_val && s != SS_REAL) return set_error(SS_EINVAL, "real_val needs SS_REAL");
  for (int32_t r = 0; r < num_roots; ++r)
    if (roots[r] < 0 || roots[r] >= g.n) return set_error(SS_EINVAL, "root out of range [0, n)");
  ss_bfs_opts def = default_opts();
  if (!o) o = &def;
  std::lock_guard<std::mutex> lock(g.mu);
  SS_HIP(hipSetDevice(g.device));
  hipStream_t st = static_cast<hipStream_t>(o->stream);
  RunPlan plan;
  int rc = plan_run(g, o, (int)s, num_roots, (int64_t)g.n + 1, st, &plan);
  if (rc) return rc;
  RunLog log((size_t)num_roots);
  for (int32_t r = 0; r < num_roots; ++r) {
    const uint32_t run = next_run_id(g);
    if ((rc = mark_event(g, plan, log.next_ev, st, &log.ev_first[r]))) return rc;
    rc = launch_init(s, g, g.ws, g.h_perm[roots[r]], plan.summ, st);
    if (rc) return rc;
    if (plan.schedule && (rc = launch_sched_init(g, g.ws, g.h_perm[roots[r]], st))) return rc;
    LevelArgs a = base_args(g, g.ws, plan, o, run, r);
    if (plan.schedule) g.ws.sched_log_levels = 0;  // the log is rewritten by this run
    rc = run_levels(g, plan, (int)s, a, g.ws.vec_a, g.ws.vec_b, st, &log, r);
    if (rc) return rc;
    if (plan.schedule)
      g.ws.sched_log_levels = std::min<int64_t>(log.iters[r], g.ws.sched_log_cap);
    if (o->iterations_out) o->iterations_out[r] = log.iters[r];
    int32_t* dist_r = dist + (int64_t)r * g.n;
    int32_t* parent_r = parent ? parent + (int64_t)r * g.n : nullptr;
    // the other semirings get parents by the DP transformation (Section II-C),
    // whose last pass also writes the distances unless real values are wanted
    const bool dp = parent_r && s != SS_SELMAX;
    if (!dp || real_val) {
      rc = launch_finalise(s, g, g.ws, dist_r, s == SS_SELMAX ? parent_r : nullptr,
                           real_val ? real_val + (int64_t)r * g.n : nullptr, st);
      if (rc) return rc;
    }
    if (dp) {
      hipEvent_t e0 = nullptr, e1 = nullptr;
      log.dp[r] = 1;
      if (plan.timing) {
        log.ev_dp[r] = log.next_ev;
        if ((rc = pool_event(g, log.next_ev++, &e0))) return rc;
        if ((rc = pool_event(g, log.next_ev++, &e1))) return rc;
      }
      // its counters go to the block behind the run's levels, addressed as
      // level 1 by the sweep
      unsigned long long* dpc =
          plan.counting ? g.ws.counters + plan.words_per_run * r + plan.lcap * kCountSlots * kCountFields
                        : nullptr;
      const int32_t src = s == SS_TROPICAL ? kDpFromTropical : kDpFromRowD;
      if ((rc = launch_dp(g, g.ws, *plan.ul, plan.as, plan.unroll, plan.waves, plan.max_groups,
                          nullptr, src, real_val ? nullptr : dist_r, parent_r, st, dpc, e0, e1)))
        return rc;
    }
    if ((rc = mark_event(g, plan, log.next_ev, st, &log.ev_last[r]))) return rc;
  }
  return collect_stats(g, o, plan, num_roots, log, st);
}

int slimsell_dp_parents(ss_graph* gp, const int32_t* dist, int32_t num_roots, int32_t* parent,
                        void* stream) {
  if (!gp) return set_error(SS_EINVAL, "graph is NULL");
  if (num_roots < 0) return set_error(SS_EINVAL, "num_roots < 0");
  if (num_roots == 0) return SS_OK;
  if (!dist || !parent) return set_error(SS_EINVAL, "dist and parent are required");
  Graph& g = *gp;
  std::lock_guard<std::mutex> lock(g.mu);
  SS_HIP(hipSetDevice(g.device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int32_t split = g.tune.split_len;
  const int32_t pack = g.tune.pack_cols < 0 ? (split > 0 ? split : 0) : g.tune.pack_cols;
  UnitList* ul = nullptr;
  int rc = get_units(g, split, pack, &ul);
  if (rc) return rc;
  const int w = g.tune.waves_per_group;
  const int64_t W = level_groups(ul->count, w, g.tune.max_groups) * w;
  const UnitList::Assignment* as = nullptr;
  if (W < ul->count && (rc = get_assignment(*ul, W, w, g.n_cu, &as, false))) return rc;
  for (int32_t r = 0; r < num_roots; ++r) {
    rc = launch_dp(g, g.ws, *ul, as, g.tune.unroll, g.tune.waves_per_group, g.tune.max_groups,
                   dist + (int64_t)r * g.n, kDpFromDist, nullptr, parent + (int64_t)r * g.n, st);
    if (rc) return rc;
  }
  return SS_OK;
}

int slimsell_bfs_batch(ss_graph* gp, const int32_t* roots, int32_t rpg, const ss_bfs_opts* o,
                       int32_t* dist) {
  if (!gp) return set_error(SS_EINVAL, "graph is NULL");
  Graph& g = *gp;
  if (rpg < 1 || rpg > 64) return set_error(SS_EINVAL, "roots_per_graph must be in 1..64");
  if (!roots || !dist) return set_error(SS_EINVAL, "roots and dist are required");
  std::vector<int32_t> root_rows, slots;
  std::vector<unsigned long long> full((size_t)g.num_graphs, 0ull);
  for (int32_t i = 0; i < g.num_graphs; ++i) {
    const int64_t ni = g.h_voff[i + 1] - g.h_voff[i];
    for (int32_t b = 0; b < rpg; ++b) {
      const int32_t r = roots[(int64_t)i * rpg + b];
      if (r == -1) continue;
      if (r < 0 || r >= ni) return set_error(SS_EINVAL, "root out of range of its graph");
      root_rows.push_back(g.h_perm[g.h_voff[i] + r]);
      slots.push_back(b);
      full[i] |= 1ull << b;
    }
  }
  ss_bfs_opts def = default_opts();
  if (!o) o = &def;
  std::lock_guard<std::mutex> lock(g.mu);
  SS_HIP(hipSetDevice(g.device));
  hipStream_t st = static_cast<hipStream_t>(o->stream);
  RunPlan plan;
  if (o->schedule) return set_error(SS_EINVAL, "batched BFS has no per-level schedule");
  int rc = plan_run(g, o, kBatchSemiring, 1, std::min<int64_t>((int64_t)g.n + 1, 65534), st,
                    &plan);
  if (rc) return rc;
  if ((rc = ensure_batch_workspace(g, (int64_t)root_rows.size(), full, st))) return rc;
  BatchWorkspace& bw = g.bw;
  if (!root_rows.empty()) {
    SS_HIP(hipMemcpyAsync(bw.root_rows, root_rows.data(), sizeof(int32_t) * root_rows.size(),
                          hipMemcpyHostToDevice, st));
    SS_HIP(hipMemcpyAsync(bw.slots, slots.data(), sizeof(int32_t) * slots.size(),
                          hipMemcpyHostToDevice, st));
  }
  RunLog log(1);
  const uint32_t run = next_run_id(g);
  if ((rc = mark_event(g, plan, log.next_ev, st, &log.ev_first[0]))) return rc;
  rc = launch_batch_init(g, bw, (int32_t)root_rows.size(), plan.summ, st);
  if (rc) return rc;
  LevelArgs a = base_args(g, g.ws, plan, o, run, 0);
  a.acc64 = bw.acc64;
  a.vis = bw.vis;
  a.full = bw.full;
  a.lvl = bw.lvl;
  rc = run_levels(g, plan, kBatchSemiring, a, bw.fa, bw.fb, st, &log, 0);
  if (rc) return rc;
  if (o->iterations_out) o->iterations_out[0] = log.iters[0];
  rc = launch_batch_finalise(g, bw, rpg, dist, st);
  if (rc) return rc;
  if ((rc = mark_event(g, plan, log.next_ev, st, &log.ev_last[0]))) return rc;
  return collect_stats(g, o, plan, 1, log, st);
}

int slimsell_sched_log(const ss_graph* g, float* out, int32_t cap, int32_t* levels) {
  if (!g || !out || cap < 0) return set_error(SS_EINVAL, "bad argument");
  const int64_t nl = std::min<int64_t>(cap, g->ws.sched_log_levels);
  if (nl > 0)
    SS_HIP(hipMemcpy(out, g->ws.sched_log, sizeof(float) * (size_t)nl * 12, hipMemcpyDeviceToHost));
  if (levels) *levels = (int32_t)nl;
  return SS_OK;
}

int slimsell_graph_parts(const ss_graph* g, int32_t* num_graphs, int64_t* n_per_graph,
                         int64_t* vertex_offset) {
  if (!g || !num_graphs) return set_error(SS_EINVAL, "NULL argument");
  *num_graphs = g->num_graphs;
  for (int32_t i = 0; i < g->num_graphs; ++i) {
    if (n_per_graph) n_per_graph[i] = g->h_voff[i + 1] - g->h_voff[i];
    if (vertex_offset) vertex_offset[i] = g->h_voff[i];
  }
  return SS_OK;
}

int slimsell_build_multi(int32_t num_graphs, const int64_t* edge_offsets, const int32_t* src,
                         const int32_t* dst, const int32_t* n_per_graph, int32_t C,
                         int32_t sigma, void* stream, ss_graph** out) {
  if (!out) return set_error(SS_EINVAL, "out is NULL");
  *out = nullptr;
  if (num_graphs < 1 || !edge_offsets || !n_per_graph)
    return set_error(SS_EINVAL, "num_graphs >= 1 with edge_offsets and n_per_graph required");
  ss_layout U;
  std::vector<int64_t> voff((size_t)num_graphs + 1, 0), roff((size_t)num_graphs + 1, 0);
  for (int32_t i = 0; i < num_graphs; ++i) {
    if (n_per_graph[i] < 1) return set_error(SS_EINVAL, "every graph needs n >= 1");
    const int64_t e0 = edge_offsets[i], e1 = edge_offsets[i + 1];
    if (e0 < 0 || e1 < e0) return set_error(SS_EINVAL, "edge_offsets must be non-decreasing");
    Layout* L = nullptr;
    int rc = build_layout(src ? src + e0 : nullptr, dst ? dst + e0 : nullptr, e1 - e0,
                          n_per_graph[i], C, sigma == 0 ? 0 : std::min(sigma, n_per_graph[i]), &L);
    if (rc) return rc;
    voff[i + 1] = voff[i] + L->n;
    roff[i + 1] = roff[i] + L->n_pad;
    if (roff[i + 1] > INT32_MAX) { delete L; return set_error(SS_EINVAL, "union too large"); }
    const int32_t ro = (int32_t)roff[i];
    const int64_t cell0 = U.cells;
    for (int32_t c : L->col) U.col.push_back(c < 0 ? -1 : c + ro);
    if (U.cs.empty()) U.cs.push_back(0);
    for (int64_t k = 1; k < (int64_t)L->cs.size(); ++k) U.cs.push_back(cell0 + L->cs[k]);
    U.cl.insert(U.cl.end(), L->cl.begin(), L->cl.end());
    for (int32_t x : L->v) U.v.push_back(x == 0 ? 0 : (int32_t)(x + voff[i]));
    for (int32_t r : L->perm) U.perm.push_back(r + ro);
    U.degree.insert(U.degree.end(), L->degree.begin(), L->degree.end());
    U.cells += L->cells;
    U.entries += L->entries;
    U.max_cl = std::max(U.max_cl, L->max_cl);
    delete L;
  }
  U.n = (int32_t)voff[num_graphs];
  U.n_pad = (int32_t)roff[num_graphs];
  U.n_chunks = U.n_pad / kC;
  U.sigma = sigma;
  ss_graph* g = nullptr;
  int rc = slimsell_build_from_layout(&U, stream, &g);
  if (rc) return rc;
  g->num_graphs = num_graphs;
  g->h_voff = voff;
  g->h_roff = roff;
  if (g->d_voff) (void)hipFree(g->d_voff);
  g->d_voff = nullptr;
  rc = dalloc(&g->d_voff, num_graphs + 1);
  if (!rc && hipMemcpy(g->d_voff, voff.data(), sizeof(int64_t) * voff.size(),
                       hipMemcpyHostToDevice) != hipSuccess)
    rc = set_error(SS_EHIP, "upload graph offsets");
  if (!rc && num_graphs > 1) {
    // A union's levels are active in some graphs and idle in others, which a
    // static assignment of units cannot foresee: one wavefront per unit
    // (eight per workgroup), so that the dispatcher balances the level, and
    // the eight-column sweep without an LDS prefix (256 ER graphs: 12.4
    // against 18.0 ms per batch with the single-graph default).
    const ss_tune t{128, 8, 8, 0, 0, 0};
    rc = slimsell_tune_set(g, &t);
  }
  if (rc) { slimsell_free(g); return rc; }
  *out = g;
  return SS_OK;
}

int slimsell_bfs_noalloc(ss_graph* gp, const int32_t* roots, int32_t num_roots, ss_semiring s,
                         const ss_bfs_opts* o, int32_t* dist, int32_t* parent, float* real_val) {
  if (!gp) return set_error(SS_EINVAL, "graph is NULL");
  Graph& g = *gp;
  if (num_roots < 0) return set_error(SS_EINVAL, "num_roots < 0");
  if (num_roots == 0) return SS_OK;
  if (!roots || !dist) return set_error(SS_EINVAL, "roots and dist are required");
  if ((int)s < 0 || (int)s > 3) return set_error(SS_EINVAL, "unknown semiring");
  if (real_val && s != SS_REAL) return set_error(SS_EINVAL, "real_val needs SS_REAL");
  for (int32_t r = 0; r < num_roots; ++r)
    if (roots[r] < 0 || roots[r] >= g.n) return set_error(SS_EINVAL, "root out of range [0, n)");
  const bool dp = parent && s != SS_SELMAX;
  Workspace w;
  const int64_t need = carve_workspace(g, (int)s, dp, nullptr, &w);
  if (need > kScratchBytes)
    return set_error(SS_EINVAL, "the allocation-free BFS needs " + std::to_string(need) +
                                    " bytes of scratch for this graph and semiring; the limit is " +
                                    std::to_string(kScratchBytes));
  ss_bfs_opts def = default_opts();
  if (!o) o = &def;
  std::lock_guard<std::mutex> lock(g.mu);
  SS_HIP(hipSetDevice(g.device));
  uint8_t* base = nullptr;
  int rc = scratch_address(g.device, &base);
  if (rc) return rc;
  (void)carve_workspace(g, (int)s, dp, base, &w);
  hipStream_t st = static_cast<hipStream_t>(o->stream);
  RunPlan plan;
  if ((rc = plan_run(g, o, (int)s, num_roots, (int64_t)g.n + 1, st, &plan, true))) return rc;
  // level tags carry the graph's run counter, and other graphs share this
  // scratch: start from a clean ring (a fill kernel, not a memset node)
  if ((rc = launch_fill_u64(reinterpret_cast<unsigned long long*>(w.any), 0ull, kRing, st)))
    return rc;
  RunLog log((size_t)num_roots);
  for (int32_t r = 0; r < num_roots; ++r) {
    const uint32_t run = next_run_id(g);
    if ((rc = launch_init(s, g, w, g.h_perm[roots[r]], plan.summ, st))) return rc;
    LevelArgs a = base_args(g, w, plan, o, run, r);
    if ((rc = run_levels(g, plan, (int)s, a, w.vec_a, w.vec_b, st, &log, r))) return rc;
    if (o->iterations_out) o->iterations_out[r] = log.iters[r];
    int32_t* dist_r = dist + (int64_t)r * g.n;
    int32_t* parent_r = parent ? parent + (int64_t)r * g.n : nullptr;
    // with the DP transformation, its last pass writes the distances too
    if (!dp || real_val) {
      rc = launch_finalise(s, g, w, dist_r, s == SS_SELMAX ? parent_r : nullptr,
                           real_val ? real_val + (int64_t)r * g.n : nullptr, st);
      if (rc) return rc;
    }
    if (dp && (rc = launch_dp(g, w, *plan.ul, plan.as, plan.unroll, plan.waves, plan.max_groups,
                              nullptr, s == SS_TROPICAL ? kDpFromTropical : kDpFromRowD,
                              real_val ? nullptr : dist_r, parent_r, st)))
      return rc;
  }
  return SS_OK;
}

}  // extern "C"
