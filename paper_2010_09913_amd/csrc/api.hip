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
#include <cstring>
#include <immintrin.h>
#include <new>
#include <string>
#include <thread>

#include "internal.h"

namespace ss {

static thread_local std::string g_last_error;

int set_error(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
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
  u.d_units = nullptr;
  u.d_pieces = nullptr;
}

static void release_graph(Graph* g) {
  if (!g) return;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(g->device);
  void* ptrs[] = {g->d_col,     g->d_cs,   g->d_cl,    g->d_v,     g->d_perm, g->d_deg,
                  g->ws.vec_a,  g->ws.vec_b, g->ws.state, g->ws.g, g->ws.d,
                  g->ws.rv,     g->ws.acc, g->ws.arrive, g->ws.any, g->ws.counters};
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
// product can change them and no gather reads them.
static int get_units(Graph& g, int32_t split, int32_t pack, UnitList** out) {
  auto key = std::make_pair(split, pack);
  auto it = g.units.find(key);
  if (it != g.units.end()) {
    *out = &it->second;
    return SS_OK;
  }
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
  UnitList ul;
  ul.split_len = split;
  ul.pack_cols = pack;
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
  auto res = g.units.emplace(key, ul);
  *out = &res.first->second;
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
  if ((rc = dalloc(&ws.any, kRing))) return rc;
  SS_HIP(hipMemset(ws.any, 0, sizeof(uint64_t) * kRing));
  void* h = nullptr;
  hipError_t e = hipHostMalloc(&h, sizeof(uint64_t) * kRing,
                               hipHostMallocMapped | hipHostMallocCoherent);
  if (e != hipSuccess) return hip_fail(e, "hipHostMalloc(report ring)");
  std::memset(h, 0, sizeof(uint64_t) * kRing);
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

}  // namespace ss

using namespace ss;

struct ss_layout : public ss::Layout {};
struct ss_graph : public ss::Graph {};

extern "C" {

const char* slimsell_last_error(void) { return g_last_error.c_str(); }

const char* slimsell_version(void) { return "slimsell-mi355x 0.1 (gfx950)"; }

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
  g->n = L->n;
  g->n_pad = L->n_pad;
  g->sigma = L->sigma;
  g->n_chunks = L->n_chunks;
  g->entries = L->entries;
  g->cells = L->cells;
  g->max_cl = L->max_cl;
  g->h_perm = L->perm;
  g->h_cl = L->cl;
  g->h_degree.resize((size_t)L->n);
  for (int32_t o = 0; o < L->n; ++o) g->h_degree[o] = L->degree[L->perm[o]];
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
  std::lock_guard<std::mutex> lock(g->mu);
  g->tune = *t;
  g->tune.pad0 = 0;
  return SS_OK;
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
  if (parent && s != SS_SELMAX) return set_error(SS_EINVAL, "parent needs SS_SELMAX");
  if (real_val && s != SS_REAL) return set_error(SS_EINVAL, "real_val needs SS_REAL");
  ss_bfs_opts def;
  std::memset(&def, 0, sizeof(def));
  def.size = sizeof(def);
  def.slimwork = 2;
  def.split_len = -1;
  if (!o) o = &def;
  if (o->size != sizeof(ss_bfs_opts)) return set_error(SS_EINVAL, "opts->size mismatch");
  if (o->slimwork < 0 || o->slimwork > 2) return set_error(SS_EINVAL, "slimwork must be 0, 1 or 2");
  for (int32_t r = 0; r < num_roots; ++r)
    if (roots[r] < 0 || roots[r] >= g.n) return set_error(SS_EINVAL, "root out of range [0, n)");
  const int waves = o->waves_per_group ? o->waves_per_group : g.tune.waves_per_group;
  if (waves != 1 && waves != 2 && waves != 4 && waves != 8 && waves != 16)
    return set_error(SS_EINVAL, "waves_per_group must be 1, 2, 4, 8 or 16");
  int32_t split = o->split_len;
  if (split < -1) return set_error(SS_EINVAL, "split_len must be >= -1");
  if (split == -1) split = g.tune.split_len;
  const int32_t pack = g.tune.pack_cols < 0 ? (split > 0 ? split : 0) : g.tune.pack_cols;
  const int unroll = g.tune.unroll;
  const int64_t max_groups = g.tune.max_groups;
  const int64_t cap = (o->max_levels > 0) ? o->max_levels : (int64_t)g.n + 1;
  if (o->level_cap < 0) return set_error(SS_EINVAL, "level_cap < 0");
  if (o->flags & ~(SS_STATS_TIME | SS_STATS_COUNTERS)) return set_error(SS_EINVAL, "bad flags");

  std::lock_guard<std::mutex> lock(g.mu);
  SS_HIP(hipSetDevice(g.device));
  hipStream_t st = static_cast<hipStream_t>(o->stream);
  UnitList* ul = nullptr;
  int rc = get_units(g, split, pack, &ul);
  if (rc) return rc;
  const bool timing = (o->flags & SS_STATS_TIME) != 0;
  const int64_t lcap = o->level_cap;
  const bool counting = (o->flags & SS_STATS_COUNTERS) && lcap > 0 && o->level_stats_out;
  const int64_t words_per_root = (lcap + 1) * kCountSlots * kCountFields;
  if (counting) {
    rc = ensure_counters(g, words_per_root * num_roots);
    if (rc) return rc;
    rc = launch_fill_u64(g.ws.counters, 0ull, words_per_root * num_roots, st);
    if (rc) return rc;
  }
  constexpr int kLookahead = 2;
  size_t next_ev = 0;
  std::vector<size_t> ev_first((size_t)num_roots, 0);
  std::vector<int32_t> launches((size_t)num_roots, 0);
  std::vector<int32_t> iters((size_t)num_roots, 0);

  for (int32_t r = 0; r < num_roots; ++r) {
    g.run_id = (g.run_id >= 0x7FFFFFF0u) ? 1u : g.run_id + 1;
    const uint32_t run = g.run_id;
    const int32_t root_row = g.h_perm[roots[r]];
    ev_first[r] = next_ev;
    if (timing) {
      hipEvent_t ev;
      if ((rc = pool_event(g, next_ev++, &ev))) return rc;
      SS_HIP(hipEventRecord(ev, st));
    }
    rc = launch_init(s, g, g.ws, root_row, st);
    if (rc) return rc;
    LevelArgs a;
    std::memset(&a, 0, sizeof(a));
    a.col = g.d_col;
    a.cs = g.d_cs;
    a.cl = g.d_cl;
    a.v = g.d_v;
    a.deg = g.d_deg;
    a.units = ul->d_units;
    a.pieces = ul->d_pieces;
    a.n_units = ul->count;
    a.state = g.ws.state;
    a.g = g.ws.g;
    a.d = g.ws.d;
    a.rv = g.ws.rv;
    a.acc = g.ws.acc;
    a.arrive = g.ws.arrive;
    a.any = g.ws.any;
    a.counters = counting ? g.ws.counters + words_per_root * r : nullptr;
    a.report = g.ws.d_report;
    a.run_id = run;
    a.n_pad = (uint32_t)g.n_pad;
    a.slimwork = o->slimwork;

    int32_t launched = 0;
    int32_t iterations = -1;
    auto launch = [&](int32_t k) -> int {
      a.level = k;
      a.vin = (k & 1) ? g.ws.vec_a : g.ws.vec_b;
      a.vout = (k & 1) ? g.ws.vec_b : g.ws.vec_a;
      a.count_stats = (counting && k <= lcap) ? 1 : 0;
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (timing) {
        int pr;
        if ((pr = pool_event(g, next_ev++, &e0))) return pr;
        if ((pr = pool_event(g, next_ev++, &e1))) return pr;
        SS_HIP(hipEventRecord(e0, st));
      }
      int lr = launch_level((int)s, waves, unroll, max_groups, a, st);
      if (lr) return lr;
      if (timing) SS_HIP(hipEventRecord(e1, st));
      return SS_OK;
    };
    for (int32_t j = 1;; ++j) {
      while (launched < j + kLookahead && launched <= cap) {
        rc = launch(++launched);
        if (rc) return rc;
      }
      bool found = false;
      rc = wait_report(g, j, run, st, &found);
      if (rc) return rc;
      if (!found) {
        iterations = j;
        break;
      }
      if (j >= cap) {
        (void)hipStreamSynchronize(st);
        return set_error(SS_EITER, "level cap reached before the BFS finished");
      }
    }
    launches[r] = launched;
    iters[r] = iterations;
    if (o->iterations_out) o->iterations_out[r] = iterations;
    rc = launch_finalise(s, g, g.ws, dist + (int64_t)r * g.n,
                         parent ? parent + (int64_t)r * g.n : nullptr,
                         real_val ? real_val + (int64_t)r * g.n : nullptr, st);
    if (rc) return rc;
    if (timing) {
      hipEvent_t ev;
      if ((rc = pool_event(g, next_ev++, &ev))) return rc;
      SS_HIP(hipEventRecord(ev, st));
    }
  }

  const bool want_levels = o->level_stats_out && lcap > 0;
  if (!(timing || counting || o->run_stats_out || want_levels)) return SS_OK;
  SS_HIP(hipStreamSynchronize(st));
  std::vector<unsigned long long> h;
  if (counting) {
    h.resize((size_t)(words_per_root * num_roots));
    SS_HIP(hipMemcpy(h.data(), g.ws.counters, sizeof(unsigned long long) * h.size(),
                     hipMemcpyDeviceToHost));
  }
  for (int32_t r = 0; r < num_roots; ++r) {
    float kernel_ms = 0.f, bfs_ms = 0.f;
    std::vector<float> lvl_ms((size_t)launches[r], 0.f);
    if (timing) {
      const size_t e = ev_first[r];
      auto ev = [&](size_t i) { return static_cast<hipEvent_t>(g.ev_pool[i]); };
      for (int32_t k = 0; k < launches[r]; ++k) {
        float ms = 0.f;
        SS_HIP(hipEventElapsedTime(&ms, ev(e + 1 + 2 * k), ev(e + 2 + 2 * k)));
        lvl_ms[k] = ms;
        kernel_ms += ms;
      }
      SS_HIP(hipEventElapsedTime(&bfs_ms, ev(e), ev(e + 1 + 2 * launches[r])));
    }
    if (o->run_stats_out) {
      ss_run_stats& rs = o->run_stats_out[r];
      rs.iterations = iters[r];
      rs.launches = launches[r];
      rs.kernel_ms = kernel_ms;
      rs.bfs_ms = bfs_ms;
    }
    if (want_levels) {
      for (int64_t k = 1; k <= lcap; ++k) {
        ss_level_stats& ls = o->level_stats_out[r * lcap + (k - 1)];
        std::memset(&ls, 0, sizeof(ls));
        if (k > iters[r]) continue;
        ls.ms = timing ? lvl_ms[k - 1] : 0.f;
        if (counting) {
          const unsigned long long* base = h.data() + words_per_root * r;
          for (int q = 0; q < kCountSlots; ++q) {
            const unsigned long long* f = base + (k * kCountSlots + q) * kCountFields;
            ls.discovered += (int64_t)f[0];
            ls.active_chunks += (int64_t)f[1];
            ls.active_cells += (int64_t)f[2];
            ls.max_active_cl = std::max<int64_t>(ls.max_active_cl, (int64_t)f[3]);
          }
        }
      }
    }
  }
  return SS_OK;
}

}  // extern "C"
