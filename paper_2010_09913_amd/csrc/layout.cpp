// Host construction of the SlimSell layout (Section III-B, "Reducing Storage
// Complexity with SlimSell"; the Sell-C-sigma layout it derives from is in
// Section II-D).  Multithreaded with std::thread; deterministic for any thread
// count because every row's neighbour list is sorted before use.
//
// Steps
//   1. canonical simple undirected graph: both directions of each tuple,
//      self-loops dropped, duplicates dropped (per-row sort + unique);
//   2. sigma-scoped sort: inside each window of sigma consecutive original IDs,
//      rows are ordered by decreasing degree, stable on the ID, which puts the
//      longer rows of every window first;
//   3. relabel: a vertex's row is its sorted position; v[row] = ID + 1;
//   4. chunks of 64 rows: cl[i] = longest row, cs = prefix of 64 * cl;
//   5. col[cs[i] + 64 j + lane] = row of the j-th neighbour, -1 as padding.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "internal.h"

namespace ss {

static int hw_threads() {
  unsigned t = std::thread::hardware_concurrency();
  if (t == 0) t = 4;
  if (t > 32) t = 32;
  return (int)t;
}

template <class F>
static void parallel_for(int64_t n, F&& f, int threads = 0) {
  if (threads <= 0) threads = hw_threads();
  if (n < 4096 || threads == 1) {
    f(0, n, 0);
    return;
  }
  std::vector<std::thread> pool;
  int64_t per = (n + threads - 1) / threads;
  for (int t = 0; t < threads; ++t) {
    int64_t b = t * per, e = std::min<int64_t>(n, b + per);
    if (b >= e) break;
    pool.emplace_back([&, b, e, t] { f(b, e, t); });
  }
  for (auto& th : pool) th.join();
}

// Dynamic row-range scheduling for the uneven per-row work.
template <class F>
static void parallel_dynamic(int64_t n, int64_t grain, F&& f) {
  int threads = hw_threads();
  if (n <= grain || threads == 1) {
    f(0, n);
    return;
  }
  std::atomic<int64_t> next{0};
  std::vector<std::thread> pool;
  for (int t = 0; t < threads; ++t) {
    pool.emplace_back([&] {
      for (;;) {
        int64_t b = next.fetch_add(grain);
        if (b >= n) break;
        f(b, std::min(n, b + grain));
      }
    });
  }
  for (auto& th : pool) th.join();
}

int build_layout(const int32_t* src, const int32_t* dst, int64_t m, int32_t n, int32_t C,
                 int32_t sigma, Layout** out) {
  if (!out) return set_error(SS_EINVAL, "out is NULL");
  *out = nullptr;
  if (n < 1) return set_error(SS_EINVAL, "n must be >= 1");
  if (m < 0) return set_error(SS_EINVAL, "m must be >= 0");
  if (m > 0 && (!src || !dst)) return set_error(SS_EINVAL, "src/dst is NULL");
  if (C != kC) return set_error(SS_EINVAL, "C must be 64 (one wavefront of rows per chunk)");
  const int64_t n_pad = ((int64_t)n + kC - 1) / kC * kC;
  if (n_pad > INT32_MAX) return set_error(SS_EINVAL, "n too large");
  if (sigma == 0 || sigma == n) sigma = (int32_t)n_pad;
  if (sigma != 1 && (sigma % kC != 0 || sigma > n_pad))
    return set_error(SS_EINVAL,
                     "sigma must be 1, 0 (all rows), n, or a multiple of 64 no larger than the "
                     "padded vertex count");

  // validate IDs
  {
    std::atomic<int> bad{0};
    parallel_for(m, [&](int64_t b, int64_t e, int) {
      for (int64_t i = b; i < e; ++i) {
        if ((uint32_t)src[i] >= (uint32_t)n || (uint32_t)dst[i] >= (uint32_t)n) {
          bad.store(1, std::memory_order_relaxed);
          return;
        }
      }
    });
    if (bad.load()) return set_error(SS_EINVAL, "vertex ID out of range [0, n)");
  }

  Layout* L = new (std::nothrow) Layout();
  if (!L) return set_error(SS_ENOMEM, "host allocation failed");
  L->n = n;
  L->n_pad = (int32_t)n_pad;
  L->sigma = sigma;
  L->n_chunks = n_pad / kC;

  try {
    // ---- 1. canonical adjacency (rowptr over original IDs) -----------------
    std::vector<std::atomic<int64_t>> cnt(n);
    parallel_for(n, [&](int64_t b, int64_t e, int) {
      for (int64_t v = b; v < e; ++v) cnt[v].store(0, std::memory_order_relaxed);
    });
    parallel_for(m, [&](int64_t b, int64_t e, int) {
      for (int64_t i = b; i < e; ++i) {
        int32_t u = src[i], w = dst[i];
        if (u == w) continue;
        cnt[u].fetch_add(1, std::memory_order_relaxed);
        cnt[w].fetch_add(1, std::memory_order_relaxed);
      }
    });
    std::vector<int64_t> rp((size_t)n + 1);
    rp[0] = 0;
    for (int32_t v = 0; v < n; ++v) rp[v + 1] = rp[v] + cnt[v].load(std::memory_order_relaxed);
    std::vector<int32_t> adj((size_t)rp[n]);
    parallel_for(n, [&](int64_t b, int64_t e, int) {
      for (int64_t v = b; v < e; ++v) cnt[v].store(rp[v], std::memory_order_relaxed);
    });
    parallel_for(m, [&](int64_t b, int64_t e, int) {
      for (int64_t i = b; i < e; ++i) {
        int32_t u = src[i], w = dst[i];
        if (u == w) continue;
        adj[cnt[u].fetch_add(1, std::memory_order_relaxed)] = w;
        adj[cnt[w].fetch_add(1, std::memory_order_relaxed)] = u;
      }
    });
    std::vector<int32_t> deg((size_t)n);
    parallel_dynamic(n, 2048, [&](int64_t b, int64_t e) {
      for (int64_t v = b; v < e; ++v) {
        int32_t* row = adj.data() + rp[v];
        int64_t len = rp[v + 1] - rp[v];
        std::sort(row, row + len);
        deg[v] = (int32_t)(std::unique(row, row + len) - row);
      }
    });

    // ---- 2./3. sigma-scoped sort and relabelling ----------------------------
    // order[row] = original ID (or -1 for phantom rows)
    std::vector<int32_t> order((size_t)n_pad);
    for (int64_t r = 0; r < n_pad; ++r) order[r] = (r < n) ? (int32_t)r : -1;
    auto degree_of = [&](int32_t v) -> int32_t { return v < 0 ? 0 : deg[v]; };
    if (sigma > 1) {
      const int64_t nwin = (n_pad + sigma - 1) / sigma;
      int32_t max_deg = 0;
      for (int32_t v = 0; v < n; ++v) max_deg = std::max(max_deg, deg[v]);
      parallel_dynamic(nwin, 1, [&](int64_t wb, int64_t we) {
        for (int64_t w = wb; w < we; ++w) {
          int64_t b = w * sigma, e = std::min<int64_t>(n_pad, b + sigma);
          if (e - b > 65536) {
            // stable counting sort by decreasing degree
            std::vector<int64_t> bucket((size_t)max_deg + 2, 0);
            for (int64_t r = b; r < e; ++r) bucket[max_deg - degree_of(order[r])]++;
            int64_t acc = 0;
            for (auto& x : bucket) { int64_t t = x; x = acc; acc += t; }
            std::vector<int32_t> tmp((size_t)(e - b));
            for (int64_t r = b; r < e; ++r) {
              int32_t v = order[r];
              tmp[bucket[max_deg - degree_of(v)]++] = v;
            }
            std::copy(tmp.begin(), tmp.end(), order.begin() + b);
          } else {
            std::stable_sort(order.begin() + b, order.begin() + e, [&](int32_t x, int32_t y) {
              return degree_of(x) > degree_of(y);
            });
          }
        }
      });
    }
    L->v.assign((size_t)n_pad, 0);
    L->perm.assign((size_t)n, 0);
    L->degree.assign((size_t)n_pad, 0);
    for (int64_t r = 0; r < n_pad; ++r) {
      int32_t v = order[r];
      if (v >= 0) {
        L->v[r] = v + 1;
        L->perm[v] = (int32_t)r;
        L->degree[r] = deg[v];
      }
    }

    // ---- 4. chunk lengths and offsets --------------------------------------
    const int64_t nc = L->n_chunks;
    L->cl.assign((size_t)nc, 0);
    L->cs.assign((size_t)nc + 1, 0);
    int32_t max_cl = 0;
    for (int64_t i = 0; i < nc; ++i) {
      int32_t mx = 0;
      for (int lane = 0; lane < kC; ++lane) mx = std::max(mx, L->degree[i * kC + lane]);
      L->cl[i] = mx;
      max_cl = std::max(max_cl, mx);
      L->cs[i + 1] = L->cs[i] + (int64_t)mx * kC;
    }
    L->max_cl = max_cl;
    L->cells = L->cs[nc];
    L->entries = 0;
    for (int32_t v = 0; v < n; ++v) L->entries += deg[v];

    // ---- 5. column-major fill with the -1 padding marker -------------------
    // A row lists its neighbours by decreasing original ID, so a scan that
    // stops at its first frontier neighbour has found the largest one.
    L->col.assign((size_t)L->cells, -1);
    const int32_t* perm = L->perm.data();
    parallel_dynamic(nc, 64, [&](int64_t cb, int64_t ce) {
      for (int64_t i = cb; i < ce; ++i) {
        int32_t* base = L->col.data() + L->cs[i];
        for (int lane = 0; lane < kC; ++lane) {
          int32_t v = L->v[i * kC + lane] - 1;
          if (v < 0) continue;
          const int32_t* nb = adj.data() + rp[v];
          const int32_t d = deg[v];
          for (int32_t j = 0; j < d; ++j) base[(int64_t)j * kC + lane] = perm[nb[d - 1 - j]];
        }
      }
    });
  } catch (const std::bad_alloc&) {
    delete L;
    return set_error(SS_ENOMEM, "host allocation failed while building the layout");
  }
  *out = L;
  return SS_OK;
}

}  // namespace ss
