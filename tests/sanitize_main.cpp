// Host code under AddressSanitizer and UndefinedBehaviorSanitizer: the
// SlimSell layout builder (layout.cpp), the oracle (oracle.c) and the seeded
// input generators (graphgen.c) on small graphs, every layout checked against
// the oracle's canonical graph and every oracle formulation against its
// queue BFS.  Built and run by tests/test_sanitizers.py; exits non-zero on
// the first mismatch (a sanitizer report aborts the process by itself).
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../paper_2010_09913_amd/csrc/internal.h"

extern "C" {
int gg_rmat(int32_t scale, int64_t m, double a, double b, double c, uint64_t seed, int32_t* src,
            int32_t* dst);
int gg_er(int64_t n, int64_t m, uint64_t seed, int32_t* src, int32_t* dst);
int64_t gg_grid_edges(int32_t w, int32_t h);
int64_t gg_grid(int32_t w, int32_t h, int64_t remove, uint64_t seed, int32_t* src, int32_t* dst);
int32_t gg_pick_roots(const int32_t* src, const int32_t* dst, int64_t m, int64_t n, int32_t k,
                      uint64_t seed, int32_t* out);
int64_t oracle_csr(const int32_t* src, const int32_t* dst, int64_t m, int32_t n, int64_t* rowptr,
                   int32_t* adj);
int64_t oracle_bfs(const int64_t* rowptr, const int32_t* adj, int32_t n, int32_t root,
                   int32_t* dist);
void oracle_parents_max(const int64_t* rowptr, const int32_t* adj, int32_t n, int32_t root,
                        const int32_t* dist, int32_t* parent);
void oracle_real_counts(const int64_t* rowptr, const int32_t* adj, int32_t n, int32_t root,
                        const int32_t* dist, float* out);
int32_t oracle_semiring_bfs(const int64_t* rowptr, const int32_t* adj, int32_t n, int32_t root,
                            int32_t semiring, int32_t max_iters, int32_t* dist, int32_t* parent,
                            float* real_val, int64_t* frontier_sizes);
}

namespace ss {
// layout.cpp reports argument errors through the library's error hook
int set_error(int code, const std::string& msg) {
  std::fprintf(stderr, "set_error(%d): %s\n", code, msg.c_str());
  return code;
}
}  // namespace ss

static int failures = 0;
#define CHECK(cond, ...)                                     \
  do {                                                       \
    if (!(cond)) {                                           \
      std::fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
      std::fprintf(stderr, __VA_ARGS__);                     \
      std::fprintf(stderr, "\n");                            \
      ++failures;                                            \
      return;                                                \
    }                                                        \
  } while (0)

struct Edges {
  std::string name;
  int32_t n;
  std::vector<int32_t> src, dst;
};

static void check_layout(const Edges& e, const std::vector<int64_t>& rowptr,
                         const std::vector<int32_t>& adj, int32_t sigma) {
  ss::Layout* L = nullptr;
  const int rc = ss::build_layout(e.src.data(), e.dst.data(), (int64_t)e.src.size(), e.n, 64,
                                  sigma, &L);
  CHECK(rc == 0 && L, "%s sigma %d: build_layout returned %d", e.name.c_str(), sigma, rc);
  CHECK(L->n == e.n && L->n_pad % 64 == 0 && L->n_pad >= L->n, "%s: sizes", e.name.c_str());
  CHECK(L->cs[0] == 0 && L->cs[L->n_chunks] == L->cells, "%s: chunk offsets", e.name.c_str());
  CHECK(L->entries == (int64_t)adj.size(), "%s: entries %lld vs %zu", e.name.c_str(),
        (long long)L->entries, adj.size());
  for (int64_t i = 0; i < L->n_chunks; ++i)
    CHECK(L->cs[i + 1] - L->cs[i] == 64 * (int64_t)L->cl[i], "%s: chunk %lld length",
          e.name.c_str(), (long long)i);
  std::vector<int32_t> row_of(L->perm);
  for (int32_t r = 0; r < L->n_pad; ++r) {
    const int64_t c = r / 64, lane = r % 64;
    const int32_t o = L->v[r] - 1;
    std::vector<int32_t> got;
    bool pad = false;
    for (int32_t j = 0; j < L->cl[c]; ++j) {
      const int32_t x = L->col[L->cs[c] + 64 * j + lane];
      if (x < 0) {
        pad = true;
        continue;
      }
      CHECK(!pad, "%s: row %d has an entry after padding", e.name.c_str(), r);
      CHECK(x < L->n_pad, "%s: row %d entry %d out of range", e.name.c_str(), r, x);
      got.push_back(L->v[x] - 1);
    }
    if (o < 0) {
      CHECK(got.empty(), "%s: phantom row %d has entries", e.name.c_str(), r);
      continue;
    }
    CHECK(row_of[o] == r, "%s: perm and v disagree at %d", e.name.c_str(), o);
    // neighbours of the original vertex, listed by decreasing original ID
    std::vector<int32_t> want(adj.begin() + rowptr[o], adj.begin() + rowptr[o + 1]);
    std::reverse(want.begin(), want.end());
    CHECK(got == want, "%s sigma %d: row %d (vertex %d) neighbours differ", e.name.c_str(),
          sigma, r, o);
    CHECK(L->degree[r] == (int32_t)want.size(), "%s: degree of row %d", e.name.c_str(), r);
  }
  delete L;
}

static void check_oracle(const Edges& e, const std::vector<int64_t>& rowptr,
                         const std::vector<int32_t>& adj) {
  std::vector<int32_t> roots(3, 0);
  int32_t k = 0;  // a graph without tuples keeps root 0 (isolated)
  if (!e.src.empty()) {
    k = gg_pick_roots(e.src.data(), e.dst.data(), (int64_t)e.src.size(), e.n, 3, 17,
                      roots.data());
    CHECK(k >= 0, "%s: pick_roots", e.name.c_str());
  }
  roots.resize(k > 0 ? k : 1);
  for (int32_t r : roots) {
    std::vector<int32_t> d(e.n), p(e.n), d2(e.n), p2(e.n);
    std::vector<float> rv(e.n), rv2(e.n);
    std::vector<int64_t> fs((size_t)e.n + 2);
    CHECK(oracle_bfs(rowptr.data(), adj.data(), e.n, r, d.data()) >= 1, "%s: bfs", e.name.c_str());
    oracle_parents_max(rowptr.data(), adj.data(), e.n, r, d.data(), p.data());
    oracle_real_counts(rowptr.data(), adj.data(), e.n, r, d.data(), rv.data());
    for (int32_t s = 0; s < 4; ++s) {
      const int32_t it = oracle_semiring_bfs(rowptr.data(), adj.data(), e.n, r, s, e.n + 1,
                                             d2.data(), s == 3 ? p2.data() : nullptr,
                                             s == 1 ? rv2.data() : nullptr, fs.data());
      CHECK(it >= 1, "%s: semiring %d failed", e.name.c_str(), s);
      CHECK(d2 == d, "%s: semiring %d distances differ from the queue BFS", e.name.c_str(), s);
      if (s == 3) CHECK(p2 == p, "%s: sel-max parents differ", e.name.c_str());
      if (s == 1) CHECK(rv2 == rv, "%s: real values differ", e.name.c_str());
    }
  }
}

static void run(const Edges& e) {
  std::vector<int64_t> rowptr((size_t)e.n + 1);
  std::vector<int32_t> adj(2 * e.src.size() + 1);
  const int64_t E = oracle_csr(e.src.data(), e.dst.data(), (int64_t)e.src.size(), e.n,
                               rowptr.data(), adj.data());
  CHECK(E >= 0, "%s: oracle_csr", e.name.c_str());
  adj.resize((size_t)E);
  for (int32_t sigma : {1, 64, 0}) check_layout(e, rowptr, adj, sigma);
  check_oracle(e, rowptr, adj);
  std::fprintf(stderr, "ok %s (n %d, %zu tuples, %lld entries)\n", e.name.c_str(), e.n,
               e.src.size(), (long long)E);
}

int main() {
  std::vector<Edges> graphs;
  {
    Edges e{"rmat-s10", 1 << 10, {}, {}};
    e.src.resize(16 << 10);
    e.dst.resize(16 << 10);
    gg_rmat(10, 16 << 10, 0.57, 0.19, 0.19, 1, e.src.data(), e.dst.data());
    graphs.push_back(e);
  }
  {
    Edges e{"er-3001", 3001, {}, {}};
    e.src.resize(9000);
    e.dst.resize(9000);
    gg_er(3001, 9000, 2, e.src.data(), e.dst.data());
    graphs.push_back(e);
  }
  {
    const int64_t m = gg_grid_edges(37, 29);
    const int64_t cut = m / 20;
    Edges e{"grid-37x29", 37 * 29, {}, {}};
    e.src.resize((size_t)(m - cut));
    e.dst.resize((size_t)(m - cut));
    gg_grid(37, 29, cut, 5, e.src.data(), e.dst.data());
    graphs.push_back(e);
  }
  {
    Edges e{"path-130-with-isolated", 200, {}, {}};
    for (int32_t i = 0; i + 1 < 130; ++i) {
      e.src.push_back(i);
      e.dst.push_back(i + 1);
      e.src.push_back(i + 1);  // duplicates and self-loops are dropped by both sides
      e.dst.push_back(i);
      e.src.push_back(i);
      e.dst.push_back(i);
    }
    graphs.push_back(e);
  }
  {
    Edges e{"single-vertex", 1, {}, {}};
    graphs.push_back(e);
  }
  for (const Edges& e : graphs) run(e);
  // argument errors are reported, not crashed on
  ss::Layout* L = nullptr;
  const int32_t s0 = 0, d0 = 5;
  if (ss::build_layout(&s0, &d0, 1, 3, 64, 0, &L) == 0 || L) {
    std::fprintf(stderr, "FAIL: an out-of-range ID was accepted\n");
    ++failures;
  }
  if (ss::build_layout(&s0, &s0, 1, 3, 32, 0, &L) == 0 || L) {
    std::fprintf(stderr, "FAIL: C = 32 was accepted\n");
    ++failures;
  }
  std::fprintf(stderr, "%d failure(s)\n", failures);
  return failures ? 1 : 0;
}
