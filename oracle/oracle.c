/*
 * ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU statement of what SlimSell BFS computes.
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * may load this library.  It shares no code, header or table with the GPU
 * path; the only common input is the seeded tuple list from graphgen.
 *
 * Paper: Besta, Marending, Solomonik, Hoefler, "SlimSell: A Vectorizable Graph
 * Representation for Breadth-First Search" (arXiv 2010.09913).  Sections are
 * cited by their titles.
 *
 * Contents
 *   oracle_csr            canonical simple undirected graph as sorted CSR
 *                         (Section II-D, "Adjacency List (AL)")
 *   oracle_bfs            textbook FIFO-queue BFS distances
 *                         (Section II-C, "Traditional BFS")
 *   oracle_bfs_omp        the same distances by a level-synchronous top-down
 *                         sweep on all host cores (CPU baseline only)
 *   oracle_parents_max    the DP transformation p = DP(d) with the largest
 *                         qualifying neighbour as the parent (Section II-C)
 *   oracle_real_counts    number of neighbours one level closer to the root
 *   oracle_lneg           the paper's logical negation of a vector (Section
 *                         II-A, "Linear Algebra")
 *   oracle_semiring_bfs   the four algebraic BFS formulations stepped literally
 *                         on dense vectors (Section III-A: tropical, real,
 *                         boolean and sel-max semirings)
 *
 * Readings taken where the paper is silent or inconsistent (each is listed in
 * the design notes of the repository):
 *   - distances are -1 for unreachable vertices and 0 for the root;
 *   - the iteration stops after the first product that discovers no vertex
 *     (one more than the root's eccentricity);
 *   - real semiring: the frontier is binarised, f_k = [x_k * g_k != 0];
 *   - boolean "x_k - g_k" is read as x_k AND g_k with g_k the unvisited mask;
 *   - sel-max uses 1-based vertex values (x_0^r = r + 1) so that 0 means
 *     "nothing"; its parent update follows the equation
 *     p_k = p_{k-1} + NOT(p_{k-1}) (.) x_k, and an empty max is 0;
 *   - the DP tie-break picks the largest neighbour ID, which is what the
 *     sel-max product yields.
 *
 * Parity is pinned by tests against Floyd-Warshall and dense brute force on
 * tiny graphs, closed forms (paths, cycles, stars, cliques, hypercubes, full
 * grids) and BFS invariants.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

/*
 * Canonical simple undirected graph (Section II-D, "Adjacency List (AL)"): every
 * tuple (u, v) with u != v contributes both directions; self-loops are dropped
 * and repeated neighbours are kept once.  rowptr has n+1 entries; adj must hold
 * 2m entries (an upper bound).  Returns the number of directed entries E, or <0.
 */
int64_t oracle_csr(const int32_t* src, const int32_t* dst, int64_t m, int32_t n,
                   int64_t* rowptr, int32_t* adj) {
  if (n < 0 || m < 0) return -1;
  int64_t* deg = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  if (!deg) return -2;
  for (int64_t i = 0; i < m; ++i) {
    int32_t u = src[i], v = dst[i];
    if (u < 0 || u >= n || v < 0 || v >= n) { free(deg); return -1; }
    if (u == v) continue;
    deg[u]++;
    deg[v]++;
  }
  rowptr[0] = 0;
  for (int32_t v = 0; v < n; ++v) rowptr[v + 1] = rowptr[v] + deg[v];
  int64_t* fill = deg; /* reuse as the per-row write cursor */
  for (int32_t v = 0; v < n; ++v) fill[v] = rowptr[v];
  for (int64_t i = 0; i < m; ++i) {
    int32_t u = src[i], v = dst[i];
    if (u == v) continue;
    adj[fill[u]++] = v;
    adj[fill[v]++] = u;
  }
  free(deg);
  /* sort every row, then squeeze out repeated neighbours */
  int64_t out = 0;
  int64_t start = 0;
  for (int32_t v = 0; v < n; ++v) {
    int64_t end = rowptr[v + 1];
    qsort(adj + start, (size_t)(end - start), sizeof(int32_t), cmp_i32);
    int64_t row_begin = out;
    for (int64_t j = start; j < end; ++j) {
      if (out > row_begin && adj[out - 1] == adj[j]) continue;
      adj[out++] = adj[j];
    }
    rowptr[v] = row_begin;
    start = end;
  }
  rowptr[n] = out;
  return out;
}

/*
 * Textbook BFS (Section II-C, "Traditional BFS"): a FIFO queue; a vertex gets
 * distance d+1 when it is first seen from a vertex at distance d.  Unreached
 * vertices keep -1.  Returns the number of reached vertices.
 */
int64_t oracle_bfs(const int64_t* rowptr, const int32_t* adj, int32_t n, int32_t root,
                   int32_t* dist) {
  for (int32_t v = 0; v < n; ++v) dist[v] = -1;
  if (root < 0 || root >= n) return -1;
  int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
  if (!queue) return -2;
  int64_t head = 0, tail = 0;
  dist[root] = 0;
  queue[tail++] = root;
  while (head < tail) {
    int32_t u = queue[head++];
    for (int64_t j = rowptr[u]; j < rowptr[u + 1]; ++j) {
      int32_t w = adj[j];
      if (dist[w] < 0) {
        dist[w] = dist[u] + 1;
        queue[tail++] = w;
      }
    }
  }
  free(queue);
  return tail;
}

/*
 * The same distances by a level-synchronous top-down sweep over all vertices,
 * parallelised with OpenMP.  It is the oracle's all-cores form, used only as a
 * CPU timing baseline.  Returns the number of levels swept.
 */
/* Threads oracle_bfs_omp runs on (for the CPU baseline's core count). */
int32_t oracle_threads(void) {
#ifdef _OPENMP
  return (int32_t)omp_get_max_threads();
#else
  return 1;
#endif
}

int32_t oracle_bfs_omp(const int64_t* rowptr, const int32_t* adj, int32_t n, int32_t root,
                       int32_t* dist) {
  for (int32_t v = 0; v < n; ++v) dist[v] = -1;
  if (root < 0 || root >= n) return -1;
  dist[root] = 0;
  int32_t level = 0;
  int changed = 1;
  while (changed) {
    changed = 0;
#pragma omp parallel for schedule(dynamic, 1024) reduction(| : changed)
    for (int32_t v = 0; v < n; ++v) {
      if (dist[v] != -1) continue;
      for (int64_t j = rowptr[v]; j < rowptr[v + 1]; ++j) {
        if (dist[adj[j]] == level) {
          dist[v] = -2; /* found this level; published below */
          changed = 1;
          break;
        }
      }
    }
    ++level;
#pragma omp parallel for schedule(static)
    for (int32_t v = 0; v < n; ++v)
      if (dist[v] == -2) dist[v] = level;
  }
  return level;
}

/*
 * DP transformation (Section II-C): for every reached v other than the root,
 * its parent is a neighbour w with d(w) = d(v) - 1.  Among several such
 * neighbours the largest ID is taken.  parent[root] = root, unreached = -1.
 */
void oracle_parents_max(const int64_t* rowptr, const int32_t* adj, int32_t n, int32_t root,
                        const int32_t* dist, int32_t* parent) {
  for (int32_t v = 0; v < n; ++v) {
    parent[v] = -1;
    if (dist[v] <= 0) continue;
    for (int64_t j = rowptr[v]; j < rowptr[v + 1]; ++j) {
      int32_t w = adj[j];
      if (dist[w] == dist[v] - 1 && w > parent[v]) parent[v] = w;
    }
  }
  if (root >= 0 && root < n) parent[root] = root;
}

/*
 * Number of neighbours one level closer to the root, as a float: the value the
 * real-semiring product holds for a vertex in the iteration that discovers it.
 * Root = 1 (its starting value), unreached = 0.
 */
void oracle_real_counts(const int64_t* rowptr, const int32_t* adj, int32_t n, int32_t root,
                        const int32_t* dist, float* out) {
  for (int32_t v = 0; v < n; ++v) {
    out[v] = 0.0f;
    if (dist[v] <= 0) continue;
    int64_t c = 0;
    for (int64_t j = rowptr[v]; j < rowptr[v + 1]; ++j)
      if (dist[adj[j]] == dist[v] - 1) ++c;
    out[v] = (float)c;
  }
  if (root >= 0 && root < n) out[root] = 1.0f;
}

/* Logical negation (Section II-A): NOT(x)^s = 1 if x^s == 0, else 0. */
void oracle_lneg(const double* x, int64_t n, double* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = (x[i] == 0.0) ? 1.0 : 0.0;
}

enum { OR_TROPICAL = 0, OR_REAL = 1, OR_BOOLEAN = 2, OR_SELMAX = 3 };

#define OR_INF 1e300 /* stands for the tropical infinity */

/*
 * The algebraic BFS of Section III-A, stepped literally on dense vectors with
 * the adjacency matrix A given by CSR (A^T = A, the graph is undirected).
 *
 *   tropical  x_0^r = 0, x_0^s = inf; x_k = f_k = A' (x) f_{k-1} over (min, +),
 *             A' = A with off-diagonal zeros set to inf and a zero diagonal;
 *             distances are the final x.
 *   real      x_0 = f_0 = e_r; x_k = A (x) f_{k-1} over (+, *);
 *             g_k = NOT(sum_{l<k} f_l); f_k = [x_k (.) g_k != 0];
 *             d = sum_l l f_l.
 *   boolean   as real over (|, &) with f_k = x_k & g_k, g_k = NOT(union f_l).
 *   sel-max   x_0^r = r+1 (1-based), f_0 = e_r, p_0 = x_0;
 *             x_k = A (x) x_{k-1} over (max, *); g_k = sum_{l<k} f_l;
 *             f_k = NOT(NOT(x_k)) minus g_k; p_k = p_{k-1} + NOT(p_{k-1}) (.) x_k;
 *             x_k <- NOT(NOT(x_k)) (.) (1, ..., n); d = union_l l f_l.
 *
 * Iterations run until one discovers no vertex (at most max_iters, 0 = n+1).
 * Outputs (0-based, original IDs): dist (-1 unreached), parent (sel-max only,
 * may be NULL), real_val (real only: x_{d(v)}^v, may be NULL), frontier_sizes
 * (number of vertices discovered by iteration k at index k-1, may be NULL,
 * capacity max_iters).  Returns the number of iterations performed (<0 on a
 * bad argument, -3 if the cap was reached before termination).
 */
int32_t oracle_semiring_bfs(const int64_t* rowptr, const int32_t* adj, int32_t n, int32_t root,
                            int32_t semiring, int32_t max_iters, int32_t* dist, int32_t* parent,
                            float* real_val, int64_t* frontier_sizes) {
  if (n <= 0 || root < 0 || root >= n || semiring < 0 || semiring > 3) return -1;
  if (max_iters <= 0) max_iters = n + 1;
  double* x = (double*)calloc((size_t)n, sizeof(double));
  double* xn = (double*)calloc((size_t)n, sizeof(double));
  double* f = (double*)calloc((size_t)n, sizeof(double));
  double* g = (double*)calloc((size_t)n, sizeof(double));
  double* ng = (double*)calloc((size_t)n, sizeof(double));
  double* p = (double*)calloc((size_t)n, sizeof(double));
  double* nn = (double*)calloc((size_t)n, sizeof(double));
  double* d = (double*)calloc((size_t)n, sizeof(double));
  if (!x || !xn || !f || !g || !ng || !p || !nn || !d) {
    free(x); free(xn); free(f); free(g); free(ng); free(p); free(nn); free(d);
    return -2;
  }
  int32_t k = 0;
  int32_t done = 0;
  int32_t rc = 0;

  for (int32_t v = 0; v < n; ++v) { dist[v] = -1; if (real_val) real_val[v] = 0.0f; }

  if (semiring == OR_TROPICAL) {
    for (int32_t v = 0; v < n; ++v) f[v] = OR_INF;
    f[root] = 0.0;
    while (!done) {
      if (k >= max_iters) { rc = -3; break; }
      ++k;
      int64_t discovered = 0;
      for (int32_t i = 0; i < n; ++i) {
        double best = f[i]; /* A'(i,i) = 0 */
        for (int64_t j = rowptr[i]; j < rowptr[i + 1]; ++j) {
          double cand = 1.0 + f[adj[j]]; /* A'(i,j) = 1 on an edge */
          if (cand < best) best = cand;
        }
        xn[i] = best;
      }
      for (int32_t i = 0; i < n; ++i) {
        if (f[i] >= OR_INF && xn[i] < OR_INF) ++discovered;
        f[i] = xn[i];
      }
      if (frontier_sizes) frontier_sizes[k - 1] = discovered;
      if (discovered == 0) done = 1;
    }
    for (int32_t v = 0; v < n; ++v) dist[v] = (f[v] >= OR_INF) ? -1 : (int32_t)f[v];
  } else if (semiring == OR_REAL || semiring == OR_BOOLEAN) {
    /* f_0 = x_0 = e_r; d accumulates l * f_l */
    f[root] = 1.0;
    for (int32_t v = 0; v < n; ++v) g[v] = f[v]; /* running sum of frontiers */
    if (real_val) real_val[root] = 1.0f;
    while (!done) {
      if (k >= max_iters) { rc = -3; break; }
      ++k;
      oracle_lneg(g, n, ng); /* g_k = NOT(sum_{l<k} f_l) */
      for (int32_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int64_t j = rowptr[i]; j < rowptr[i + 1]; ++j) {
          if (semiring == OR_REAL) acc += f[adj[j]];          /* (+, *), A(i,j) = 1 */
          else acc = (acc != 0.0 || f[adj[j]] != 0.0) ? 1.0 : 0.0; /* (|, &) */
        }
        x[i] = acc;
      }
      int64_t discovered = 0;
      for (int32_t i = 0; i < n; ++i) {
        double fk = (semiring == OR_REAL) ? ((x[i] * ng[i] != 0.0) ? 1.0 : 0.0)
                                          : ((x[i] != 0.0 && ng[i] != 0.0) ? 1.0 : 0.0);
        if (fk != 0.0) {
          ++discovered;
          d[i] += (double)k * fk;
          if (real_val) real_val[i] = (float)x[i];
        }
        xn[i] = fk;
      }
      for (int32_t i = 0; i < n; ++i) { f[i] = xn[i]; g[i] += f[i]; }
      if (frontier_sizes) frontier_sizes[k - 1] = discovered;
      if (discovered == 0) done = 1;
    }
    for (int32_t v = 0; v < n; ++v) dist[v] = (g[v] != 0.0) ? (int32_t)d[v] : -1;
  } else { /* OR_SELMAX */
    x[root] = (double)root + 1.0;
    f[root] = 1.0;
    for (int32_t v = 0; v < n; ++v) { p[v] = x[v]; g[v] = f[v]; }
    while (!done) {
      if (k >= max_iters) { rc = -3; break; }
      ++k;
      for (int32_t i = 0; i < n; ++i) {
        double acc = 0.0; /* empty max: nothing reaches i */
        for (int64_t j = rowptr[i]; j < rowptr[i + 1]; ++j) {
          double cand = 1.0 * x[adj[j]]; /* A(i,j) = 1 times x_{k-1}^j */
          if (cand > acc) acc = cand;
        }
        xn[i] = acc;
      }
      oracle_lneg(xn, n, nn);
      oracle_lneg(nn, n, nn); /* NOT(NOT(x_k)) */
      oracle_lneg(p, n, ng);  /* NOT(p_{k-1}) */
      int64_t discovered = 0;
      for (int32_t i = 0; i < n; ++i) {
        double fk = (nn[i] != 0.0 && g[i] == 0.0) ? 1.0 : 0.0; /* NOT NOT x_k minus g_k */
        p[i] = p[i] + ng[i] * xn[i];
        if (fk != 0.0) { ++discovered; d[i] += (double)k * fk; }
        f[i] = fk;
        x[i] = nn[i] * ((double)i + 1.0); /* NOT NOT x_k (.) (1..n) */
      }
      for (int32_t i = 0; i < n; ++i) g[i] += f[i];
      if (frontier_sizes) frontier_sizes[k - 1] = discovered;
      if (discovered == 0) done = 1;
    }
    for (int32_t v = 0; v < n; ++v) {
      dist[v] = (g[v] != 0.0) ? (int32_t)d[v] : -1;
      if (parent) parent[v] = (p[v] != 0.0) ? (int32_t)p[v] - 1 : -1;
    }
  }
  free(x); free(xn); free(f); free(g); free(ng); free(p); free(nn); free(d);
  return rc < 0 ? rc : k;
}
