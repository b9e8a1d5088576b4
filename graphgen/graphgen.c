/*
 * Seeded synthetic graph inputs: R-MAT (Kronecker) tuples, Erdos-Renyi G(n, M)
 * tuples, a W x H 4-neighbour grid with a fixed fraction of edges removed, and
 * root selection.  Output is a raw list of (src, dst) tuples; self-loops and
 * duplicates are left in, the consumer canonicalises.
 *
 * This module only draws random inputs.  It holds none of the BFS method's
 * arithmetic and is the one piece of code that both the oracle and the GPU
 * path use.
 *
 * Random numbers come from a counter-based generator: the SplitMix64 output
 * function (Steele, Lea and Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014) applied to (seed, stream, counter).  Every draw is
 * a pure function of its indices, so generation is deterministic under any
 * thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static inline uint64_t sm64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

/* One 64-bit draw for (seed, stream, counter). */
static inline uint64_t draw(uint64_t seed, uint64_t stream, uint64_t ctr) {
  uint64_t key = sm64(seed ^ sm64(stream + 0x632BE59BD9B4E019ull));
  return sm64(key + ctr * 0x9E3779B97F4A7C15ull);
}

/* Uniform double in [0, 1) from the top 53 bits. */
static inline double u01(uint64_t r) { return (double)(r >> 11) * (1.0 / 9007199254740992.0); }

/* Uniform integer in [0, bound) by multiply-high (Lemire). */
static inline uint64_t bounded(uint64_t r, uint64_t bound) {
  return (uint64_t)(((unsigned __int128)r * bound) >> 64);
}

uint64_t gg_draw(uint64_t seed, uint64_t stream, uint64_t ctr) { return draw(seed, stream, ctr); }

/* Seeded permutation of [0, n) by Fisher-Yates. */
static void seeded_perm(int32_t* p, int64_t n, uint64_t seed, uint64_t stream) {
  for (int64_t i = 0; i < n; ++i) p[i] = (int32_t)i;
  for (int64_t i = n - 1; i > 0; --i) {
    int64_t j = (int64_t)bounded(draw(seed, stream, (uint64_t)i), (uint64_t)(i + 1));
    int32_t t = p[i]; p[i] = p[j]; p[j] = t;
  }
}

/*
 * R-MAT tuples: each of the m tuples descends `scale` levels of the 2x2
 * quadrant recursion with probabilities (a, b, c, 1-a-b-c).  Vertex labels are
 * then shuffled by a seeded permutation, as the Graph500 Kronecker generator
 * does, so that a label carries no degree information.
 */
int gg_rmat(int32_t scale, int64_t m, double a, double b, double c, uint64_t seed,
            int32_t* src, int32_t* dst) {
  if (scale < 1 || scale > 30 || m < 0 || !src || !dst) return -1;
  const int64_t n = (int64_t)1 << scale;
  const double ab = a + b, abc = a + b + c;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    uint32_t u = 0, v = 0;
    for (int32_t l = 0; l < scale; ++l) {
      double r = u01(draw(seed, 1, (uint64_t)i * 64u + (uint64_t)l));
      uint32_t bu = 0, bv = 0;
      if (r < a) { bu = 0; bv = 0; }
      else if (r < ab) { bu = 0; bv = 1; }
      else if (r < abc) { bu = 1; bv = 0; }
      else { bu = 1; bv = 1; }
      u = (u << 1) | bu;
      v = (v << 1) | bv;
    }
    src[i] = (int32_t)u;
    dst[i] = (int32_t)v;
  }
  int32_t* perm = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  if (!perm) return -2;
  seeded_perm(perm, n, seed, 2);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    src[i] = perm[src[i]];
    dst[i] = perm[dst[i]];
  }
  free(perm);
  return 0;
}

/* Erdos-Renyi G(n, M): m tuples with both endpoints uniform on [0, n). */
int gg_er(int64_t n, int64_t m, uint64_t seed, int32_t* src, int32_t* dst) {
  if (n < 1 || n > 2147483647 || m < 0 || !src || !dst) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    src[i] = (int32_t)bounded(draw(seed, 1, 2 * (uint64_t)i), (uint64_t)n);
    dst[i] = (int32_t)bounded(draw(seed, 1, 2 * (uint64_t)i + 1), (uint64_t)n);
  }
  return 0;
}

/* Number of undirected edges of the full W x H 4-neighbour grid. */
int64_t gg_grid_edges(int32_t w, int32_t h) {
  return (int64_t)(w - 1) * h + (int64_t)w * (h - 1);
}

/*
 * W x H grid, vertex id = y*W + x, with exactly `remove` edges deleted,
 * chosen uniformly without replacement by a partial Fisher-Yates shuffle of
 * the edge indices.  Horizontal edges are numbered first (y*(W-1)+x), then
 * vertical ones ((W-1)*H + y*W + x).  Kept edges are written in index order.
 * Returns the number of tuples written, or <0 on error.
 */
int64_t gg_grid(int32_t w, int32_t h, int64_t remove, uint64_t seed, int32_t* src, int32_t* dst) {
  if (w < 1 || h < 1 || (int64_t)w * h > 2147483647) return -1;
  const int64_t e = gg_grid_edges(w, h);
  if (remove < 0 || remove > e || !src || !dst) return -1;
  uint8_t* gone = (uint8_t*)calloc((size_t)e + 1, 1);
  int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * ((size_t)e + 1));
  if (!gone || !idx) { free(gone); free(idx); return -2; }
  for (int64_t i = 0; i < e; ++i) idx[i] = i;
  for (int64_t i = 0; i < remove; ++i) {
    int64_t j = i + (int64_t)bounded(draw(seed, 3, (uint64_t)i), (uint64_t)(e - i));
    int64_t t = idx[i]; idx[i] = idx[j]; idx[j] = t;
    gone[idx[i]] = 1;
  }
  free(idx);
  const int64_t nh = (int64_t)(w - 1) * h;
  int64_t out = 0;
  for (int64_t k = 0; k < e; ++k) {
    if (gone[k]) continue;
    int64_t u, v;
    if (k < nh) {
      int64_t y = k / (w - 1), x = k % (w - 1);
      u = y * w + x; v = u + 1;
    } else {
      int64_t q = k - nh, y = q / w, x = q % w;
      u = y * w + x; v = u + w;
    }
    src[out] = (int32_t)u;
    dst[out] = (int32_t)v;
    ++out;
  }
  free(gone);
  return out;
}

/*
 * Parameters of a set of Erdos-Renyi graphs with log-uniform sizes:
 * n_i = round(2^U), U ~ U[lo_log2, hi_log2]; mean degree rho_i ~ U[rho_lo, rho_hi];
 * m_i = round(n_i * rho_i / 2) tuples; sub_seed_i is the seed of graph i.
 */
int gg_er_set_params(int32_t count, double lo_log2, double hi_log2, double rho_lo, double rho_hi,
                     uint64_t seed, int64_t* n_out, int64_t* m_out, uint64_t* sub_seed_out) {
  if (count < 0 || !n_out || !m_out || !sub_seed_out) return -1;
  for (int32_t i = 0; i < count; ++i) {
    double uu = u01(draw(seed, 5, 2 * (uint64_t)i));
    double ur = u01(draw(seed, 5, 2 * (uint64_t)i + 1));
    double n = floor(pow(2.0, lo_log2 + (hi_log2 - lo_log2) * uu) + 0.5);
    double rho = rho_lo + (rho_hi - rho_lo) * ur;
    n_out[i] = (int64_t)n;
    m_out[i] = (int64_t)floor(n * rho / 2.0 + 0.5);
    sub_seed_out[i] = draw(seed, 6, (uint64_t)i);
  }
  return 0;
}

/*
 * Draw up to k roots uniformly without replacement from the vertices that
 * appear in at least one tuple whose endpoints differ (exactly the vertices of
 * nonzero degree once self-loops are dropped).  Returns the number drawn.
 */
int32_t gg_pick_roots(const int32_t* src, const int32_t* dst, int64_t m, int64_t n, int32_t k,
                      uint64_t seed, int32_t* out) {
  if (n < 1 || k < 0 || !src || !dst || !out) return -1;
  uint8_t* seen = (uint8_t*)calloc((size_t)n, 1);
  if (!seen) return -2;
  for (int64_t i = 0; i < m; ++i) {
    if (src[i] != dst[i]) { seen[src[i]] = 1; seen[dst[i]] = 1; }
  }
  int64_t cnt = 0;
  for (int64_t v = 0; v < n; ++v) cnt += seen[v];
  int32_t* cand = (int32_t*)malloc(sizeof(int32_t) * (size_t)(cnt + 1));
  if (!cand) { free(seen); return -2; }
  int64_t j = 0;
  for (int64_t v = 0; v < n; ++v) if (seen[v]) cand[j++] = (int32_t)v;
  free(seen);
  int32_t take = (int32_t)(cnt < k ? cnt : k);
  for (int32_t i = 0; i < take; ++i) {
    int64_t r = i + (int64_t)bounded(draw(seed, 7, (uint64_t)i), (uint64_t)(cnt - i));
    int32_t t = cand[i]; cand[i] = cand[r]; cand[r] = t;
    out[i] = cand[i];
  }
  free(cand);
  return take;
}
