// DP transformation on the GPU (Section II-C): parents from distances.
//
// For a reached vertex v other than the root, its parent is a neighbour one
// level closer to the root; the largest such original ID is taken (the
// tie-break the sel-max semiring produces), the root is its own parent and an
// unreached vertex has none.  This is what the tropical, real and boolean
// formulations need after the BFS to report parents ("DP" in the paper's
// measurements); sel-max computes them during the BFS.
//
// Three kernels: the row distances and their 2-bit codes (distance mod 3, 3
// = unreached, four rows per byte); one pass of the level kernel under the
// Dp policy (kernels.hip), which sweeps the SlimSell layout with the reached
// rows live, gathers codes, reads v of the neighbours whose code is one level
// closer and keeps the largest, each row stopping at its first hit; and the
// map from rows back to original IDs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "device.h"
#include "internal.h"

namespace ss {

// Row-order distances and their codes, one thread per row; the SlimChunk
// combine buffer and the arrival counters start at zero.  The distances come
// from the original-order `dist` (a gather through v), or, right after a BFS
// on this workspace, from its own row-order state: the tropical distance
// vector (kInf: unreached) or the distances the real and boolean forms keep
// in `drow` itself.  The best v of a row needs no clearing: the sweep writes
// it for every row of every chunk it processes, and only reached rows (all
// in processed chunks) read it.  n_pad is a multiple of 64, so a wavefront
// is either wholly in range or wholly out.
__global__ void dp_prep_kernel(int32_t n_pad, int64_t n_chunks, const int32_t* v,
                               const int32_t* dist, int32_t src, const int32_t* state,
                               int32_t* drow, uint8_t* code, int32_t* acc, int32_t* arrive) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n_chunks) arrive[r] = 0;
  if (r >= n_pad) return;
  int32_t d;
  if (src == kDpFromRowD) {
    d = drow[r];  // -1 for unreached and phantom rows
  } else {
    const int32_t o = v[r] - 1;
    if (src == kDpFromDist) {
      d = o >= 0 ? dist[o] : -1;
    } else {
      const int32_t f = state[r];
      d = (o < 0 || f >= kInf) ? -1 : f;
    }
    drow[r] = d;
  }
  acc[r] = 0;
  const uint32_t c = d < 0 ? 3u : (uint32_t)(d % 3);
  const uint32_t c1 = __shfl_down(c, 1), c2 = __shfl_down(c, 2), c3 = __shfl_down(c, 3);
  if ((threadIdx.x & 3) == 0) code[r >> 2] = (uint8_t)(c | (c1 << 2) | (c2 << 4) | (c3 << 6));
}

// Row order -> original IDs, one thread per original ID (coalesced writes,
// gathered reads): the root (distance 0) is its own parent; a reached vertex
// with no qualifying neighbour (only for inconsistent input) and an
// unreached one get -1.  `best` holds v (original ID + 1) of the parent.
// With `dist` (not NULL) the pass also writes the distances (-1: unreached),
// so a BFS followed by the transformation converts its distances here, in
// the same gather, instead of in a pass of its own.
__global__ void dp_finalise_kernel(int32_t n, const int32_t* perm, const int32_t* drow,
                                   const int32_t* best, int32_t* parent, int32_t* dist) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n) return;
  const int32_t row = __builtin_nontemporal_load(perm + o);
  const int32_t d = drow[row];
  if (dist) __builtin_nontemporal_store(d, dist + o);
  int32_t p = -1;
  if (d == 0) p = (int32_t)o;
  else if (d > 0) {
    const int32_t b = best[row];
    p = b > 0 ? b - 1 : -1;
  }
  __builtin_nontemporal_store(p, parent + o);
}

int launch_dp(const Graph& g, const Workspace& ws, const UnitList& ul,
              const UnitList::Assignment* as, int unroll, int waves, int64_t max_groups,
              const int32_t* dist, int32_t src, int32_t* dist_out, int32_t* parent,
              void* stream, unsigned long long* counters, void* ev_begin, void* ev_end) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t work = std::max<int64_t>(g.n_pad, g.n_chunks);
  const unsigned blocks = (unsigned)((work + 255) / 256);
  dp_prep_kernel<<<blocks, 256, 0, st>>>((int32_t)g.n_pad, g.n_chunks, g.d_v, dist, src, ws.state,
                                         ws.d, ws.g, ws.acc, ws.arrive);
  int rc = check_launch("dp_prep_kernel");
  if (rc) return rc;
  LevelArgs a;
  std::memset(&a, 0, sizeof(a));
  a.col = g.d_col;
  a.cs = g.d_cs;
  a.cl = g.d_cl;
  a.v = g.d_v;
  a.deg = g.d_deg;
  a.units = ul.d_units;
  a.pieces = ul.d_pieces;
  a.n_units = ul.count;
  a.bundle = ul.d_bundle;
  a.arrive2 = ul.d_arrive2;
  a.piece_cols = ul.split_len;
  if (as) {
    a.units = as->d_units;
    a.wave_off = as->d_off;
  }
  a.vin = ws.g;       // the codes
  a.state = ws.state; // best v per row
  a.d = ws.d;         // row distances
  a.acc = ws.acc;
  a.arrive = ws.arrive;
  a.any = ws.any;
  a.counters = counters;
  a.count_stats = counters ? 1 : 0;
  a.n_pad = (uint32_t)g.n_pad;
  a.level = 1;        // one pass; the level tags and reports are not used
  a.slimwork = 2;
  // the prefix of the codes each workgroup stages in LDS (the graph's
  // configured prefix size; codes are a quarter byte per row)
  const int64_t want = std::min<int64_t>(g.n_pad / 4, (int64_t)g.tune.lds_kib * 1024);
  a.lds_bytes = (uint32_t)(std::min<int64_t>(want, g.lds_cap > 0 ? g.lds_cap : 0) / 16 * 16);
  if (ul.count > 0) {
    if (ev_begin && hipEventRecord(static_cast<hipEvent_t>(ev_begin), st) != hipSuccess)
      return set_error(SS_EHIP, "hipEventRecord (DP sweep)");
    if ((rc = launch_level(kDpSemiring, waves, unroll, max_groups, a, stream))) return rc;
    if (ev_end && hipEventRecord(static_cast<hipEvent_t>(ev_end), st) != hipSuccess)
      return set_error(SS_EHIP, "hipEventRecord (DP sweep)");
  }
  const unsigned n_blocks = (unsigned)((g.n + 255) / 256);
  if (n_blocks)
    dp_finalise_kernel<<<n_blocks, 256, 0, st>>>((int32_t)g.n, g.d_perm, ws.d, ws.state, parent,
                                                 src == kDpFromDist ? nullptr : dist_out);
  return check_launch("dp_finalise_kernel");
}

}  // namespace ss
