// DP transformation on the GPU (Section II-C): parents from distances.
//
// For a reached vertex v other than the root, its parent is a neighbour one
// level closer to the root; the largest such original ID is taken (the
// tie-break the sel-max semiring produces), the root is its own parent and an
// unreached vertex has none.  This is what the tropical, real and boolean
// formulations need after the BFS to report parents ("DP" in the paper's
// measurements); sel-max computes them during the BFS.
//
// One sweep of the SlimSell layout with every row live: lane = row, column
// by column.  The gathered vector is not the distance itself but a 2-bit code
// per row, distance mod 3 (3 = unreached): a neighbour u of a vertex at
// level k is at level k-1, k or k+1, which the code tells apart, so the
// gathered array is n/4 bytes (1 MB for 4M vertices, resident in L2) instead
// of 4n.  A hit then reads v[u] (original ID + 1).  A row lists its
// neighbours by decreasing original ID, so a lane stops at its first hit.
// Pieces of split chunks combine with atomicMax, which is order-independent.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.h"
#include "internal.h"

namespace ss {

constexpr int64_t kDpCodeLds = 48 * 1024;  // codes of the first 192K rows
constexpr int64_t kDpVLds = 16 * 1024;     // v of the first 4K rows

struct DpArgs {
  const int32_t* col;
  const int64_t* cs;
  const int32_t* cl;
  const int32_t* v;
  const int32_t* deg;
  const Unit* units;
  const int32_t* pieces;
  int64_t n_units;
  const int32_t* drow;  // distance of each row (-1 unreached or phantom)
  const uint8_t* code;  // 2-bit distance mod 3 per row, 4 rows per byte
  int32_t* acc;         // largest v of a qualifying neighbour, per row
  uint32_t n_pad;
  uint32_t code_lds, v_lds;  // bytes of codes and of v staged in LDS (multiples of 16)
};

// Row-order distances and their codes, one thread per row.  n_pad is a
// multiple of 64, so a wavefront is either wholly in range or wholly out.
__global__ void dp_prep_kernel(int32_t n_pad, const int32_t* v, const int32_t* dist, int32_t* drow,
                               uint8_t* code, int32_t* acc) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_pad) return;
  const int32_t o = v[r] - 1;
  const int32_t d = o >= 0 ? dist[o] : -1;
  drow[r] = d;
  acc[r] = 0;
  const uint32_t c = d < 0 ? 3u : (uint32_t)(d % 3);
  const uint32_t c1 = __shfl_down(c, 1), c2 = __shfl_down(c, 2), c3 = __shfl_down(c, 3);
  if ((threadIdx.x & 3) == 0) code[r >> 2] = (uint8_t)(c | (c1 << 2) | (c2 << 4) | (c3 << 6));
}

// With STAGED, each workgroup first copies the first code_lds bytes of the
// codes and the first v_lds bytes of v into LDS: with a full sort the rows of
// highest degree, the most gathered, come first.
template <int U, bool STAGED>
__global__ void dp_sweep_kernel(DpArgs a) {
  extern __shared__ uint8_t lds[];
  const int lane = threadIdx.x & (kC - 1);
  const int wave = threadIdx.x / kC;
  const int waves = blockDim.x / kC;
  const Rsrc rc = make_rsrc(a.code, a.n_pad / 4u);
  const Rsrc rv = make_rsrc(a.v, a.n_pad * 4u);
  Stage sc{lds, 0u}, sv{lds + a.code_lds, 0u};
  if (STAGED) {
    const uint4* c4 = reinterpret_cast<const uint4*>(a.code);
    const uint4* v4 = reinterpret_cast<const uint4*>(a.v);
    uint4* d4 = reinterpret_cast<uint4*>(lds);
    const uint32_t nc = a.code_lds / 16u, nv = a.v_lds / 16u;
    for (uint32_t i = threadIdx.x; i < nc + nv; i += blockDim.x)
      d4[i] = i < nc ? c4[i] : v4[i - nc];
    __syncthreads();
    sc.bytes = a.code_lds;
    sv.bytes = a.v_lds;
  }
  for (int64_t u = (int64_t)blockIdx.x * waves + wave; u < a.n_units;
       u += (int64_t)gridDim.x * waves) {
    const Unit w = a.units[u];
    const bool piece = (w.c1 == w.c0 + 1) && a.pieces[w.c0] > 1;
    for (int32_t c = w.c0; c < w.c1; ++c) {
      const int32_t row = c * kC + lane;
      const int32_t d = a.drow[row];
      const bool on = d >= 1;
      if (!__any(on)) continue;  // acc is already 0
      const uint32_t want = on ? (uint32_t)((d - 1) % 3) : 4u;  // 4 matches no code
      int32_t j0 = 0, j1 = a.cl[c];
      if (w.c1 == w.c0 + 1) {
        j0 = w.j0;
        j1 = w.j1;
      }
      const int32_t lim = wave_max(on ? a.deg[row] : 0);
      const int32_t hi = lim < j1 ? lim : j1;
      const int32_t* p = a.col + a.cs[c] + (int64_t)j0 * kC + lane;
      int32_t best = 0;
      int32_t j = j0;
      for (; j + U <= hi; j += U) {
        int32_t cc[U];
#pragma unroll
        for (int t = 0; t < U; ++t) cc[t] = on ? __builtin_nontemporal_load(p + (int64_t)t * kC) : -1;
        uint32_t b[U];
#pragma unroll
        for (int t = 0; t < U; ++t)
          b[t] = gather_b8<STAGED>(rc, sc, cc[t] >= 0 ? (uint32_t)cc[t] >> 2 : kOob);
        int32_t x[U];
#pragma unroll
        for (int t = 0; t < U; ++t) {
          const bool hit = cc[t] >= 0 && ((b[t] >> ((cc[t] & 3) * 2)) & 3u) == want;
          x[t] = (int32_t)gather_b32<STAGED>(rv, sv, hit ? (uint32_t)cc[t] << 2 : kOob);
        }
#pragma unroll
        for (int t = 0; t < U; ++t) best = x[t] > best ? x[t] : best;
        p += (int64_t)U * kC;
        if (best > 0) break;  // rows list neighbours by decreasing ID: the first is the largest
      }
      for (; best == 0 && j < hi; ++j) {
        const int32_t c1 = on ? __builtin_nontemporal_load(p) : -1;
        const uint32_t b1 = gather_b8<STAGED>(rc, sc, c1 >= 0 ? (uint32_t)c1 >> 2 : kOob);
        const bool hit = c1 >= 0 && ((b1 >> ((c1 & 3) * 2)) & 3u) == want;
        const int32_t x1 = (int32_t)gather_b32<STAGED>(rv, sv, hit ? (uint32_t)c1 << 2 : kOob);
        best = x1 > best ? x1 : best;
        p += kC;
      }
      if (piece) {
        if (best > 0) atomicMax(&a.acc[row], best);
      } else {
        a.acc[row] = best;
      }
    }
  }
}

// Row order -> original IDs: root (distance 0) is its own parent; a reached
// vertex with no qualifying neighbour (only for inconsistent input) and an
// unreached one get -1.
__global__ void dp_finalise_kernel(int32_t n_pad, const int32_t* v, const int32_t* drow,
                                   const int32_t* acc, int32_t* parent) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_pad) return;
  const int32_t o = v[r] - 1;
  if (o < 0) return;
  const int32_t d = drow[r];
  const int32_t best = acc[r];
  parent[o] = d == 0 ? o : ((d > 0 && best > 0) ? best - 1 : -1);
}

int launch_dp(const Graph& g, const Workspace& ws, const UnitList& ul, int unroll, int waves,
              int64_t max_groups, const int32_t* dist, int32_t* parent, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  const unsigned rows_blocks = (unsigned)((g.n_pad + 255) / 256);
  dp_prep_kernel<<<rows_blocks, 256, 0, st>>>((int32_t)g.n_pad, g.d_v, dist, ws.d, ws.g, ws.acc);
  int rc = check_launch("dp_prep_kernel");
  if (rc) return rc;
  DpArgs a;
  a.col = g.d_col;
  a.cs = g.d_cs;
  a.cl = g.d_cl;
  a.v = g.d_v;
  a.deg = g.d_deg;
  a.units = ul.d_units;
  a.pieces = ul.d_pieces;
  a.n_units = ul.count;
  a.drow = ws.d;
  a.code = ws.g;
  a.acc = ws.acc;
  a.n_pad = (uint32_t)g.n_pad;
  // LDS prefixes: up to 48 KiB of codes and 16 KiB of v, within what the
  // device gives a workgroup
  const int64_t cap = g.lds_cap > 0 ? g.lds_cap : 0;
  int64_t cb = std::min<int64_t>(g.n_pad / 4, kDpCodeLds) / 16 * 16;
  int64_t vb = std::min<int64_t>(g.n_pad * 4, kDpVLds) / 16 * 16;
  if (cb + vb > cap) {
    cb = std::min<int64_t>(cb, cap) / 16 * 16;
    vb = std::max<int64_t>(0, cap - cb) / 16 * 16;
  }
  a.code_lds = (uint32_t)cb;
  a.v_lds = (uint32_t)vb;
  if (ul.count > 0) {
    int64_t blocks = (ul.count + waves - 1) / waves;
    if (max_groups > 0 && blocks > max_groups) blocks = max_groups;
    const dim3 grid((unsigned)blocks), block((unsigned)(waves * kC));
    const size_t lds = (size_t)(cb + vb);
    if (lds == 0) {
      if (unroll == 4)
        dp_sweep_kernel<4, false><<<grid, block, 0, st>>>(a);
      else if (unroll == 16)
        dp_sweep_kernel<16, false><<<grid, block, 0, st>>>(a);
      else
        dp_sweep_kernel<8, false><<<grid, block, 0, st>>>(a);
    } else {
      if (unroll == 4)
        dp_sweep_kernel<4, true><<<grid, block, lds, st>>>(a);
      else if (unroll == 16)
        dp_sweep_kernel<16, true><<<grid, block, lds, st>>>(a);
      else
        dp_sweep_kernel<8, true><<<grid, block, lds, st>>>(a);
    }
    if ((rc = check_launch("dp_sweep_kernel"))) return rc;
  }
  dp_finalise_kernel<<<rows_blocks, 256, 0, st>>>((int32_t)g.n_pad, g.d_v, ws.d, ws.acc, parent);
  return check_launch("dp_finalise_kernel");
}

}  // namespace ss
