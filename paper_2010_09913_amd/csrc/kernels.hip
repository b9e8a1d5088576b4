// HIP kernels of one SlimSell BFS on gfx950 (CDNA4).
//
// One chunk of 64 rows is one 64-lane wavefront: lane = row inside the chunk,
// so the column-major chunk layout (Section II-C, Sell-C-sigma) turns every
// column step into one coalesced 256-byte load of `col`.  A padding cell
// (-1, Section III-B) exec-masks its lane: no gather, no contribution.
//
// Level k (k >= 1) computes x_k from the previous frontier under one semiring
// (Section III-A), derives the new frontier and updates distances/parents in
// the same kernel (the post-processing of the semiring listing), skips chunks
// whose rows are all final (SlimWork, Section III-C) with one wavefront ballot,
// and combines the pieces of split chunks (SlimChunk, Section III-D) with
// order-independent atomics; the last piece to arrive post-processes the chunk.
//
// Update discipline: the gathered vector is double-buffered (Jacobi), except
// for the tropical semiring, which keeps one distance vector and reads every
// value written during the current level (which is exactly k) as infinity, so
// each gather still sees f_{k-1}.  Skipped chunks write nothing: a row whose
// whole chunk is final can only neighbour rows discovered no later than the
// next level, whose update masks it out, so stale values there never reach a
// row that is still undiscovered.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace ss {

__device__ __forceinline__ uint64_t level_tag(uint32_t run_id, int32_t level) {
  return ((uint64_t)run_id << 32) | (uint32_t)level;
}

// ------------------------------------------------------------ semirings ---
//
// Gathers use raw buffer loads: an offset past the end of the buffer returns
// zero without a memory access, so a padding cell (-1) or a bitmap miss needs
// no branch and every load of an unrolled block is issued before the first
// wait.
//
// Each policy gives: live(row), true while the row's value can still change
// (the SlimWork criterion of Section III-C); block<U>(c, acc), the product
// terms of U columns for this lane's row (the gathers); the order-independent
// atomic used to merge SlimChunk pieces; post(row, acc), the per-semiring
// post-processing of the listing in Section III-A; and publish(chunk, mask),
// which stores the chunk's new frontier word where the frontier is a bitmap.

using Rsrc = __amdgpu_buffer_rsrc_t;
constexpr uint32_t kOob = 0x80000000u;  // any offset >= the buffer size reads as 0
constexpr int kRsrcWord3 = 0x00020000;  // raw buffer, gfx9 family

__device__ __forceinline__ Rsrc make_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, kRsrcWord3);
}
__device__ __forceinline__ uint32_t off_of(int32_t c, int shift) {
  return c >= 0 ? ((uint32_t)c << shift) : kOob;
}

// Returning atomics, so that the wait that follows covers their completion.
__device__ __forceinline__ void keep(int32_t v) { asm volatile("" ::"v"(v)); }
__device__ __forceinline__ void wait_memory() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Tropical (min, +): x_k = f_k = A' (x) f_{k-1}, A' has 1 on edges, 0 on the
// diagonal and infinity elsewhere.  The frontier is the distance vector.
struct Tropical {
  using Acc = int32_t;
  __device__ static Acc identity() { return kInf; }
  __device__ static Rsrc rsrc(const LevelArgs& a) { return make_rsrc(a.state, a.n_pad * 4u); }
  __device__ static bool live(const LevelArgs& a, int32_t row) { return a.state[row] == kInf; }
  // terms 1 + f_{k-1}^c; a value >= k was written in this level and stands for infinity
  template <int U>
  __device__ static Acc block(const LevelArgs& a, Rsrc r, const int32_t (&c)[U], Acc acc) {
    int32_t y[U];
#pragma unroll
    for (int t = 0; t < U; ++t) y[t] = __builtin_amdgcn_raw_buffer_load_b32(r, off_of(c[t], 2), 0, 0);
#pragma unroll
    for (int t = 0; t < U; ++t) {
      const int32_t term = (c[t] >= 0 && y[t] < a.level) ? y[t] + 1 : kInf;
      acc = term < acc ? term : acc;
    }
    return acc;
  }
  __device__ static void atomic_combine(const LevelArgs& a, int32_t row, Acc v) {
    keep(atomicMin(&a.acc[row], v));
  }
  __device__ static Acc take(const LevelArgs& a, int32_t row) { return atomicExch(&a.acc[row], kInf); }
  // f_k^row = min(f_{k-1}^row, acc): the zero diagonal of A' keeps the old value
  __device__ static bool post(const LevelArgs& a, int32_t row, Acc acc) {
    const int32_t own = a.state[row];
    const bool fresh = (own == kInf) && (acc != kInf);
    if (fresh) a.state[row] = acc;
    return fresh;
  }
  __device__ static void publish(const LevelArgs&, int32_t, uint64_t, int) {}
};

// Real (+, *): x_k = A (x) f_{k-1}; f_k = [x_k (.) g_k != 0]; d^row = k where
// the row enters the frontier.  Sums of 0/1 values of at most the degree are
// exact in fp32.
struct Real {
  using Acc = float;
  __device__ static Acc identity() { return 0.0f; }
  __device__ static Rsrc rsrc(const LevelArgs& a) { return make_rsrc(a.vin, a.n_pad * 4u); }
  __device__ static bool live(const LevelArgs& a, int32_t row) { return a.g[row] != 0; }
  template <int U>
  __device__ static Acc block(const LevelArgs&, Rsrc r, const int32_t (&c)[U], Acc acc) {
    float y[U];
#pragma unroll
    for (int t = 0; t < U; ++t)
      y[t] = __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off_of(c[t], 2), 0, 0));
#pragma unroll
    for (int t = 0; t < U; ++t) acc += y[t];
    return acc;
  }
  __device__ static void atomic_combine(const LevelArgs& a, int32_t row, Acc v) {
    keep(__float_as_int(atomicAdd(reinterpret_cast<float*>(&a.acc[row]), v)));
  }
  __device__ static Acc take(const LevelArgs& a, int32_t row) {
    return atomicExch(reinterpret_cast<float*>(&a.acc[row]), 0.0f);
  }
  __device__ static bool post(const LevelArgs& a, int32_t row, Acc acc) {
    const uint8_t gg = a.g[row];
    const bool fresh = (acc * (float)gg) != 0.0f;
    static_cast<float*>(a.vout)[row] = fresh ? 1.0f : 0.0f;
    if (fresh) {
      a.d[row] = a.level;
      a.g[row] = 0;
      a.rv[row] = acc;
    }
    return fresh;
  }
  __device__ static void publish(const LevelArgs&, int32_t, uint64_t, int) {}
};

// Boolean (|, &): x_k = A (x) f_{k-1}; f_k = x_k & g_k with a uint8 frontier.
struct Boolean {
  using Acc = uint32_t;
  __device__ static Acc identity() { return 0u; }
  __device__ static Rsrc rsrc(const LevelArgs& a) { return make_rsrc(a.vin, a.n_pad); }
  __device__ static bool live(const LevelArgs& a, int32_t row) { return a.g[row] != 0; }
  template <int U>
  __device__ static Acc block(const LevelArgs&, Rsrc r, const int32_t (&c)[U], Acc acc) {
    uint32_t y[U];
#pragma unroll
    for (int t = 0; t < U; ++t) y[t] = __builtin_amdgcn_raw_buffer_load_b8(r, off_of(c[t], 0), 0, 0);
#pragma unroll
    for (int t = 0; t < U; ++t) acc |= y[t];
    return acc;
  }
  __device__ static void atomic_combine(const LevelArgs& a, int32_t row, Acc v) {
    keep((int32_t)atomicOr(reinterpret_cast<uint32_t*>(&a.acc[row]), v));
  }
  __device__ static Acc take(const LevelArgs& a, int32_t row) {
    return atomicExch(reinterpret_cast<uint32_t*>(&a.acc[row]), 0u);
  }
  __device__ static bool post(const LevelArgs& a, int32_t row, Acc acc) {
    const bool fresh = (acc != 0u) && (a.g[row] != 0);
    static_cast<uint8_t*>(a.vout)[row] = fresh ? 1 : 0;
    if (fresh) {
      a.d[row] = a.level;
      a.g[row] = 0;
    }
    return fresh;
  }
  __device__ static void publish(const LevelArgs&, int32_t, uint64_t, int) {}
};

// Sel-max (max, *): x_k = A (x) x_{k-1}; p_k = p_{k-1} + NOT(p_{k-1}) (.) x_k;
// f_k = NOT NOT x_k minus the visited set; x_k <- NOT NOT x_k (.) v with
// v = original ID + 1, so the max picks the largest original ID among the
// neighbours one level closer.  The x vector is held factored as
// x_{k-1} = f_{k-1} (.) v: a frontier bitmap with one 64-bit word per chunk
// (the wavefront ballot of the rows that entered the frontier) and the static
// v.  A gather tests one bit and reads v only on a hit, so the product is
// evaluated exactly while the gathered array is 32 times smaller.
struct SelMax {
  using Acc = int32_t;
  __device__ static Acc identity() { return 0; }
  __device__ static Rsrc rsrc(const LevelArgs& a) {
    return make_rsrc(a.vin, (uint32_t)(a.n_pad / kC) * 8u);
  }
  __device__ static bool live(const LevelArgs& a, int32_t row) { return a.state[row] == 0; }
  template <int U>
  __device__ static Acc block(const LevelArgs& a, Rsrc r, const int32_t (&c)[U], Acc acc) {
    const Rsrc rv = make_rsrc(a.v, a.n_pad * 4u);
    uint32_t w[U];
#pragma unroll
    for (int t = 0; t < U; ++t)  // the 32-bit half of the chunk word holding bit c
      w[t] = __builtin_amdgcn_raw_buffer_load_b32(r, c[t] >= 0 ? ((uint32_t)c[t] >> 5) << 2 : kOob,
                                                  0, 0);
    int32_t x[U];
#pragma unroll
    for (int t = 0; t < U; ++t) {
      const bool hit = c[t] >= 0 && ((w[t] >> (c[t] & 31)) & 1u);
      x[t] = __builtin_amdgcn_raw_buffer_load_b32(rv, hit ? (uint32_t)c[t] << 2 : kOob, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < U; ++t) acc = x[t] > acc ? x[t] : acc;
    return acc;
  }
  __device__ static void atomic_combine(const LevelArgs& a, int32_t row, Acc v) {
    keep(atomicMax(&a.acc[row], v));
  }
  __device__ static Acc take(const LevelArgs& a, int32_t row) { return atomicExch(&a.acc[row], 0); }
  __device__ static bool post(const LevelArgs& a, int32_t row, Acc acc) {
    const bool fresh = (a.state[row] == 0) && (acc != 0);
    if (fresh) {
      a.state[row] = acc;
      a.d[row] = a.level;
    }
    return fresh;
  }
  __device__ static void publish(const LevelArgs& a, int32_t chunk, uint64_t mask, int lane) {
    if (lane == 0) static_cast<uint64_t*>(a.vout)[chunk] = mask;
  }
};

// Batched boolean SpMM (multi-source BFS): each row carries a 64-bit mask,
// bit b for root slot b.  X = OR over the row's neighbours of F_{k-1};
// new = X & ~visited; visited |= new; F_k = new; the level of every new bit is
// recorded in the row's 64 x 16-bit level record.  A row is final once every
// slot its graph uses has reached it.
struct Batch {
  using Acc = unsigned long long;
  __device__ static Acc identity() { return 0ull; }
  __device__ static Rsrc rsrc(const LevelArgs& a) { return make_rsrc(a.vin, a.n_pad * 8u); }
  __device__ static bool live(const LevelArgs& a, int32_t row) {
    const Acc full = a.full[row / kC];
    return (a.vis[row] & full) != full;
  }
  template <int U>
  __device__ static Acc block(const LevelArgs&, Rsrc r, const int32_t (&c)[U], Acc acc) {
    Acc y[U];
#pragma unroll
    for (int t = 0; t < U; ++t) {
      const auto w = __builtin_amdgcn_raw_buffer_load_b64(r, off_of(c[t], 3), 0, 0);
      y[t] = ((Acc)w[1] << 32) | (Acc)w[0];
    }
#pragma unroll
    for (int t = 0; t < U; ++t) acc |= y[t];
    return acc;
  }
  __device__ static void atomic_combine(const LevelArgs& a, int32_t row, Acc v) {
    keep((int32_t)atomicOr(&a.acc64[row], v));
  }
  __device__ static Acc take(const LevelArgs& a, int32_t row) { return atomicExch(&a.acc64[row], 0ull); }
  __device__ static bool post(const LevelArgs& a, int32_t row, Acc acc) {
    const Acc seen = a.vis[row];
    Acc fresh = acc & ~seen & a.full[row / kC];
    static_cast<Acc*>(a.vout)[row] = fresh;
    if (fresh) {
      a.vis[row] = seen | fresh;
      uint16_t* lv = a.lvl + (int64_t)row * 64;
      const uint16_t k = (uint16_t)a.level;
      for (Acc m = fresh; m; m &= m - 1) lv[__ffsll((long long)m) - 1] = k;
    }
    return fresh != 0ull;
  }
  __device__ static void publish(const LevelArgs&, int32_t, uint64_t, int) {}
};

// ---------------------------------------------------------- level kernel ---

__device__ __forceinline__ int32_t wave_max(int32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const int32_t o = __shfl_xor(v, off);
    v = o > v ? o : v;
  }
  return v;
}

// Sweep `ncols` columns of one chunk for this lane's row, U columns at a time:
// U independent streaming loads of `col`, then the U gathers of the block.  A
// lane that is off (its row is final) issues no loads at all.
template <class S, int U>
__device__ __forceinline__ typename S::Acc sweep(const LevelArgs& a, Rsrc r,
                                                 const int32_t* __restrict__ p, int32_t ncols,
                                                 bool on) {
  typename S::Acc acc = S::identity();
  if (!on) return acc;
  int32_t j = 0;
  for (; j + U <= ncols; j += U) {
    int32_t c[U];
#pragma unroll
    for (int t = 0; t < U; ++t) c[t] = __builtin_nontemporal_load(p + (int64_t)t * kC);
    acc = S::template block<U>(a, r, c, acc);
    p += (int64_t)U * kC;
  }
  for (; j < ncols; ++j) {
    int32_t c[1] = {__builtin_nontemporal_load(p)};
    acc = S::template block<1>(a, r, c, acc);
    p += kC;
  }
  return acc;
}

// Post-process the rows of one chunk; returns how many entered the frontier.
template <class S>
__device__ __forceinline__ uint32_t finish_rows(const LevelArgs& a, int32_t chunk, int32_t row,
                                                typename S::Acc acc, int lane) {
  const bool fresh = S::post(a, row, acc);
  const uint64_t mask = __ballot(fresh);
  S::publish(a, chunk, mask, lane);
  return (uint32_t)__popcll(mask);
}

// One BFS level.  slimwork: 0 = every row of every chunk is computed;
// 1 = chunks whose rows are all final are skipped (Section III-C);
// 2 = additionally a lane whose row is final issues no loads and the sweep
// stops at the longest row that is still live.
template <class S, int U>
__global__ void level_kernel(LevelArgs a) {
  const int lane = threadIdx.x & (kC - 1);
  const int wave = threadIdx.x / kC;
  const int waves = blockDim.x / kC;

  // Stop if the previous level discovered nothing, and tell the host what the
  // previous level found (one thread of the first workgroup).
  if (a.level > 1) {
    const uint64_t want = level_tag(a.run_id, a.level - 1);
    const bool prev_found = (a.any[(a.level - 1) % kRing] == want);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      __hip_atomic_store(&a.report[(a.level - 1) % kRing], (want << 1) | (prev_found ? 1u : 0u),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    if (!prev_found) return;
  }

  const Rsrc rs = S::rsrc(a);
  // per-wavefront tallies, flushed once at the end
  uint32_t found = 0, n_chunks = 0;
  uint64_t n_cols = 0;
  int32_t max_cl = 0;

  for (int64_t u = (int64_t)blockIdx.x * waves + wave; u < a.n_units;
       u += (int64_t)gridDim.x * waves) {
    const Unit w = a.units[u];
    const bool piece = (w.c1 == w.c0 + 1);
    for (int32_t c = w.c0; c < w.c1; ++c) {
      const int32_t row = c * kC + lane;
      const bool live = S::live(a, row);
      if (a.slimwork && !__any(live)) continue;  // whole chunk final
      int32_t j0 = 0, j1 = a.cl[c];
      if (piece) { j0 = w.j0; j1 = w.j1; }
      if (j0 == 0) {
        ++n_chunks;
        const int32_t len = a.cl[c];
        max_cl = len > max_cl ? len : max_cl;
      }
      const bool on = (a.slimwork >= 2) ? live : true;
      int32_t hi = j1;
      if (a.slimwork >= 2) {
        const int32_t lim = wave_max(on ? a.deg[row] : 0);
        hi = lim < j1 ? lim : j1;
      }
      const int32_t ncols = hi > j0 ? hi - j0 : 0;
      n_cols += (uint64_t)ncols;
      const int32_t* p = a.col + a.cs[c] + (int64_t)j0 * kC + lane;
      typename S::Acc acc = sweep<S, U>(a, rs, p, ncols, on);
      const int32_t npieces = piece ? a.pieces[c] : 1;
      if (npieces == 1) {
        found += finish_rows<S>(a, c, row, acc, lane);
      } else {
        // SlimChunk: combine this piece, the last one to arrive post-processes.
        // Pieces exchange data only through device-scope atomics: each piece's
        // combine has completed before its arrival is counted, so the last
        // arrival's exchange sees every piece.
        S::atomic_combine(a, row, acc);
        wait_memory();
        int last = 0;
        if (lane == 0) last = (atomicAdd(&a.arrive[c], 1) == npieces - 1);
        last = __shfl(last, 0);
        if (last) {
          acc = S::take(a, row);
          if (lane == 0) a.arrive[c] = 0;
          found += finish_rows<S>(a, c, row, acc, lane);
        }
      }
    }
  }
  if (lane == 0) {
    if (found) a.any[a.level % kRing] = level_tag(a.run_id, a.level);
    if (a.count_stats && (found | n_chunks | n_cols)) {
      unsigned long long* ctr =
          a.counters + ((int64_t)a.level * kCountSlots + (blockIdx.x % kCountSlots)) * kCountFields;
      if (found) atomicAdd(&ctr[0], (unsigned long long)found);
      if (n_chunks) {
        atomicAdd(&ctr[1], (unsigned long long)n_chunks);
        atomicMax(&ctr[3], (unsigned long long)max_cl);
      }
      if (n_cols) atomicAdd(&ctr[2], (unsigned long long)n_cols * kC);
    }
  }
}

// ----------------------------------------------------------- init kernel ---

// Level-0 vectors (Section III-A): tropical x_0 = f_0 = e_r-style distances,
// real/boolean f_0 = e_r with filter g = NOT f_0, sel-max x_0 = p_0 = (r+1) e_r.
// Phantom rows start final so SlimWork can skip them.
template <int SEMI>
__global__ void init_kernel(int32_t n, int32_t n_pad, int64_t n_chunks, const int32_t* v,
                            int32_t root_row, void* va, void* vb, int32_t* state, uint8_t* g,
                            int32_t* d, float* rv, int32_t* acc, int32_t* arrive) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n_chunks) arrive[r] = 0;
  if (r >= n_pad) return;
  // sel-max: one bitmap word per chunk is initialised below
  const bool root = (r == root_row);
  const bool phantom = (v[r] == 0);
  if (SEMI == SS_TROPICAL) {
    state[r] = root ? 0 : (phantom ? 0 : kInf);
    acc[r] = kInf;
    return;
  }
  d[r] = root ? 0 : -1;
  g[r] = (root || phantom) ? 0 : 1;
  if (SEMI == SS_REAL) {
    static_cast<float*>(va)[r] = root ? 1.0f : 0.0f;
    static_cast<float*>(vb)[r] = 0.0f;
    rv[r] = root ? 1.0f : 0.0f;
    reinterpret_cast<float*>(acc)[r] = 0.0f;
  } else if (SEMI == SS_BOOLEAN) {
    static_cast<uint8_t*>(va)[r] = root ? 1 : 0;
    static_cast<uint8_t*>(vb)[r] = 0;
    acc[r] = 0;
  } else {  // SS_SELMAX: frontier bitmap f_0 = e_r (x_0 = f_0 (.) v), p_0 = x_0
    if (r < n_chunks)
      static_cast<uint64_t*>(va)[r] = (r == root_row / kC) ? (1ull << (root_row % kC)) : 0ull;
    state[r] = root ? v[r] : (phantom ? -1 : 0);
    acc[r] = 0;
  }
}

// ------------------------------------------------------- finalise kernel ---

// Row order -> original IDs; infinity -> -1; 1-based parents -> 0-based.
template <int SEMI>
__global__ void finalise_kernel(int32_t n, const int32_t* perm, const int32_t* state,
                                const int32_t* d, const float* rv, int32_t* dist, int32_t* parent,
                                float* real_val) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n) return;
  const int32_t row = perm[o];
  if (SEMI == SS_TROPICAL) {
    const int32_t f = state[row];
    dist[o] = (f >= kInf) ? -1 : f;
    return;
  }
  dist[o] = d[row];
  if (SEMI == SS_SELMAX && parent) {
    const int32_t pr = state[row];
    parent[o] = (pr > 0) ? pr - 1 : -1;
  }
  if (SEMI == SS_REAL && real_val) real_val[o] = rv[row];
}

// Batched level 0: every row starts with an empty mask (phantom rows are
// final); then each used root slot sets its bit and level 0 at its root row.
__global__ void batch_init_kernel(int32_t n_pad, int64_t n_chunks, const int32_t* v,
                                  unsigned long long* vis, unsigned long long* fa,
                                  unsigned long long* acc64, int32_t* arrive) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n_chunks) arrive[r] = 0;
  if (r >= n_pad) return;
  vis[r] = (v[r] == 0) ? ~0ull : 0ull;
  fa[r] = 0ull;
  acc64[r] = 0ull;
}

__global__ void batch_roots_kernel(int32_t count, const int32_t* root_rows, const int32_t* slots,
                                   unsigned long long* vis, unsigned long long* fa,
                                   uint16_t* lvl) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int32_t row = root_rows[i];
  const unsigned long long bit = 1ull << slots[i];
  atomicOr(&vis[row], bit);
  atomicOr(&fa[row], bit);
  lvl[(int64_t)row * 64 + slots[i]] = 0;
}

// Row records -> dist[graph block][slot][vertex]; unreached and unused = -1.
__global__ void batch_finalise_kernel(int64_t n, int32_t num_graphs, const int64_t* voff,
                                      const int32_t* perm, const unsigned long long* vis,
                                      const uint16_t* lvl, int32_t rpg, int32_t* dist) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n) return;
  int32_t lo = 0, hi = num_graphs - 1;  // graph of o: last i with voff[i] <= o
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) / 2;
    if (voff[mid] <= o) lo = mid; else hi = mid - 1;
  }
  const int64_t base = voff[lo], ni = voff[lo + 1] - base;
  const int32_t row = perm[o];
  const unsigned long long seen = vis[row];
  const uint16_t* lv = lvl + (int64_t)row * 64;
  int32_t* out = dist + (int64_t)rpg * base + (o - base);
  for (int32_t b = 0; b < rpg; ++b) out[(int64_t)b * ni] = ((seen >> b) & 1ull) ? (int32_t)lv[b] : -1;
}

template <class T>
__global__ void fill_kernel(T* p, T value, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

// --------------------------------------------------------------- launchers ---

static int check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(SS_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  return SS_OK;
}

static inline unsigned blocks_for(int64_t n, int threads) {
  return (unsigned)((n + threads - 1) / threads);
}

int launch_init(int semiring, const Graph& g, const Workspace& ws, int32_t root_row,
                void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t work = g.n_pad > g.n_chunks ? g.n_pad : g.n_chunks;
  const unsigned blocks = blocks_for(work, 256);
#define SS_INIT(S)                                                                             \
  init_kernel<S><<<blocks, 256, 0, st>>>(g.n, g.n_pad, g.n_chunks, g.d_v, root_row, ws.vec_a, \
                                         ws.vec_b, ws.state, ws.g, ws.d, ws.rv, ws.acc,       \
                                         ws.arrive)
  switch (semiring) {
    case SS_TROPICAL: SS_INIT(SS_TROPICAL); break;
    case SS_REAL: SS_INIT(SS_REAL); break;
    case SS_BOOLEAN: SS_INIT(SS_BOOLEAN); break;
    case SS_SELMAX: SS_INIT(SS_SELMAX); break;
    default: return set_error(SS_EINVAL, "unknown semiring");
  }
#undef SS_INIT
  return check_launch("init_kernel");
}

template <class S>
static void launch_level_t(int waves, int unroll, unsigned grid, const LevelArgs& a,
                           hipStream_t st) {
  if (unroll == 4)
    level_kernel<S, 4><<<grid, waves * kC, 0, st>>>(a);
  else if (unroll == 16)
    level_kernel<S, 16><<<grid, waves * kC, 0, st>>>(a);
  else
    level_kernel<S, 8><<<grid, waves * kC, 0, st>>>(a);
}

int launch_level(int semiring, int waves, int unroll, int64_t max_groups, const LevelArgs& a,
                 void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  int64_t groups = (a.n_units + waves - 1) / waves;
  if (groups < 1) groups = 1;
  if (max_groups > 0 && groups > max_groups) groups = max_groups;
  const unsigned grid = (unsigned)groups;
  switch (semiring) {
    case SS_TROPICAL: launch_level_t<Tropical>(waves, unroll, grid, a, st); break;
    case SS_REAL: launch_level_t<Real>(waves, unroll, grid, a, st); break;
    case SS_BOOLEAN: launch_level_t<Boolean>(waves, unroll, grid, a, st); break;
    case SS_SELMAX: launch_level_t<SelMax>(waves, unroll, grid, a, st); break;
    case kBatchSemiring: launch_level_t<Batch>(waves, unroll, grid, a, st); break;
    default: return set_error(SS_EINVAL, "unknown semiring");
  }
  return check_launch("level_kernel");
}

int launch_finalise(int semiring, const Graph& g, const Workspace& ws, int32_t* dist,
                    int32_t* parent, float* real_val, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  const unsigned blocks = blocks_for(g.n, 256);
#define SS_FIN(S)                                                                          \
  finalise_kernel<S><<<blocks, 256, 0, st>>>(g.n, g.d_perm, ws.state, ws.d, ws.rv, dist, \
                                             parent, real_val)
  switch (semiring) {
    case SS_TROPICAL: SS_FIN(SS_TROPICAL); break;
    case SS_REAL: SS_FIN(SS_REAL); break;
    case SS_BOOLEAN: SS_FIN(SS_BOOLEAN); break;
    case SS_SELMAX: SS_FIN(SS_SELMAX); break;
    default: return set_error(SS_EINVAL, "unknown semiring");
  }
#undef SS_FIN
  return check_launch("finalise_kernel");
}

int launch_fill_i32(int32_t* p, int32_t value, int64_t count, void* stream) {
  if (count <= 0) return SS_OK;
  unsigned blocks = blocks_for(count, 256);
  if (blocks > 4096) blocks = 4096;
  fill_kernel<int32_t><<<blocks, 256, 0, static_cast<hipStream_t>(stream)>>>(p, value, count);
  return check_launch("fill_kernel");
}

int launch_batch_init(const Graph& g, const BatchWorkspace& b, int32_t count, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  batch_init_kernel<<<blocks_for(g.n_pad, 256), 256, 0, st>>>(g.n_pad, g.n_chunks, g.d_v, b.vis,
                                                              b.fa, b.acc64, g.ws.arrive);
  int rc = check_launch("batch_init_kernel");
  if (rc || count == 0) return rc;
  batch_roots_kernel<<<blocks_for(count, 256), 256, 0, st>>>(count, b.root_rows, b.slots, b.vis,
                                                             b.fa, b.lvl);
  return check_launch("batch_roots_kernel");
}

int launch_batch_finalise(const Graph& g, const BatchWorkspace& b, int32_t rpg, int32_t* dist,
                          void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  batch_finalise_kernel<<<blocks_for(g.n, 256), 256, 0, st>>>(
      g.n, g.num_graphs, g.d_voff, g.d_perm, b.vis, b.lvl, rpg, dist);
  return check_launch("batch_finalise_kernel");
}

int launch_fill_u64(unsigned long long* p, unsigned long long value, int64_t count,
                    void* stream) {
  if (count <= 0) return SS_OK;
  unsigned blocks = blocks_for(count, 256);
  if (blocks > 4096) blocks = 4096;
  fill_kernel<unsigned long long><<<blocks, 256, 0, static_cast<hipStream_t>(stream)>>>(
      p, value, count);
  return check_launch("fill_kernel");
}

}  // namespace ss
