// HIP kernels of one SlimSell BFS on gfx950 (CDNA4).
//
// One chunk of 64 rows is one 64-lane wavefront: lane = row inside the chunk,
// so the column-major chunk layout (Section II-D, Sell-C-sigma) turns every
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

#include "device.h"
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

// Tropical (min, +): x_k = f_k = A' (x) f_{k-1}, A' has 1 on edges, 0 on the
// diagonal and infinity elsewhere.  The frontier is the distance vector.
struct Tropical {
  static constexpr bool kSingleRoot = true;
  static constexpr bool kBitmapFrontier = false;
  __device__ static void skip_chunk(const LevelArgs&, int32_t) {}
  using Acc = int32_t;
  // the first product term a row receives is its final value
  static constexpr bool kFirstHitFinal = true;
  // per-lane value the product terms of a row depend on (none here)
  __device__ static uint32_t context(const LevelArgs&, int32_t) { return 0u; }
  __device__ static bool settled(Acc acc) { return acc != kInf; }
  __device__ static Acc identity() { return kInf; }
  __device__ static Rsrc rsrc(const LevelArgs& a) { return make_rsrc(a.state, a.n_pad * 4u); }
  using Raw = int32_t;  // the word the live test reads
  __device__ static Raw raw(const LevelArgs& a, int32_t row) { return a.state[row]; }
  __device__ static bool is_live(const LevelArgs&, Raw w, int32_t) { return w == kInf; }
  __device__ static bool live(const LevelArgs& a, int32_t row) { return a.state[row] == kInf; }
  __device__ static bool still_live(const LevelArgs&, int32_t, bool live, bool fresh) {
    return live && !fresh;
  }
  // terms 1 + f_{k-1}^c; a value >= k was written in this level and stands for infinity
  __device__ static const void* staged(const LevelArgs& a) { return a.state; }
  template <int U, bool STAGED>
  __device__ static Acc block(const LevelArgs& a, Rsrc r, Stage st, const int32_t (&c)[U],
                              Acc acc, uint32_t) {
    uint32_t y[U];
    bool got[U];
    gather_rows<U, STAGED, 1>(r, st, c, y, got);
    // a term left unread (its chunk had no frontier row) is infinity: a live
    // row has no neighbour closer than the previous level
#pragma unroll
    for (int t = 0; t < U; ++t) {
      const int32_t term = (got[t] && (int32_t)y[t] < a.level) ? (int32_t)y[t] + 1 : kInf;
      acc = term < acc ? term : acc;
    }
    return acc;
  }
  __device__ static void atomic_combine(const LevelArgs& a, int32_t row, Acc v) {
    keep(atomicMin(&a.acc[row], v));
  }
  __device__ static Acc take(const LevelArgs& a, int32_t row) { return atomicExch(&a.acc[row], kInf); }
  // push: a frontier row u (distance k-1) offers k to its neighbours
  __device__ static Acc push_value(const LevelArgs& a, int32_t) { return a.level; }
  __device__ static bool claim(const LevelArgs& a, int32_t w, Acc v) {
    return atomicMin(&a.acc[w], v) == kInf;
  }
  __device__ static void publish_one(const LevelArgs&, int32_t) {}
  // the row entered the frontier at `level` (its distance)
  __device__ static bool entered(const LevelArgs& a, int32_t row, int32_t level) {
    return a.state[row] == level;
  }
  // f_k^row = min(f_{k-1}^row, acc): the zero diagonal of A' keeps the old value
  __device__ static bool post(const LevelArgs& a, int32_t row, Acc acc, bool live) {
    const bool fresh = live && (acc != kInf);  // live: own value still infinity
    if (fresh) a.state[row] = acc;
    return fresh;
  }
  __device__ static void publish(const LevelArgs&, int32_t, uint64_t, int) {}
};

// Real (+, *): x_k = A (x) f_{k-1}; f_k = [x_k (.) g_k != 0]; d^row = k where
// the row enters the frontier.  Sums of 0/1 values of at most the degree are
// exact in fp32.
struct Real {
  static constexpr bool kSingleRoot = true;
  static constexpr bool kBitmapFrontier = false;
  __device__ static void skip_chunk(const LevelArgs&, int32_t) {}
  using Acc = float;
  // a row's value is known only after all its terms (a sum of frontier terms)
  static constexpr bool kFirstHitFinal = false;
  // per-lane value the product terms of a row depend on (none here)
  __device__ static uint32_t context(const LevelArgs&, int32_t) { return 0u; }
  __device__ static bool settled(Acc) { return false; }
  __device__ static Acc identity() { return 0.0f; }
  __device__ static Rsrc rsrc(const LevelArgs& a) { return make_rsrc(a.vin, a.n_pad * 4u); }
  using Raw = uint32_t;
  __device__ static Raw raw(const LevelArgs& a, int32_t row) { return a.g[row]; }
  __device__ static bool is_live(const LevelArgs&, Raw w, int32_t) { return w != 0u; }
  __device__ static bool live(const LevelArgs& a, int32_t row) { return a.g[row] != 0; }
  __device__ static bool still_live(const LevelArgs&, int32_t, bool live, bool fresh) {
    return live && !fresh;
  }
  __device__ static const void* staged(const LevelArgs& a) { return a.vin; }
  template <int U, bool STAGED>
  __device__ static Acc block(const LevelArgs&, Rsrc r, Stage st, const int32_t (&c)[U],
                              Acc acc, uint32_t) {
    uint32_t y[U];
    bool got[U];
    gather_rows<U, STAGED, 1>(r, st, c, y, got);  // unread terms are 0.0f
#pragma unroll
    for (int t = 0; t < U; ++t) acc += __uint_as_float(y[t]);
    return acc;
  }
  __device__ static void atomic_combine(const LevelArgs& a, int32_t row, Acc v) {
    keep(__float_as_int(atomicAdd(reinterpret_cast<float*>(&a.acc[row]), v)));
  }
  __device__ static Acc take(const LevelArgs& a, int32_t row) {
    return atomicExch(reinterpret_cast<float*>(&a.acc[row]), 0.0f);
  }
  __device__ static Acc push_value(const LevelArgs&, int32_t) { return 1.0f; }
  __device__ static bool claim(const LevelArgs& a, int32_t w, Acc v) {
    return atomicAdd(reinterpret_cast<float*>(&a.acc[w]), v) == 0.0f;
  }
  __device__ static void publish_one(const LevelArgs&, int32_t) {}
  __device__ static bool entered(const LevelArgs& a, int32_t row, int32_t level) {
    return a.d[row] == level;
  }
  __device__ static bool post(const LevelArgs& a, int32_t row, Acc acc, bool live) {
    const bool fresh = live && acc != 0.0f;  // x_k (.) g_k != 0, live: g_k = 1
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
  static constexpr bool kSingleRoot = true;
  static constexpr bool kBitmapFrontier = false;
  __device__ static void skip_chunk(const LevelArgs&, int32_t) {}
  using Acc = uint32_t;
  // the first product term a row receives is its final value
  static constexpr bool kFirstHitFinal = true;
  // per-lane value the product terms of a row depend on (none here)
  __device__ static uint32_t context(const LevelArgs&, int32_t) { return 0u; }
  __device__ static bool settled(Acc acc) { return acc != 0u; }
  __device__ static Acc identity() { return 0u; }
  __device__ static Rsrc rsrc(const LevelArgs& a) { return make_rsrc(a.vin, a.n_pad); }
  using Raw = uint32_t;
  __device__ static Raw raw(const LevelArgs& a, int32_t row) { return a.g[row]; }
  __device__ static bool is_live(const LevelArgs&, Raw w, int32_t) { return w != 0u; }
  __device__ static bool live(const LevelArgs& a, int32_t row) { return a.g[row] != 0; }
  __device__ static bool still_live(const LevelArgs&, int32_t, bool live, bool fresh) {
    return live && !fresh;
  }
  __device__ static const void* staged(const LevelArgs& a) { return a.vin; }
  template <int U, bool STAGED>
  __device__ static Acc block(const LevelArgs&, Rsrc r, Stage st, const int32_t (&c)[U],
                              Acc acc, uint32_t) {
    uint32_t y[U];
    bool got[U];
    gather_rows<U, STAGED, 0>(r, st, c, y, got);  // unread terms are 0
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
  __device__ static Acc push_value(const LevelArgs&, int32_t) { return 1u; }
  __device__ static bool claim(const LevelArgs& a, int32_t w, Acc v) {
    return atomicOr(reinterpret_cast<uint32_t*>(&a.acc[w]), v) == 0u;
  }
  __device__ static void publish_one(const LevelArgs&, int32_t) {}
  __device__ static bool entered(const LevelArgs& a, int32_t row, int32_t level) {
    return a.d[row] == level;
  }
  __device__ static bool post(const LevelArgs& a, int32_t row, Acc acc, bool live) {
    const bool fresh = (acc != 0u) && live;  // live: g_k = 1
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
  static constexpr bool kSingleRoot = true;
  // the frontier is a bitmap with one word per chunk; in a scheduled run a
  // chunk the level skips gets a zero word, so every chunk's word tells
  // exactly which rows entered at this level (a push level after it scans
  // the words instead of every row's distance)
  static constexpr bool kBitmapFrontier = true;
  __device__ static void skip_chunk(const LevelArgs& a, int32_t chunk) {
    static_cast<uint64_t*>(a.vout)[chunk] = 0ull;
  }
  using Acc = int32_t;
  // the first product term a row receives is its final value
  static constexpr bool kFirstHitFinal = true;
  // per-lane value the product terms of a row depend on (none here)
  __device__ static uint32_t context(const LevelArgs&, int32_t) { return 0u; }
  __device__ static bool settled(Acc acc) { return acc != 0; }
  __device__ static Acc identity() { return 0; }
  __device__ static Rsrc rsrc(const LevelArgs& a) {
    return make_rsrc(a.vin, (uint32_t)(a.n_pad / kC) * 8u);
  }
  using Raw = int32_t;
  __device__ static Raw raw(const LevelArgs& a, int32_t row) { return a.state[row]; }
  __device__ static bool is_live(const LevelArgs&, Raw w, int32_t) { return w == 0; }
  __device__ static bool live(const LevelArgs& a, int32_t row) { return a.state[row] == 0; }
  __device__ static bool still_live(const LevelArgs&, int32_t, bool live, bool fresh) {
    return live && !fresh;
  }
  __device__ static const void* staged(const LevelArgs& a) { return a.vin; }
  template <int U, bool STAGED>
  __device__ static Acc block(const LevelArgs& a, Rsrc r, Stage st, const int32_t (&c)[U],
                              Acc acc, uint32_t) {
    const Rsrc rv = make_rsrc(a.v, a.n_pad * 4u);
    uint32_t w[U];  // the 32-bit half of the chunk word holding bit c (0 if unread)
    bool got[U];
    gather_rows<U, STAGED, 2>(r, st, c, w, got);
    bool hit[U];
    bool some = false;
#pragma unroll
    for (int t = 0; t < U; ++t) {
      hit[t] = c[t] >= 0 && ((w[t] >> (c[t] & 31)) & 1u);
      some = some || hit[t];
    }
    // Most blocks of the first and the late levels hit no frontier row: one
    // wave-uniform test then spares the address unit U loads of v.
    if (__any(some)) {
      int32_t x[U];
#pragma unroll
      for (int t = 0; t < U; ++t)
        x[t] = __builtin_amdgcn_raw_buffer_load_b32(rv, hit[t] ? (uint32_t)c[t] << 2 : kOob, 0, 0);
      __builtin_amdgcn_sched_barrier(0);  // all U loads in flight before the first use
#pragma unroll
      for (int t = 0; t < U; ++t) acc = x[t] > acc ? x[t] : acc;
    }
    return acc;
  }
  __device__ static void atomic_combine(const LevelArgs& a, int32_t row, Acc v) {
    keep(atomicMax(&a.acc[row], v));
  }
  __device__ static Acc take(const LevelArgs& a, int32_t row) { return atomicExch(&a.acc[row], 0); }
  __device__ static Acc push_value(const LevelArgs& a, int32_t u) { return a.v[u]; }
  __device__ static bool claim(const LevelArgs& a, int32_t w, Acc v) {
    return atomicMax(&a.acc[w], v) == 0;
  }
  // a row entering the frontier in a push level sets its bit in the word
  __device__ static void publish_one(const LevelArgs& a, int32_t row) {
    atomicOr(static_cast<unsigned long long*>(a.vout) + (row >> 6), 1ull << (row & 63));
  }
  __device__ static bool entered(const LevelArgs& a, int32_t row, int32_t level) {
    return a.d[row] == level;
  }
  __device__ static bool post(const LevelArgs& a, int32_t row, Acc acc, bool live) {
    const bool fresh = live && (acc != 0);  // live: p still 0
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
  static constexpr bool kSingleRoot = false;
  static constexpr bool kBitmapFrontier = false;
  __device__ static void skip_chunk(const LevelArgs&, int32_t) {}
  using Acc = unsigned long long;
  // a row's masks are known only after all its terms (an OR over neighbours)
  static constexpr bool kFirstHitFinal = false;
  // per-lane value the product terms of a row depend on (none here)
  __device__ static uint32_t context(const LevelArgs&, int32_t) { return 0u; }
  __device__ static bool settled(Acc) { return false; }
  __device__ static Acc identity() { return 0ull; }
  __device__ static Rsrc rsrc(const LevelArgs& a) { return make_rsrc(a.vin, a.n_pad * 8u); }
  using Raw = unsigned long long;
  __device__ static Raw raw(const LevelArgs& a, int32_t row) { return a.vis[row]; }
  __device__ static bool is_live(const LevelArgs& a, Raw w, int32_t chunk) {
    const Acc full = a.full[chunk];
    return (w & full) != full;
  }
  __device__ static bool live(const LevelArgs& a, int32_t row) {
    const Acc full = a.full[row / kC];
    return (a.vis[row] & full) != full;
  }
  // the visited mask post just wrote (this lane's own store)
  __device__ static bool still_live(const LevelArgs& a, int32_t row, bool, bool) {
    return live(a, row);
  }
  __device__ static const void* staged(const LevelArgs& a) { return a.vin; }
  template <int U, bool STAGED>
  __device__ static Acc block(const LevelArgs&, Rsrc r, Stage st, const int32_t (&c)[U],
                              Acc acc, uint32_t) {
    Acc y[U];
    gather_masks<U, STAGED>(r, st, c, y);  // unread masks are 0
#pragma unroll
    for (int t = 0; t < U; ++t) acc |= y[t];
    return acc;
  }
  __device__ static void atomic_combine(const LevelArgs& a, int32_t row, Acc v) {
    keep((int32_t)atomicOr(&a.acc64[row], v));
  }
  __device__ static Acc take(const LevelArgs& a, int32_t row) { return atomicExch(&a.acc64[row], 0ull); }
  __device__ static bool post(const LevelArgs& a, int32_t row, Acc acc, bool) {
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

// DP transformation (Section II-C) as one more pass of the level kernel:
// the parent of a reached row other than the root is its largest-ID
// neighbour one level closer.  The gathered vector is a code of two bits per
// row, distance mod 3 (3 = unreached), four rows per byte: a neighbour of a
// row at level k sits at level k-1, k or k+1, so the code tells the closer
// ones apart, and the gathered array is n/4 bytes.  A hit reads v of the
// neighbour (original ID + 1) and the max keeps the largest; rows list their
// neighbours by decreasing original ID, so a row stops at its first hit, as
// under sel-max.  The live rows are the reached ones other than the root (d
// holds row distances); each row's best v goes to `state`.
struct Dp {
  static constexpr bool kSingleRoot = true;
  static constexpr bool kBitmapFrontier = false;
  __device__ static void skip_chunk(const LevelArgs&, int32_t) {}
  using Acc = int32_t;
  // the first hit is the largest qualifying ID
  static constexpr bool kFirstHitFinal = true;
  // the code a qualifying neighbour of this lane's row carries (4: none)
  __device__ static uint32_t context(const LevelArgs& a, int32_t row) {
    const int32_t d = a.d[row];
    return d >= 1 ? (uint32_t)((d - 1) % 3) : 4u;
  }
  __device__ static bool settled(Acc acc) { return acc != 0; }
  __device__ static Acc identity() { return 0; }
  __device__ static Rsrc rsrc(const LevelArgs& a) { return make_rsrc(a.vin, a.n_pad / 4u); }
  using Raw = int32_t;
  __device__ static Raw raw(const LevelArgs& a, int32_t row) { return a.d[row]; }
  __device__ static bool is_live(const LevelArgs&, Raw w, int32_t) { return w >= 1; }
  __device__ static bool live(const LevelArgs& a, int32_t row) { return a.d[row] >= 1; }
  __device__ static bool still_live(const LevelArgs&, int32_t, bool live, bool fresh) {
    return live && !fresh;
  }
  __device__ static const void* staged(const LevelArgs& a) { return a.vin; }
  template <int U, bool STAGED>
  __device__ static Acc block(const LevelArgs& a, Rsrc r, Stage st, const int32_t (&c)[U],
                              Acc acc, uint32_t want) {
    const Rsrc rv = make_rsrc(a.v, a.n_pad * 4u);
    uint32_t y[U];  // the code byte holding row c (0 if unread)
    bool got[U];
    gather_rows<U, STAGED, 3>(r, st, c, y, got);
    bool hit[U];
    bool some = false;
#pragma unroll
    for (int t = 0; t < U; ++t) {
      hit[t] = c[t] >= 0 && ((y[t] >> ((c[t] & 3) * 2)) & 3u) == want;
      some = some || hit[t];
    }
    if (__any(some)) {
      int32_t x[U];
#pragma unroll
      for (int t = 0; t < U; ++t)
        x[t] = __builtin_amdgcn_raw_buffer_load_b32(rv, hit[t] ? (uint32_t)c[t] << 2 : kOob, 0, 0);
      __builtin_amdgcn_sched_barrier(0);  // all U loads in flight before the first use
#pragma unroll
      for (int t = 0; t < U; ++t) acc = x[t] > acc ? x[t] : acc;
    }
    return acc;
  }
  __device__ static void atomic_combine(const LevelArgs& a, int32_t row, Acc v) {
    keep(atomicMax(&a.acc[row], v));
  }
  __device__ static Acc take(const LevelArgs& a, int32_t row) { return atomicExch(&a.acc[row], 0); }
  __device__ static bool post(const LevelArgs& a, int32_t row, Acc acc, bool) {
    a.state[row] = acc;
    return false;
  }
  __device__ static void publish(const LevelArgs&, int32_t, uint64_t, int) {}
};

// ---------------------------------------------------------- level kernel ---


// Sweep `ncols` columns of one chunk for this lane's row, U columns at a time:
// U independent streaming loads of `col`, then the U gathers of the block.  A
// lane that is off (its row is final) issues no loads at all.  Where the
// first product term a row receives is already its final value (tropical,
// boolean, and sel-max, whose rows list their neighbours by decreasing
// original ID), the lane stops after the block that produced it (SlimWork
// mode 2; modes 0 and 1 compute every term); `cols` receives the columns the
// lane loaded.
//
// VAL (the Sell-C-sigma comparator of Section II-D): a second stream, val,
// runs beside col and decides whether a cell is an edge (1) or padding (0);
// the padding cells of that col hold a valid row, so only val marks them.
template <class S, int U, bool STAGED, bool VAL = false>
__device__ __forceinline__ typename S::Acc sweep(const LevelArgs& a, Rsrc r, Stage st,
                                                 const int32_t* __restrict__ p, int32_t ncols,
                                                 bool on, uint32_t ctx, int32_t& cols) {
  typename S::Acc acc = S::identity();
  cols = 0;
  if (!on) return acc;
  const int32_t* __restrict__ pv = VAL ? a.val + (p - a.col) : nullptr;
  const bool stop = a.slimwork >= 2;  // modes 0 and 1 compute every term
  int32_t j = 0;
  bool go = true;
  if (ncols >= 2 * U) {
    // Software pipeline: the next block's col (and val) loads are in flight
    // while this block's gathers (which depend on its col values) are
    // served, so a block costs one memory latency instead of two.  (A second
    // block of depth measured no faster and costs U more registers.)
    int32_t c[U], w[U], nc[U], nw[U];
#pragma unroll
    for (int t = 0; t < U; ++t) {
      c[t] = __builtin_nontemporal_load(p + (int64_t)t * kC);
      if (VAL) w[t] = __builtin_nontemporal_load(pv + (int64_t)t * kC);
    }
    p += (int64_t)U * kC;
    if (VAL) pv += (int64_t)U * kC;
    for (j = U; j + U <= ncols; j += U) {
#pragma unroll
      for (int t = 0; t < U; ++t) {
        nc[t] = __builtin_nontemporal_load(p + (int64_t)t * kC);
        if (VAL) nw[t] = __builtin_nontemporal_load(pv + (int64_t)t * kC);
      }
      if (VAL) {
#pragma unroll
        for (int t = 0; t < U; ++t) c[t] = w[t] ? c[t] : -1;
      }
      acc = S::template block<U, STAGED>(a, r, st, c, acc, ctx);
      if (S::kFirstHitFinal && stop && S::settled(acc)) {
        go = false;
        break;
      }
#pragma unroll
      for (int t = 0; t < U; ++t) {
        c[t] = nc[t];
        if (VAL) w[t] = nw[t];
      }
      p += (int64_t)U * kC;
      if (VAL) pv += (int64_t)U * kC;
    }
    if (go) {
      if (VAL) {
#pragma unroll
        for (int t = 0; t < U; ++t) c[t] = w[t] ? c[t] : -1;
      }
      acc = S::template block<U, STAGED>(a, r, st, c, acc, ctx);
      go = !(S::kFirstHitFinal && stop && S::settled(acc));
      cols = j;
    } else {
      cols = j + U;  // the prefetched block was loaded too
    }
  }
  if (go) {
    for (; j + U <= ncols; j += U) {
      int32_t c[U];
#pragma unroll
      for (int t = 0; t < U; ++t) c[t] = __builtin_nontemporal_load(p + (int64_t)t * kC);
      if (VAL) {
        int32_t w[U];
#pragma unroll
        for (int t = 0; t < U; ++t) w[t] = __builtin_nontemporal_load(pv + (int64_t)t * kC);
#pragma unroll
        for (int t = 0; t < U; ++t) c[t] = w[t] ? c[t] : -1;
        pv += (int64_t)U * kC;
      }
      acc = S::template block<U, STAGED>(a, r, st, c, acc, ctx);
      p += (int64_t)U * kC;
      cols = j + U;
      if (S::kFirstHitFinal && stop && S::settled(acc)) {
        go = false;
        break;
      }
    }
  }
  if (go && j < ncols) {
    // the ragged tail of fewer than U columns as one block: the columns past
    // the end repeat the last address (a cache hit) and are masked to padding,
    // so the tail costs one load round trip rather than one per column
    const int32_t rem = ncols - j;
    int32_t c[U];
#pragma unroll
    for (int t = 0; t < U; ++t) {
      const int64_t o = (int64_t)(t < rem ? t : rem - 1) * kC;
      c[t] = __builtin_nontemporal_load(p + o);
      if (VAL) c[t] = __builtin_nontemporal_load(pv + o) ? c[t] : -1;
    }
#pragma unroll
    for (int t = 0; t < U; ++t) c[t] = t < rem ? c[t] : -1;
    acc = S::template block<U, STAGED>(a, r, st, c, acc, ctx);
    cols = ncols;
  }
  return acc;
}


__device__ __forceinline__ uint64_t lanes_below(int lane) { return (1ull << lane) - 1ull; }

// Post-process the rows of one chunk; returns how many entered the frontier
// and adds their degrees to `fdeg`.
template <class S>
__device__ __forceinline__ uint32_t finish_rows(const LevelArgs& a, int32_t chunk, int32_t row,
                                                typename S::Acc acc, bool live, int lane,
                                                bool record, uint64_t& fdeg) {
  const bool fresh = S::post(a, row, acc, live);
  const uint64_t mask = __ballot(fresh);
  S::publish(a, chunk, mask, lane);
  if (record && lane == 0 && mask)  // the chunk has a frontier row for the next level
    atomicOr(a.summ + (int64_t)(a.level % 3) * a.summ_words + (chunk >> 5), 1u << (chunk & 31));
  // a chunk whose rows are all final stays final: later levels skip it
  // without reading its rows
  if (a.done && !__any(S::still_live(a, row, live, fresh)) && lane == 0) a.done[chunk] = 1;
  if (fresh) fdeg += (uint64_t)a.deg[row];
  return (uint32_t)__popcll(mask);
}

__device__ __forceinline__ uint64_t wave_sum64(uint64_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Flush the tallies of one workgroup into the statistics and schedule
// counters: every wavefront adds its tallies in LDS, then one thread adds the
// workgroup's totals to its slot (and sets the level's "found" tag), so a
// level issues a few global atomics per workgroup instead of per wavefront.
// Every thread of the workgroup must call it.  Without counters it only sets
// the tag, with no workgroup barrier.
__device__ __forceinline__ void flush_counters(const LevelArgs& a, int lane, uint32_t found,
                                               uint32_t n_chunks, uint64_t n_cells,
                                               int32_t max_cl, uint64_t fdeg_lane) {
  __shared__ unsigned long long tally[kCountFields];  // found, chunks, cells, max cl, fdeg
  if (!a.count_stats && !a.ring_ctr) {
    // nothing is counted (the condition is the same in every thread): only
    // the level's "found" tag, from each wavefront that found rows
    if (lane == 0 && found) a.any[a.level % kRing] = level_tag(a.run_id, a.level);
    return;
  }
  const uint64_t fdeg = wave_sum64(fdeg_lane);
  if (threadIdx.x < kCountFields) tally[threadIdx.x] = 0ull;
  __syncthreads();
  if (lane == 0) {
    if (found) atomicAdd(&tally[0], (unsigned long long)found);
    if (n_chunks) {
      atomicAdd(&tally[1], (unsigned long long)n_chunks);
      atomicMax(&tally[3], (unsigned long long)max_cl);
    }
    if (n_cells) atomicAdd(&tally[2], (unsigned long long)n_cells);
    if (fdeg) atomicAdd(&tally[4], (unsigned long long)fdeg);
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const unsigned long long t[kCountFields] = {tally[0], tally[1], tally[2], tally[3], tally[4]};
  if (t[0]) a.any[a.level % kRing] = level_tag(a.run_id, a.level);
  if (!(t[0] | t[1] | t[2] | t[4])) return;
  unsigned long long* dst[2] = {nullptr, nullptr};
  if (a.count_stats)
    dst[0] = a.counters + ((int64_t)a.level * kCountSlots + blockIdx.x % kCountSlots) * kCountFields;
  if (a.ring_ctr)
    dst[1] = a.ring_ctr +
             ((int64_t)(a.level % kRing) * kRingSlots + blockIdx.x % kRingSlots) * kCountFields;
  for (unsigned long long* ctr : dst) {
    if (!ctr) continue;
    if (t[0]) atomicAdd(&ctr[0], t[0]);
    if (t[1]) {
      atomicAdd(&ctr[1], t[1]);
      atomicMax(&ctr[3], t[3]);
    }
    if (t[2]) atomicAdd(&ctr[2], t[2]);
    if (t[4]) atomicAdd(&ctr[4], t[4]);
  }
}

// One BFS level.  slimwork: 0 = every row of every chunk is computed;
// 1 = chunks whose rows are all final are skipped (Section III-C);
// 2 = additionally a lane whose row is final issues no loads, the sweep
// stops at the longest row that is still live, and a row whose value became
// final stops its scan.
// The work of one level for one workgroup: stage the LDS prefix, sweep the
// work units assigned to this workgroup's wavefronts, post-process, count.
template <class S, int U, bool STAGED, bool VAL = false>
__device__ __forceinline__ void level_body(const LevelArgs& a, const Unit* units,
                                           const int32_t* pieces, int64_t n_units,
                                           const int32_t* bundle, int32_t* arrive2,
                                           int32_t piece_cols, const int32_t* wave_off,
                                           uint8_t* lds_stage) {
  const int lane = threadIdx.x & (kC - 1);
  const int wave = threadIdx.x / kC;
  const int waves = blockDim.x / kC;
  const Rsrc rs = S::rsrc(a);
  Stage st{lds_stage, 0u};
  // This wavefront's work units: with a per-wavefront assignment (wave_off)
  // the consecutive units [wave_off[w], wave_off[w + 1]), else units w,
  // w + W, w + 2 W, ... of the grid's W wavefronts.  Its first 64 are read
  // here (see the unit loop below).
  const int64_t gw = (int64_t)blockIdx.x * waves + wave;
  int64_t r0 = gw, step = (int64_t)gridDim.x * waves, count = 0;
  if (wave_off) {
    r0 = wave_off[gw];
    step = 1;
    count = wave_off[gw + 1] - r0;
  } else if (gw < n_units) {
    count = (n_units - gw + step - 1) / step;
  }
  // (a wavefront with a single unit learns as much from the unit's row
  // states, which it reads anyway, one dependent load sooner)
  const bool skip_done = a.done != nullptr && a.slimwork != 0 && count > 1;
  // lane k's unit: its first chunk, and whether it is a single chunk (or a
  // piece of one), whose flag may retire it
  int32_t mine_c0 = 0;
  bool mine_one = false;
  bool want = lane < count;
  if (want) {
    const Unit u = units[r0 + (int64_t)lane * step];
    mine_c0 = u.c0;
    mine_one = u.c1 == u.c0 + 1;
  }
  if (a.summ) {
    // clear the summary the next level writes (read by the level before this one)
    uint32_t* next = a.summ + (int64_t)((a.level + 1) % 3) * a.summ_words;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.summ_words;
         i += (int64_t)gridDim.x * blockDim.x)
      next[i] = 0u;
  }
  // the previous level left a summary only if it used one itself
  const bool have = a.summ && a.summ[3 * (int64_t)a.summ_words + (a.level - 1) % 3] != 0u;
  if (STAGED) {
    // The previous level's frontier summary (if it left one) goes to LDS
    // behind the prefix's place, and its set bits are counted, in all and
    // among the chunks the prefix covers.  The level filters its gathers by
    // it when few chunks hold frontier rows (the same decision in every
    // workgroup: all count the same summary).  The vector's first
    // a.lds_bytes (a multiple of 16) are then copied into LDS, unless the
    // level filters and no chunk the prefix covers holds a frontier row: then
    // every term the prefix would serve is the identity and is not read.
    __shared__ uint32_t flagged, flagged_prefix;
    st.summ = a.lds_bytes;
    bool stage = true;
    if (have) {
      if (threadIdx.x == 0) {
        flagged = 0u;
        flagged_prefix = 0u;
      }
      __syncthreads();
      const uint32_t* prev = a.summ + (int64_t)((a.level - 1) % 3) * a.summ_words;
      uint32_t* sd = reinterpret_cast<uint32_t*>(lds_stage + a.lds_bytes);
      uint32_t cnt = 0u, cnt_p = 0u;
      for (int32_t i = threadIdx.x; i < a.summ_words; i += blockDim.x) {
        const uint32_t w = prev[i];
        sd[i] = w;
        cnt += (uint32_t)__popc(w);
        if (i < a.prefix_words) cnt_p += (uint32_t)__popc(w);
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        cnt += __shfl_xor(cnt, off);
        cnt_p += __shfl_xor(cnt_p, off);
      }
      if (lane == 0 && cnt) atomicAdd(&flagged, cnt);
      if (lane == 0 && cnt_p) atomicAdd(&flagged_prefix, cnt_p);
      __syncthreads();
      st.filter = (int64_t)flagged <= (int64_t)a.filter_limit;
      stage = !st.filter || flagged_prefix != 0u;
    }
    if (stage) {
      const uint4* src = static_cast<const uint4*>(S::staged(a));
      uint4* dst = reinterpret_cast<uint4*>(lds_stage);
      for (uint32_t i = threadIdx.x; i < a.lds_bytes / 16u; i += blockDim.x) dst[i] = src[i];
      __syncthreads();
      st.bytes = a.lds_bytes;
    }
  }
  // A level records its own frontier summary only when it used the filter:
  // after a level with a wide frontier the next one is usually wide too, and
  // recording it would cost one atomic per chunk for nothing.
  const bool record = STAGED && st.filter;
  if (a.summ && blockIdx.x == 0 && threadIdx.x == 0)
    a.summ[3 * (int64_t)a.summ_words + a.level % 3] = record ? 1u : 0u;
  // per-wavefront tallies, flushed once at the end
  uint32_t found = 0, n_chunks = 0;
  uint64_t n_cols = 0, fdeg = 0;
  int32_t max_cl = 0;

  // This wavefront's units 64 at a time: lane k reads the descriptor of the
  // k-th and, for a unit of one chunk, the chunk's "all rows final" flag, so
  // one ballot names the units to sweep (a level whose chunks are mostly
  // final pays two memory round trips per 64 units instead of one per unit).
  // While one unit is swept, the next one's chunk extent, degrees and row
  // states are in flight.  (The first batch's descriptors were requested
  // before the LDS staging, so their latency overlaps it.)
  for (int64_t b = 0; b < count; b += kC) {
    if (b != 0) {
      want = b + lane < count;
      if (want) {
        const Unit u = units[r0 + (b + lane) * step];
        mine_c0 = u.c0;
        mine_one = u.c1 == u.c0 + 1;
      }
    }
    if (want && skip_done && mine_one && a.done[mine_c0] != 0) {
      want = false;
      if (a.variant) S::skip_chunk(a, mine_c0);  // a push level may follow
    }
    uint64_t todo = __ballot(want);
    // the next unit to sweep and its first chunk's metadata (loads in flight)
    Unit nw{0, 0, 0, 0};
    int32_t n_len = 0, n_dg = 0;
    int64_t n_start = 0;
    typename S::Raw n_raw{};
    auto next = [&]() -> bool {
      if (!todo) return false;
      const int k = __ffsll((long long)todo) - 1;
      todo &= todo - 1;
      // the same address in every lane: the descriptor is wave-uniform
      const Unit u = units[r0 + (b + k) * step];
      nw.c0 = __builtin_amdgcn_readfirstlane(u.c0);
      nw.c1 = __builtin_amdgcn_readfirstlane(u.c1);
      nw.j0 = __builtin_amdgcn_readfirstlane(u.j0);
      nw.j1 = __builtin_amdgcn_readfirstlane(u.j1);
      n_len = a.cl[nw.c0];
      n_start = a.cs[nw.c0];
      n_dg = a.deg[nw.c0 * kC + lane];
      n_raw = S::raw(a, nw.c0 * kC + lane);
      return true;
    };
    bool more = next();
    while (more) {
    const Unit w = nw;
    const int32_t f_len = n_len, f_dg = n_dg;
    const int64_t f_start = n_start;
    const typename S::Raw f_raw = n_raw;
    more = next();
    const bool piece = (w.c1 == w.c0 + 1);
    for (int32_t c = w.c0; c < w.c1; ++c) {
      const int32_t row = c * kC + lane;
      // the first chunk's extent, degrees and states were read ahead; the
      // other chunks of a packed run read theirs together
      int32_t len = f_len, dg = f_dg;
      int64_t start = f_start;
      typename S::Raw rw = f_raw;
      if (c != w.c0) {
        len = a.cl[c];
        start = a.cs[c];
        dg = a.deg[row];
        rw = S::raw(a, row);
      }
      const bool live = S::is_live(a, rw, c);
      if (a.slimwork && !__any(live)) {  // whole chunk final
        if (a.variant && lane == 0) S::skip_chunk(a, c);
        continue;
      }
      int32_t j0 = 0, j1 = len;
      if (piece) { j0 = w.j0; j1 = w.j1; }
      if (j0 == 0) {
        ++n_chunks;
        max_cl = len > max_cl ? len : max_cl;
      }
      const bool on = (a.slimwork >= 2) ? live : true;
      int32_t hi = j1;
      if (a.slimwork >= 2) {
        const int32_t lim = wave_max(on ? dg : 0);
        hi = lim < j1 ? lim : j1;
      }
      const int32_t ncols = hi > j0 ? hi - j0 : 0;
      const int32_t* p = a.col + start + (int64_t)j0 * kC + lane;
      int32_t lane_cols;
      typename S::Acc acc =
          sweep<S, U, STAGED, VAL>(a, rs, st, p, ncols, on, S::context(a, row), lane_cols);
      n_cols += (uint64_t)wave_max(lane_cols);  // columns the wavefront streamed
      const int32_t npieces = piece ? pieces[c] : 1;
      if (npieces == 1) {
        found += finish_rows<S>(a, c, row, acc, live, lane, record, fdeg);
      } else {
        // SlimChunk: combine this piece, the last one to arrive post-processes.
        // Pieces exchange data only through device-scope atomics: each piece's
        // combine has completed before its arrival is counted, and a bundle
        // is counted in the chunk only after all its pieces were, so the last
        // arrival's exchange sees every piece.
        if (acc != S::identity()) S::atomic_combine(a, row, acc);  // identity: no change
        wait_memory();
        int last = 0;
        if (lane == 0) {
          const int32_t q = j0 / piece_cols;                   // piece index in the chunk
          const int32_t nb = (npieces + kBundle - 1) / kBundle;  // bundles of the chunk
          const int32_t bq = q / kBundle;
          const int32_t bsize = min(kBundle, npieces - bq * kBundle);
          int32_t* bc = arrive2 + bundle[c] + bq;
          if (atomicAdd(bc, 1) == bsize - 1) {
            atomicExch(bc, 0);  // every piece of the bundle has arrived: ready for the next level
            last = (atomicAdd(&a.arrive[c], 1) == nb - 1);
          }
        }
        last = __shfl(last, 0);
        if (last) {
          acc = S::take(a, row);
          if (lane == 0) a.arrive[c] = 0;
          found += finish_rows<S>(a, c, row, acc, live, lane, record, fdeg);
        }
      }
    }
    }
  }
  flush_counters(a, lane, found, n_chunks, n_cols * kC, max_cl, fdeg);
}


template <class S, int U, bool STAGED, bool VAL>
__device__ __forceinline__ void level_entry(const LevelArgs& a, uint8_t* lds_stage) {
  if (a.level > 1) {
    // Stop if the previous level discovered nothing, and tell the host what
    // the previous level found (one thread of the first workgroup).
    const uint64_t want = level_tag(a.run_id, a.level - 1);
    const bool prev_found = (a.any[(a.level - 1) % kRing] == want);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      __hip_atomic_store(&a.report[(a.level - 1) % kRing], (want << 1) | (prev_found ? 1u : 0u),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    if (!prev_found) return;
  }
  level_body<S, U, STAGED, VAL>(a, a.units, a.pieces, a.n_units, a.bundle, a.arrive2,
                                a.piece_cols, a.wave_off, lds_stage);
}

template <class S, int U, bool STAGED, bool VAL = false>
__global__ void level_kernel(LevelArgs a) {
  extern __shared__ uint8_t lds_stage[];
  level_entry<S, U, STAGED, VAL>(a, lds_stage);
}

// The four-column form held to 64 registers per lane, so that eight
// wavefronts share each SIMD: two 16-wavefront workgroups per compute unit,
// twice the wavefronts of the eight-column form, for levels that are bound
// by the latency of their per-chunk loads rather than by the column stream.
template <class S, bool STAGED>
__global__ void __launch_bounds__(1024, 8) level_kernel_w8(LevelArgs a) {
  extern __shared__ uint8_t lds_stage[];
  level_entry<S, 4, STAGED, false>(a, lds_stage);
}

// ------------------------------------------------------- persistent form ---
//
// All levels of one run in a single cooperative launch: the grid is no larger
// than what the device keeps resident at once, levels are separated by a
// grid barrier, and every workgroup reads the same "found" tag after it, so
// all leave the loop together.  The barrier's spin has a wall-clock deadline:
// a workgroup that passes it records an error and returns, so every wave
// always exits.

__device__ __forceinline__ bool grid_barrier(unsigned* bar, unsigned nblocks, uint64_t limit,
                                             int* error) {
  __shared__ int ok;
  // Every wavefront's stores and atomics of the level must have reached L2
  // before thread 0 releases them: the workgroup barrier alone does not wait
  // for them.
  wait_memory();
  __syncthreads();
  if (threadIdx.x == 0) {
    ok = 1;
    // One release before arriving and one acquire after the wait: the
    // arrival counter only grows (64-bit, cleared before the launch), so
    // barrier e is passed once it reaches (e + 1) * nblocks, and polling it
    // needs no ordering of its own.  (Full fences on both sides in every
    // workgroup cost about three times as much per barrier.)
    unsigned long long* count = reinterpret_cast<unsigned long long*>(bar);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned long long arrived = atomicAdd(count, 1ull);
    const unsigned long long target = (arrived / nblocks + 1ull) * nblocks;
    const uint64_t t0 = wall_clock64();
    while (__hip_atomic_load(count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(2);
      if (wall_clock64() - t0 > limit) {
        atomicExch(error, 1);
        ok = 0;
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  return ok != 0;
}

template <class S, int U, bool STAGED>
__global__ void persistent_kernel(LevelArgs a, void* buf_a, void* buf_b, int32_t cap,
                                  unsigned* bar, int32_t* status, uint64_t limit) {
  extern __shared__ uint8_t lds_stage[];
  for (int32_t k = 1; k <= cap; ++k) {
    a.level = k;
    a.vin = (k & 1) ? buf_a : buf_b;
    a.vout = (k & 1) ? buf_b : buf_a;
    a.count_stats = a.count_stats && (k <= status[2]);
    level_body<S, U, STAGED>(a, a.units, a.pieces, a.n_units, a.bundle, a.arrive2, a.piece_cols,
                             nullptr, lds_stage);
    if (!grid_barrier(bar, gridDim.x, limit, &status[1])) return;
    if (a.any[k % kRing] != level_tag(a.run_id, k)) {
      if (blockIdx.x == 0 && threadIdx.x == 0) status[0] = k;  // levels run
      return;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) status[0] = -1;  // cap reached
}

// ------------------------------------------------------------ push levels ---
//
// The same product computed from the frontier side (the sparse-vector form
// of Section II-C): every row u of the previous level's frontier queue offers
// its term to each neighbour w that is still live, through the semiring's
// atomic; the first offer to w claims it for this level's queue.  A second
// kernel then post-processes the claimed rows.  Since A is symmetric, row u's
// cells in the SlimSell layout are its neighbours.

constexpr int kPushSegment = 1024;  // longer rows are cut into segments of this many cells

// Rows claimed by a workgroup are staged in LDS and appended to the level's
// queue with one atomic per workgroup at the end of the phase (an atomic
// per wavefront and column on the one queue counter, from every XCD, is
// serialised by the memory system, about 57 ns each).  A batch that does
// not fit goes to the queue directly.  `cut` is where the first such batch
// began: the staged rows are exactly [0, min(n, cut)).
constexpr int kPushStage = 2048;
struct PushStage {
  int32_t n, cut, base;
  int32_t rows[kPushStage];
};

// A push phase inside a kernel that also runs pull levels stages its rows
// in the LDS of the prefix (not in use on a push level), if it is large
// enough: a static buffer would cost the pull levels occupancy.
template <bool STAGED>
__device__ __forceinline__ PushStage* push_stage(const LevelArgs& a, uint8_t* lds_stage) {
  return (STAGED && a.lds_bytes >= sizeof(PushStage)) ? reinterpret_cast<PushStage*>(lds_stage)
                                                     : nullptr;
}

// Every thread of the workgroup calls these (ps == nullptr: no staging).
__device__ __forceinline__ void stage_begin(PushStage* ps) {
  if (!ps) return;
  if (threadIdx.x == 0) {
    ps->n = 0;
    ps->cut = kPushStage;
  }
  __syncthreads();
}

__device__ __forceinline__ void stage_flush(const LevelArgs& a, PushStage* ps) {
  if (!ps) return;
  __syncthreads();
  const int32_t cnt = ps->n < ps->cut ? ps->n : ps->cut;
  if (threadIdx.x == 0 && cnt > 0) ps->base = atomicAdd(&a.qn[a.level % kRing], cnt);
  __syncthreads();
  for (int32_t i = threadIdx.x; i < cnt; i += blockDim.x) a.q_out[ps->base + i] = ps->rows[i];
}

template <class S>
__device__ __forceinline__ void push_one(const LevelArgs& a, int32_t w, typename S::Acc val,
                                         int lane, PushStage* ps) {
  bool claimed = false;
  if (w >= 0 && S::live(a, w)) claimed = S::claim(a, w, val);
  const uint64_t m = __ballot(claimed);
  if (!m) return;
  const int leader = __ffsll((long long)m) - 1;
  const int32_t cnt = (int32_t)__popcll(m);
  int32_t slot = 0, base = -1;
  if (lane == leader) {
    if (ps) slot = atomicAdd(&ps->n, cnt);
    if (!ps || slot + cnt > kPushStage) {
      if (ps && slot < kPushStage) ps->cut = slot;  // the one batch that crosses the end
      base = atomicAdd(&a.qn[a.level % kRing], cnt);
    }
  }
  slot = __shfl(slot, leader);
  base = __shfl(base, leader);
  const int32_t r = __popcll(m & lanes_below(lane));
  if (claimed) {
    if (base < 0) ps->rows[slot + r] = w;
    else a.q_out[base + r] = w;
  }
}

// Short frontier rows: one lane each.  Long rows are cut into segments of
// kPushSegment cells that go to the segment list for push_segments_kernel,
// so a few high-degree rows do not serialise on a few wavefronts.
// The push phases are written for any grid: wavefront `gw` of `nw`.
__device__ __forceinline__ int32_t load_count(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The frontier rows of level k-1 come from the queue the push post of level
// k-1 (or the scheduled run's init) filled, or, after a pull level, which
// keeps no queue, from a scan of the rows that entered at level k-1.
template <class S>
__device__ __forceinline__ void push_scatter_body(const LevelArgs& a, int64_t gw, int64_t nw,
                                                  PushStage* ps) {
  const int lane = threadIdx.x & (kC - 1);
  stage_begin(ps);
  const bool scan = a.level > 1 && a.variant[(a.level - 1) % kRing] < kPullVariants &&
                    a.variant[(a.level - 1) % kRing] >= 0;
  const int64_t nq = scan ? (int64_t)a.n_pad : (int64_t)load_count(&a.qn[(a.level - 1) % kRing]);
  uint64_t cells = 0;
  for (int64_t base = gw * kC; base < nq; base += nw * kC) {
    const int64_t i = base + lane;
    int32_t u = -1;
    if (i < nq) {
      if (!scan) {
        u = a.q_in[i];
      } else if (S::kBitmapFrontier) {
        // the previous level's frontier word of this chunk (one load for the
        // wavefront's 64 rows instead of one distance per row)
        const uint64_t wd = static_cast<const uint64_t*>(a.vin)[base >> 6];
        if ((wd >> lane) & 1ull) u = (int32_t)i;
      } else if (S::entered(a, (int32_t)i, a.level - 1)) {
        u = (int32_t)i;
      }
    }
    const int32_t du = u >= 0 ? a.deg[u] : 0;
    const bool big = du > kPushLaneMax;
    if (u >= 0 && !big) {
      const int32_t* p = a.col + a.cs[u >> 6] + (u & 63);
      const typename S::Acc val = S::push_value(a, u);
      for (int32_t j = 0; j < du; ++j) push_one<S>(a, p[(int64_t)j * kC], val, lane, ps);
      cells += (uint64_t)du;
    }
    // long rows: reserve their segments with one atomic per wavefront
    const int32_t nseg = big ? (du + kPushSegment - 1) / kPushSegment : 0;
    int32_t excl = nseg;  // exclusive prefix over the wavefront
#pragma unroll
    for (int off = 1; off < kC; off <<= 1) {
      const int32_t y = __shfl_up(excl, off);
      if (lane >= off) excl += y;
    }
    const int32_t total = __shfl(excl, kC - 1);
    excl -= nseg;
    if (total) {
      int32_t start = 0;
      if (lane == 0) start = atomicAdd(a.seg_n, total);
      start = __shfl(start, 0);
      for (int32_t q = 0; q < nseg; ++q)
        a.segs[start + excl + q] = make_int2(u, q * kPushSegment);
    }
  }
  stage_flush(a, ps);
  flush_counters(a, lane, 0, 0, wave_sum64(cells), 0, 0);
}

// Long frontier rows, one segment of kPushSegment cells per wavefront pass.
template <class S>
__device__ __forceinline__ void push_segments_body(const LevelArgs& a, int64_t gw, int64_t nw,
                                                   PushStage* ps) {
  const int lane = threadIdx.x & (kC - 1);
  stage_begin(ps);
  const int32_t ns = load_count(a.seg_n);
  uint64_t cells = 0;
  for (int64_t s = gw; s < ns; s += nw) {
    const int2 sg = a.segs[s];
    const int32_t u = sg.x, j0 = sg.y;
    const int32_t du = a.deg[u];
    const int32_t j1 = j0 + kPushSegment < du ? j0 + kPushSegment : du;
    const int32_t* p = a.col + a.cs[u >> 6] + (u & 63);
    const typename S::Acc val = S::push_value(a, u);
    for (int32_t j = j0 + lane; j - lane < j1; j += kC)
      push_one<S>(a, j < j1 ? p[(int64_t)j * kC] : -1, val, lane, ps);
    cells += (uint64_t)(j1 - j0);
  }
  stage_flush(a, ps);
  flush_counters(a, lane, 0, 0, lane == 0 ? cells : 0, 0, 0);
}

// Post-process the rows claimed this level: lane `lane` of wavefront `gw`
// of `nw` takes queue entries gw*64+lane, (gw+nw)*64+lane, ...
template <class S>
__device__ __forceinline__ void push_post_body(const LevelArgs& a, int64_t gw, int64_t nw) {
  const int lane = threadIdx.x & (kC - 1);
  const int32_t nt = load_count(&a.qn[a.level % kRing]);
  uint32_t found = 0;
  uint64_t fdeg = 0;
  for (int64_t i = gw * kC + lane; i - lane < nt; i += nw * kC) {
    const bool mine = i < nt;
    const int32_t w = mine ? a.q_out[i] : 0;
    bool fresh = false;
    if (mine) {
      fresh = S::post(a, w, S::take(a, w), S::live(a, w));
      if (fresh) {
        S::publish_one(a, w);
        fdeg += (uint64_t)a.deg[w];
      }
    }
    found += (uint32_t)__popcll(__ballot(fresh));
  }
  flush_counters(a, lane, found, 0, 0, 0, fdeg);
}

__device__ __forceinline__ int64_t grid_wave() {
  return ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kC;
}
__device__ __forceinline__ int64_t grid_waves() { return ((int64_t)gridDim.x * blockDim.x) / kC; }

// Launched after the level kernel of every scheduled level (which runs the
// push scatter itself); they return at once unless the variant is push.
template <class S>
__global__ void push_segments_kernel(LevelArgs a) {
  if (a.variant[a.level % kRing] != kPush) return;
  __shared__ PushStage ps;
  push_segments_body<S>(a, grid_wave(), grid_waves(), &ps);
}

template <class S>
__global__ void push_post_kernel(LevelArgs a) {
  if (a.variant[a.level % kRing] != kPush) return;
  push_post_body<S>(a, grid_wave(), grid_waves());
}

// -------------------------------------------------------------- schedule ---
//
// At the start of every scheduled level k each workgroup stops the run if
// level k-1 found nothing, else updates the running totals and picks level
// k's variant from six features of the frontier: by the MLP (6 -> 32 -> 32 ->
// 4, ReLU; smallest predicted log-time wins) when a model is loaded and gives
// finite scores, else by the fixed heuristic (pull once the frontier's edges
// exceed 1/14 of the unvisited edges, otherwise push).  The counters, queue
// length and segment count of a level are cleared one level ahead.
struct SchedArgs {
  int32_t level;
  uint32_t run_id;
  uint64_t* any;
  uint64_t* report;
  int32_t* variant;
  int32_t* qn;
  int32_t* seg_n;         // [2] push segment counts by level parity
  unsigned long long* ring_ctr;
  double* sums;           // [0] discovered so far, [1] their degrees, [2] previous frontier size
  const float* model;     // nullptr = no model
  const float* anchors;   // the model's training domain [n_anchors][6], or nullptr
  const float* box;       // [12] the anchors' box widened by tau: lower, then upper bounds
  const float* cells;     // [6] bins per unit of each feature, then kCellWords bit words
  uint64_t* decided;      // [kRing] published decisions (tag << 3 | variant + 2), or nullptr
  uint64_t* in_box;       // host-visible word: set when the model decides a level, or nullptr
  int32_t eager;          // stage the model before the domain test (else only inside the domain)
  int32_t n_anchors;
  float tau2;             // squared distance to the nearest anchor the model may answer at
  float* log;             // [log_cap * 12]
  int32_t log_cap;
  int32_t mode;           // 1 learned, 2 heuristic, 3.. forced variant (mode - 3)
  int32_t heuristic_pull; // pull variant used by the heuristic
  double n, two_m;        // vertices, directed edges (2m)
  float log2n, l2n, l2m;  // log2 n, log2 max(n, 2), log2(1 + max(2m, 1))
};

// Workgroup scratch of the schedule.  `sums` are the running totals: [0]
// vertices discovered so far, [1] their degrees, [2] the previous frontier's
// size.
struct SchedShared {
  float w[kModelSize];         // the model's parameters, staged once per level
  float box[2 * kFeatures];    // the training domain's box (lower, upper)
  float cscale[kFeatures];     // the box's cell map: bins per unit of each feature
  uint32_t cells[kCellWords];  // and one bit per cell (set: near some anchor)
  float x[kFeatures], out[kVariants];
  double sums[3];
  float mf, mu;
  int32_t v, stop;
  uint64_t pub;  // the level's published decision word, if any
};

// Lane j's value of v, bit for bit (the builtin's value is an integer).
__device__ __forceinline__ float lane_value(float v, int j) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), j));
}

// Level k's variant, from level k-1's counters, computed by a whole
// workgroup (at least 32 threads; every thread must call it).  Advances
// `sh.sums` past level k-1.  A `writer` workgroup records the decision in
// the variant ring and the schedule log.  The arithmetic is the same in every
// workgroup, so all workgroups that call it with the same counters agree.
__device__ int32_t schedule_pick(const SchedArgs& s, int32_t k, SchedShared& sh, bool writer) {
  const int t = threadIdx.x;
  const uint64_t tag = level_tag(s.run_id, k) & ((1ull << 61) - 1);
  // A workgroup that starts after the writer has decided this level (a
  // later round of workgroups) takes the published decision.  Every
  // workgroup reaches the same decision (and any variant leaves the same
  // BFS state).
  if (t == 0)
    sh.pub = (s.decided && !writer)
                 ? __hip_atomic_load(&s.decided[k % kRing], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                 : 0ull;
  // The model (and its domain box) is staged into LDS by the whole
  // workgroup, and each thread holds one anchor of the training domain, in
  // the same round of loads as the counters below, so scoring a level costs
  // no global-memory round trip of its own.
  // Where no level of the last learned run on this graph was inside the
  // model's domain (`eager` clear), only the box and its cell map are staged
  // up front, and the model and anchors only for a level in a cell near
  // some anchor.
  const bool learned = (s.mode == 1) && s.model;
  const bool eager = learned && s.eager;
  float anc[kFeatures];
  const bool has_anc = learned && s.anchors && t < s.n_anchors;
  auto stage_model = [&]() {
    // (the second layer's weights transposed, so that lane u reading weight
    // (u, j) of every hidden unit u at once touches consecutive words)
    constexpr int kW2 = 32 * kFeatures + 32;
    for (int i = t; i < kModelSize; i += blockDim.x) {
      const int q = i - kW2;
      sh.w[(q >= 0 && q < 32 * 32) ? kW2 + (q & 31) * 32 + (q >> 5) : i] = s.model[i];
    }
    if (has_anc) {
#pragma unroll
      for (int f = 0; f < kFeatures; ++f) anc[f] = s.anchors[t * kFeatures + f];
    }
  };
  if (learned && s.box) {
    for (int i = t; i < 3 * kFeatures + kCellWords; i += blockDim.x) {
      if (i < 2 * kFeatures) sh.box[i] = s.box[i];
      else if (i < 3 * kFeatures) sh.cscale[i - 2 * kFeatures] = s.cells[i - 2 * kFeatures];
      else sh.cells[i - 3 * kFeatures] = __float_as_uint(s.cells[i - 2 * kFeatures]);
    }
  }
  if (eager) stage_model();
  // Level k-1's counters: written by earlier kernels (or, in the persistent
  // form, before the grid barrier, whose acquire makes them visible), so
  // plain loads see them.  The lanes of the first wavefront load one slot
  // each, all in flight at once, and add them up exactly (integers); its
  // lane 0 forms the features.
  if (t < kC) {
    unsigned long long nf_u = 0ull, mf_u = 0ull;
    if (t < kRingSlots) {
      const unsigned long long* c =
          s.ring_ctr + ((int64_t)((k - 1) % kRing) * kRingSlots + t) * kCountFields;
      nf_u = c[0];
      mf_u = c[4];
    }
#pragma unroll
    for (int off = kRingSlots / 2; off > 0; off >>= 1) {
      nf_u += __shfl_xor(nf_u, off);
      mf_u += __shfl_xor(mf_u, off);
    }
    if (t == 0) {
      const double nf = (double)nf_u, mf = (double)mf_u;
      sh.stop = (k > 1 && nf_u == 0ull) ? 1 : 0;  // the previous level found nothing
      if (k > 1) {
        sh.sums[0] += nf;
        sh.sums[1] += mf;
      }
      // the logarithms are taken in single precision (the features are
      // single-precision values)
      const double mu0 = fmax(s.two_m - sh.sums[1], 0.0);
      const float lnf = log2f((float)(1.0 + nf)), lmf = log2f((float)(1.0 + mf));
      const float lmu = log2f((float)(1.0 + mu0));
      sh.x[0] = lnf / s.l2n;
      sh.x[1] = lmf / s.l2m;
      sh.x[2] = lmu / s.l2m;
      sh.x[3] = fminf(fmaxf((lmf - lnf) / 16.0f, 0.0f), 1.0f);
      sh.x[4] = fminf(fmaxf((lmu - s.log2n) / 8.0f, -1.0f), 1.0f);
      sh.x[5] = fminf(fmaxf((lmf - lmu) / 16.0f, -1.0f), 1.0f);
      sh.sums[2] = nf;
      sh.mf = (float)mf;
      sh.mu = (float)mu0;
    }
  }
  // the anchors are needed in registers from here on: without this the
  // compiler issues their loads only where they are used, after the barrier
  if (eager && has_anc) {
#pragma unroll
    for (int f = 0; f < kFeatures; ++f) asm volatile("" ::"v"(anc[f]));
  }
  __syncthreads();
  if ((sh.pub >> 3) == tag) return (int32_t)(sh.pub & 7u) - 2;
  if (sh.stop) {
    if (writer && t == 0 && s.decided)
      __hip_atomic_store(&s.decided[k % kRing], (tag << 3) | (uint64_t)(kStop + 2),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (writer && t == 0) s.variant[k % kRing] = kStop;
    return kStop;
  }
  // The fixed heuristic (the direction rule of Beamer et al. with alpha =
  // 14): pull once the frontier's edges exceed 1/14 of the unvisited edges.
  // Every thread evaluates it (and every workgroup alike).
  const int32_t h = (sh.mf * 14.0f > sh.mu) ? s.heuristic_pull : kPush;
  int32_t v = s.mode >= 3 ? s.mode - 3 : h;
  // Learned: the model's choice stands only for a level inside its training
  // domain (within tau of an anchor); outside it, the heuristic's.  A level
  // outside the anchors' box widened by tau is outside for sure; otherwise
  // every thread measures its anchor's distance to the level's features and
  // the nearest decides.  Only then does the first wavefront score the four
  // variants with the MLP, one hidden unit per lane, in registers.
  bool use_model = learned;
  if (use_model && s.anchors && s.box) {
    bool in = true;
    int cell = 0, stride = 1;
    for (int f = 0; f < kFeatures; ++f) {
      in = in && sh.x[f] >= sh.box[f] && sh.x[f] <= sh.box[kFeatures + f];
      const int q = (int)fminf(fmaxf(floorf((sh.x[f] - sh.box[f]) * sh.cscale[f]), 0.0f),
                               (float)(kCellBins - 1));
      cell += q * stride;
      stride *= kCellBins;
    }
    // inside the box, a level in a cell that meets no anchor's cube is
    // outside the domain as well
    in = in && ((sh.cells[cell >> 5] >> (cell & 31)) & 1u) != 0u;
    use_model = in;  // the same value in every thread
  }
  if (use_model && !eager) {
    stage_model();
    if (!s.anchors) __syncthreads();  // (otherwise the anchor test's barrier)
  }
  if (use_model && s.anchors) {
    // inside the domain iff some anchor lies within tau: each thread tests
    // its own (the comparison is exact, so every workgroup agrees), and one
    // barrier ORs the answers
    bool near = false;
    if (has_anc) {
      float d2 = 0.f;
#pragma unroll
      for (int f = 0; f < kFeatures; ++f) {
        const float df = sh.x[f] - anc[f];
        d2 = fmaf(df, df, d2);
      }
      near = d2 <= s.tau2;
    }
    for (int i = t + blockDim.x; i < s.n_anchors; i += blockDim.x) {  // small workgroups
      float d2 = 0.f;
#pragma unroll
      for (int f = 0; f < kFeatures; ++f) {
        const float df = sh.x[f] - s.anchors[i * kFeatures + f];
        d2 = fmaf(df, df, d2);
      }
      near = near || d2 <= s.tau2;
    }
    use_model = __syncthreads_or(near ? 1 : 0) != 0;
  }
  if (use_model) {
    // inside the domain: tell the host to stage up front on the next run
    if (writer && t == 0 && s.in_box)
      __hip_atomic_store(s.in_box, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    if (t < kC) {
      const float* W1 = sh.w;
      const float* b1 = W1 + 32 * kFeatures;
      const float* W2t = b1 + 32;  // [j][u]: transposed when staged
      const float* b2 = W2t + 32 * 32;
      const float* W3 = b2 + 32;
      const float* b3 = W3 + kVariants * 32;
      const int u = t & 31;  // hidden unit of this lane (lanes 32..63 mirror 0..31)
      float hh = b1[u];
#pragma unroll
      for (int i = 0; i < kFeatures; ++i) hh = fmaf(W1[u * kFeatures + i], sh.x[i], hh);
      hh = hh > 0.f ? hh : 0.f;
      // layer 2: hidden unit j of layer 1 is read from lane j
      float h2 = b2[u];
#pragma unroll
      for (int j = 0; j < 32; ++j) h2 = fmaf(W2t[j * 32 + u], lane_value(hh, j), h2);
      h2 = h2 > 0.f ? h2 : 0.f;
      // layer 3 in every lane (lane u scores variant u mod 4): a branch
      // around it would let the compiler compute h2 only in the lanes that
      // take the branch, while the readlanes read it from all 32
      const int v3 = u & (kVariants - 1);
      float o = b3[v3];
#pragma unroll
      for (int j = 0; j < 32; ++j) o = fmaf(W3[v3 * 32 + j], lane_value(h2, j), o);
      if (t < kVariants) sh.out[t] = o;
      // lane 0: the lowest score, if every score is finite (else the heuristic)
      const float o0 = lane_value(o, 0), o1 = lane_value(o, 1), o2 = lane_value(o, 2),
                  o3 = lane_value(o, 3);
      if (t == 0) {
        int32_t m = 0;
        float om = o0;
        if (o1 < om) { m = 1; om = o1; }
        if (o2 < om) { m = 2; om = o2; }
        if (o3 < om) { m = 3; om = o3; }
        const bool finite = isfinite(o0) && isfinite(o1) && isfinite(o2) && isfinite(o3);
        sh.v = finite ? m : h;
      }
    }
    __syncthreads();
    v = sh.v;
  }
  // the records go out last, so no wavefront waits for them at a barrier;
  // only the writer publishes (stores from every workgroup to one word are
  // serialised by the memory system, about 57 ns each)
  if (writer && t == 0 && s.decided)
    __hip_atomic_store(&s.decided[k % kRing], (tag << 3) | (uint64_t)(v + 2), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  if (t == 0 && writer) {
    s.variant[k % kRing] = v;
    if (s.log && k <= s.log_cap) {
      float* L = s.log + (int64_t)(k - 1) * 12;
      for (int i = 0; i < kFeatures; ++i) L[i] = sh.x[i];
      for (int i = 0; i < kVariants; ++i) L[kFeatures + i] = use_model ? sh.out[i] : 0.f;
      L[10] = (float)v;
      L[11] = (float)k;
    }
  }
  return v;
}

// Clear what level k accumulates into: its counters, queue length and push
// segment count (one workgroup).
__device__ __forceinline__ void sched_clear_level(const SchedArgs& s, int32_t k) {
  unsigned long long* mine = s.ring_ctr + (int64_t)(k % kRing) * kRingSlots * kCountFields;
  for (int i = threadIdx.x; i < kRingSlots * kCountFields; i += blockDim.x) mine[i] = 0ull;
  if (threadIdx.x == 0) {
    s.qn[k % kRing] = 0;
    s.seg_n[k & 1] = 0;
  }
}

// One scheduled level k: every workgroup computes the level's variant from
// level k-1's counters (same inputs and arithmetic everywhere, so all agree)
// and runs the pull variant or the push scatter; workgroup 0 reports level
// k-1 to the host, records the decision and the running totals, and clears
// what level k+1 accumulates into.  The running totals are double-buffered
// by level parity: level k reads buffer (k-1)&1 and writes buffer k&1.
template <class S, int U, bool STAGED>
__device__ __forceinline__ void sched_level_entry(const LevelArgs& a, const SchedArgs& s,
                                                  uint8_t* lds_stage) {
  __shared__ SchedShared sh;
  const int32_t k = a.level;
  const bool writer = blockIdx.x == 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < 3; ++i) sh.sums[i] = s.sums[4 * ((k - 1) & 1) + i];
  const int32_t v = schedule_pick(s, k, sh, writer);
  if (writer && threadIdx.x == 0) {
    if (k > 1) {
      const uint64_t tag = level_tag(s.run_id, k - 1);
      __hip_atomic_store(&s.report[(k - 1) % kRing], (tag << 1) | (v != kStop ? 1u : 0u),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    for (int i = 0; i < 3; ++i) s.sums[4 * (k & 1) + i] = sh.sums[i];
  }
  if (v == kStop) return;
  if (writer) sched_clear_level(s, k + 1);
  if (v < kPullVariants)
    level_body<S, U, STAGED>(a, a.vunits[v], a.vpieces[v], a.vn_units[v], a.vbundle[v],
                             a.varrive2[v], a.vpiece_cols[v], a.vwave_off[v], lds_stage);
  else
    push_scatter_body<S>(a, grid_wave(), grid_waves(), push_stage<STAGED>(a, lds_stage));
}

template <class S, int U, bool STAGED>
__global__ void sched_level_kernel(LevelArgs a, SchedArgs s) {
  extern __shared__ uint8_t lds_stage[];
  sched_level_entry<S, U, STAGED>(a, s, lds_stage);
}

// The four-column form held to 64 registers per lane, as for plain levels:
// two 16-wavefront workgroups per compute unit.
template <class S, bool STAGED>
__global__ void __launch_bounds__(1024, 8) sched_level_kernel_w8(LevelArgs a, SchedArgs s) {
  extern __shared__ uint8_t lds_stage[];
  sched_level_entry<S, 4, STAGED>(a, s, lds_stage);
}

// Level-0 state of a scheduled run: the root is the frontier queue, and the
// synthetic level-0 counters hold one discovered vertex of degree deg(root).
// Level 1's counters, queue length and segment count start at zero too (the
// persistent form clears one level ahead).
__global__ void sched_init_kernel(int32_t root_row, const int32_t* deg, int32_t* q0, int32_t* qn,
                                  int32_t* seg_n, unsigned long long* ring_ctr, double* sums) {
  const int t = threadIdx.x;
  for (int i = t; i < 2 * kRingSlots * kCountFields; i += blockDim.x) ring_ctr[i] = 0ull;
  __syncthreads();
  if (t == 0) {
    const int32_t d = deg[root_row];
    q0[0] = root_row;
    qn[0] = 1;
    qn[1] = 0;
    seg_n[1] = 0;
    ring_ctr[0] = 1ull;
    ring_ctr[4] = (unsigned long long)d;
    sums[0] = 1.0;
    sums[1] = (double)d;
    sums[2] = 0.0;
    sums[3] = 0.0;
  }
}

// ------------------------------------------------ persistent schedule form ---
//
// A scheduled run in one cooperative launch.  Every workgroup computes each
// level's variant itself from the previous level's counters (identical
// inputs, identical arithmetic, so all take the same branch and meet the
// same barriers); workgroup 0 records it and clears the next level's
// counters.  A pull level is one phase; a push level is scatter, segments
// (only when long rows were queued) and post, each closed by a grid barrier.

template <class S, int U, bool STAGED>
__global__ void persistent_sched_kernel(LevelArgs a, SchedArgs s, void* buf_a, void* buf_b,
                                        int32_t* q0, int32_t* q1, int32_t cap, unsigned* bar,
                                        int32_t* status, uint64_t limit) {
  extern __shared__ uint8_t lds_stage[];
  __shared__ SchedShared sh;
  const bool writer = blockIdx.x == 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < 3; ++i) sh.sums[i] = s.sums[i];
  const int64_t gw = grid_wave(), nw = grid_waves();
  const int32_t count_stats = a.count_stats;
  for (int32_t k = 1; k <= cap; ++k) {
    a.level = k;
    a.vin = (k & 1) ? buf_a : buf_b;
    a.vout = (k & 1) ? buf_b : buf_a;
    a.q_in = (k & 1) ? q0 : q1;
    a.q_out = (k & 1) ? q1 : q0;
    a.seg_n = s.seg_n + (k & 1);
    a.count_stats = count_stats && (k <= status[2]);
    const int32_t v = schedule_pick(s, k, sh, writer);
    if (v == kStop) {  // level k-1 found nothing (every workgroup sees the same counters)
      if (writer && threadIdx.x == 0) status[0] = k - 1;
      return;
    }
    if (writer && k < cap) sched_clear_level(s, k + 1);
    if (v < kPullVariants) {
      level_body<S, U, STAGED>(a, a.vunits[v], a.vpieces[v], a.vn_units[v], a.vbundle[v],
                             a.varrive2[v], a.vpiece_cols[v], nullptr, lds_stage);
    } else {
      push_scatter_body<S>(a, gw, nw, push_stage<STAGED>(a, lds_stage));
      if (!grid_barrier(bar, gridDim.x, limit, &status[1])) return;
      if (load_count(a.seg_n) > 0) {
        push_segments_body<S>(a, gw, nw, push_stage<STAGED>(a, lds_stage));
        if (!grid_barrier(bar, gridDim.x, limit, &status[1])) return;
      }
      push_post_body<S>(a, gw, nw);
    }
    if (!grid_barrier(bar, gridDim.x, limit, &status[1])) return;
    if (a.any[k % kRing] != level_tag(a.run_id, k)) {
      if (writer && threadIdx.x == 0) status[0] = k;  // levels run
      return;
    }
  }
  if (writer && threadIdx.x == 0) status[0] = -1;  // cap reached
}

// ----------------------------------------------------------- init kernel ---

// Level-0 vectors (Section III-A): tropical x_0 = f_0 = e_r-style distances,
// real/boolean f_0 = e_r with filter g = NOT f_0, sel-max x_0 = p_0 = (r+1) e_r.
// Phantom rows start final so SlimWork can skip them.
template <int SEMI>
__global__ void init_kernel(int32_t n, int32_t n_pad, int64_t n_chunks, const int32_t* v,
                            int32_t root_row, void* va, void* vb, int32_t* state, uint8_t* g,
                            int32_t* d, float* rv, int32_t* acc, int32_t* arrive, uint32_t* summ,
                            int32_t summ_words, uint8_t* done) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n_chunks) {
    arrive[r] = 0;
    if (done) done[r] = 0;
  }
  if (summ && r < summ_words) {
    // level 0's frontier summary holds the root's chunk; level 1's starts empty
    const int32_t rc = root_row / kC;
    summ[r] = (r == rc >> 5) ? (1u << (rc & 31)) : 0u;
    summ[summ_words + r] = 0u;
    if (r == 0) summ[3 * (int64_t)summ_words] = 1u;  // level 0's summary is valid
  }
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
  if (SEMI != SS_SELMAX) g[r] = (root || phantom) ? 0 : 1;  // sel-max reads no filter
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
    // Both bitmap buffers start clean: a push level adds bits to a buffer
    // that still holds older bits, which is safe only for bits of this run.
    if (r < n_chunks) {
      static_cast<uint64_t*>(va)[r] = (r == root_row / kC) ? (1ull << (root_row % kC)) : 0ull;
      static_cast<uint64_t*>(vb)[r] = 0ull;
    }
    state[r] = root ? v[r] : (phantom ? -1 : 0);
    acc[r] = 0;
  }
}

// ------------------------------------------------------- finalise kernel ---

// Row order -> original IDs; infinity -> -1; 1-based parents -> 0-based.
// One thread per original ID, so the outputs are written coalesced; the
// row-order values are gathered.  (Scattering from row order instead writes
// partial lines and measured more than twice as slow.)
template <int SEMI>
__global__ void finalise_kernel(int32_t n, const int32_t* perm, const int32_t* state,
                                const int32_t* d, const float* rv, int32_t* dist, int32_t* parent,
                                float* real_val) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n) return;
  // the outputs are written once and not read again here: streaming stores
  const int32_t row = __builtin_nontemporal_load(perm + o);
  if (SEMI == SS_TROPICAL) {
    const int32_t f = state[row];
    __builtin_nontemporal_store((f >= kInf) ? -1 : f, dist + o);
    return;
  }
  const int32_t dr = d[row];
  const int32_t pr = (SEMI == SS_SELMAX && parent) ? state[row] : 0;
  __builtin_nontemporal_store(dr, dist + o);
  if (SEMI == SS_SELMAX && parent) __builtin_nontemporal_store((pr > 0) ? pr - 1 : -1, parent + o);
  if (SEMI == SS_REAL && real_val) __builtin_nontemporal_store(rv[row], real_val + o);
}

// Batched level 0: every row starts with an empty mask (phantom rows are
// final); then each used root slot sets its bit and level 0 at its root row.
__global__ void batch_init_kernel(int32_t n_pad, int64_t n_chunks, const int32_t* v,
                                  unsigned long long* vis, unsigned long long* fa,
                                  unsigned long long* acc64, int32_t* arrive, uint32_t* summ,
                                  int32_t summ_words, uint8_t* done) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n_chunks) {
    arrive[r] = 0;
    if (done) done[r] = 0;
  }
  if (summ && r < summ_words) {
    // level 0's summary gets the roots' chunks (next kernel); level 1's starts empty
    summ[r] = 0u;
    summ[summ_words + r] = 0u;
    if (r == 0) summ[3 * (int64_t)summ_words] = 1u;  // level 0's summary is valid
  }
  if (r >= n_pad) return;
  vis[r] = (v[r] == 0) ? ~0ull : 0ull;
  fa[r] = 0ull;
  acc64[r] = 0ull;
}

__global__ void batch_roots_kernel(int32_t count, const int32_t* root_rows, const int32_t* slots,
                                   unsigned long long* vis, unsigned long long* fa,
                                   uint16_t* lvl, uint32_t* summ) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int32_t row = root_rows[i];
  const unsigned long long bit = 1ull << slots[i];
  atomicOr(&vis[row], bit);
  atomicOr(&fa[row], bit);
  if (summ) atomicOr(&summ[row / kC >> 5], 1u << ((row / kC) & 31));
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
  // the row's level record is 128 contiguous bytes: read it 16 bytes (eight
  // slots) at a time instead of one 2-byte load per slot
  const uint4* lv = reinterpret_cast<const uint4*>(lvl + (int64_t)row * 64);
  int32_t* out = dist + (int64_t)rpg * base + (o - base);
  const int32_t nq = (rpg + 7) / 8;
  uint4 w[8];  // all loads in flight before the first store
#pragma unroll
  for (int q = 0; q < 8; ++q) w[q] = q < nq ? lv[q] : make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const uint32_t x[4] = {w[q].x, w[q].y, w[q].z, w[q].w};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int32_t b = q * 8 + k;
      if (b < rpg) {
        const int32_t level = (int32_t)((x[k >> 1] >> ((k & 1) * 16)) & 0xFFFFu);
        // every output is written once and never read here: stream it
        __builtin_nontemporal_store(((seen >> b) & 1ull) ? level : -1, out + (int64_t)b * ni);
      }
    }
  }
}

template <class T>
__global__ void fill_kernel(T* p, T value, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

// --------------------------------------------------------------- launchers ---

static inline unsigned blocks_for(int64_t n, int threads) {
  return (unsigned)((n + threads - 1) / threads);
}

int launch_init(int semiring, const Graph& g, const Workspace& ws, int32_t root_row, bool summary,
                void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t work = g.n_pad > g.n_chunks ? g.n_pad : g.n_chunks;
  const unsigned blocks = blocks_for(work, 256);
  uint32_t* summ = summary ? ws.summ : nullptr;
#define SS_INIT(S)                                                                             \
  init_kernel<S><<<blocks, 256, 0, st>>>(g.n, g.n_pad, g.n_chunks, g.d_v, root_row, ws.vec_a, \
                                         ws.vec_b, ws.state, ws.g, ws.d, ws.rv, ws.acc,       \
                                         ws.arrive, summ, ws.summ_words, ws.done)
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

template <class S, bool STAGED>
static void launch_level_u(int waves, int unroll, unsigned grid, const LevelArgs& a,
                           hipStream_t st) {
  const size_t lds = STAGED ? level_lds(a) : 0;
  if (a.val)  // the Sell-C-sigma comparator is built for one unroll depth
    level_kernel<S, 8, STAGED, true><<<grid, waves * kC, lds, st>>>(a);
  else if (unroll == 4) {
    if constexpr (S::kSingleRoot)
      level_kernel_w8<S, STAGED><<<grid, waves * kC, lds, st>>>(a);
    else
      level_kernel<S, 4, STAGED><<<grid, waves * kC, lds, st>>>(a);
  }
  else if (unroll == 16)
    level_kernel<S, 16, STAGED><<<grid, waves * kC, lds, st>>>(a);
  else
    level_kernel<S, 8, STAGED><<<grid, waves * kC, lds, st>>>(a);
}

template <class S>
static void launch_level_t(int waves, int unroll, unsigned grid, const LevelArgs& a,
                           hipStream_t st) {
  if (level_lds(a))
    launch_level_u<S, true>(waves, unroll, grid, a, st);
  else
    launch_level_u<S, false>(waves, unroll, grid, a, st);
}

int launch_level(int semiring, int waves, int unroll, int64_t max_groups, const LevelArgs& a,
                 void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t groups = level_groups(a.n_units, waves, max_groups);
  const unsigned grid = (unsigned)groups;
  switch (semiring) {
    case SS_TROPICAL: launch_level_t<Tropical>(waves, unroll, grid, a, st); break;
    case SS_REAL: launch_level_t<Real>(waves, unroll, grid, a, st); break;
    case SS_BOOLEAN: launch_level_t<Boolean>(waves, unroll, grid, a, st); break;
    case SS_SELMAX: launch_level_t<SelMax>(waves, unroll, grid, a, st); break;
    case kBatchSemiring: launch_level_t<Batch>(waves, unroll, grid, a, st); break;
    case kDpSemiring: launch_level_t<Dp>(waves, unroll, grid, a, st); break;
    default: return set_error(SS_EINVAL, "unknown semiring");
  }
  return check_launch("level_kernel");
}

int launch_push(int semiring, const LevelArgs& a, bool segments, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  constexpr unsigned kGroups = 2048, kThreads = 256;
  switch (semiring) {
#define SS_PUSH(S)                                                  \
  if (segments) push_segments_kernel<S><<<kGroups, kThreads, 0, st>>>(a); \
  push_post_kernel<S><<<kGroups / 2, kThreads, 0, st>>>(a);          \
  break;
    case SS_TROPICAL: SS_PUSH(Tropical)
    case SS_REAL: SS_PUSH(Real)
    case SS_BOOLEAN: SS_PUSH(Boolean)
    case SS_SELMAX: SS_PUSH(SelMax)
#undef SS_PUSH
    default: return set_error(SS_EINVAL, "push needs a single-root semiring");
  }
  return check_launch("push kernels");
}

static SchedArgs sched_args(const SchedLaunch& p, int32_t level, uint32_t run_id) {
  SchedArgs s;
  s.level = level;
  s.run_id = run_id;
  s.any = p.any;
  s.report = p.report;
  s.variant = p.variant;
  s.qn = p.qn;
  s.seg_n = p.seg_n;
  s.ring_ctr = p.ring_ctr;
  s.sums = p.sums;
  s.model = p.model;
  s.anchors = p.anchors;
  s.box = p.box;
  s.cells = p.cells;
  s.decided = p.decided;
  s.in_box = p.in_box;
  s.eager = p.eager;
  s.n_anchors = p.n_anchors;
  s.tau2 = p.tau2;
  s.log = p.log;
  s.log_cap = p.log_cap;
  s.mode = p.mode;
  s.heuristic_pull = p.heuristic_pull;
  s.n = p.n;
  s.two_m = p.two_m;
  s.log2n = (float)std::log2(p.n);
  s.l2n = (float)std::log2(p.n > 2.0 ? p.n : 2.0);
  s.l2m = (float)std::log2(1.0 + (p.two_m > 1.0 ? p.two_m : 1.0));
  return s;
}

template <class S, bool STAGED>
static void launch_sched_level_u(int waves, int unroll, unsigned grid, const LevelArgs& a,
                                 const SchedArgs& sa, hipStream_t st) {
  const size_t lds = STAGED ? level_lds(a) : 0;
  if (unroll == 4)
    sched_level_kernel_w8<S, STAGED><<<grid, waves * kC, lds, st>>>(a, sa);
  else if (unroll == 16)
    sched_level_kernel<S, 16, STAGED><<<grid, waves * kC, lds, st>>>(a, sa);
  else
    sched_level_kernel<S, 8, STAGED><<<grid, waves * kC, lds, st>>>(a, sa);
}

int launch_sched_level(int semiring, int waves, int unroll, int64_t max_groups,
                       const LevelArgs& a, const SchedLaunch& p, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  int64_t groups = (a.n_units + waves - 1) / waves;
  if (groups < 1) groups = 1;
  if (max_groups > 0 && groups > max_groups) groups = max_groups;
  const unsigned grid = (unsigned)groups;
  const SchedArgs sa = sched_args(p, a.level, a.run_id);
#define SS_SL(S)                                                      \
  if (level_lds(a))                                                   \
    launch_sched_level_u<S, true>(waves, unroll, grid, a, sa, st);    \
  else                                                                \
    launch_sched_level_u<S, false>(waves, unroll, grid, a, sa, st);   \
  break;
  switch (semiring) {
    case SS_TROPICAL: SS_SL(Tropical)
    case SS_REAL: SS_SL(Real)
    case SS_BOOLEAN: SS_SL(Boolean)
    case SS_SELMAX: SS_SL(SelMax)
#undef SS_SL
    default: return set_error(SS_EINVAL, "a scheduled run needs a single-root semiring");
  }
  return check_launch("sched_level_kernel");
}

int launch_sched_init(const Graph& g, const Workspace& ws, int32_t root_row, void* stream) {
  sched_init_kernel<<<1, 64, 0, static_cast<hipStream_t>(stream)>>>(root_row, g.d_deg, ws.q[0],
                                                                     ws.qn, ws.seg_n, ws.ring_ctr,
                                                                     ws.sched_sums);
  return check_launch("sched_init_kernel");
}

// The persistent grid is one 1024-thread workgroup per compute unit: a shape
// every CU can hold at once, so all workgroups are resident and the grid
// barrier cannot wait on a workgroup that has not started.
constexpr int kPersistentWaves = 16;

template <class S, bool STAGED>
static int launch_persistent_u(int unroll, const LevelArgs& a, void* buf_a, void* buf_b,
                               const PersistentRun& r, hipStream_t st) {
  const size_t lds = STAGED ? level_lds(a) : 0;
  const void* fn;
  if (r.sched) {
    if constexpr (S::kSingleRoot) {
      fn = unroll == 4    ? (const void*)persistent_sched_kernel<S, 4, STAGED>
           : unroll == 16 ? (const void*)persistent_sched_kernel<S, 16, STAGED>
                          : (const void*)persistent_sched_kernel<S, 8, STAGED>;
    } else {
      return set_error(SS_EINVAL, "a scheduled run needs a single-root semiring");
    }
  } else {
    fn = unroll == 4    ? (const void*)persistent_kernel<S, 4, STAGED>
         : unroll == 16 ? (const void*)persistent_kernel<S, 16, STAGED>
                        : (const void*)persistent_kernel<S, 8, STAGED>;
  }
  int per_cu = 0, dev = 0, cus = 0, coop = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kPersistentWaves * kC, lds);
  if (e != hipSuccess) return set_error(SS_EHIP, std::string("occupancy: ") + hipGetErrorString(e));
  if (!coop) return set_error(SS_EUNSUP, "the device has no cooperative launch");
  if (per_cu < 1) return set_error(SS_EUNSUP, "persistent kernel does not fit on a compute unit");
  int64_t grid = cus;
  if (r.max_groups > 0 && grid > r.max_groups) grid = r.max_groups;
  LevelArgs aa = a;
  int32_t cap = r.cap;
  unsigned* bar = r.bar;
  int32_t* status = r.status;
  uint64_t limit = r.limit;
  if (r.sched) {
    SchedArgs sa = sched_args(*r.sched, 0, a.run_id);
    sa.decided = nullptr;  // all workgroups are resident: each decides, and keeps its totals
    int32_t* q0 = r.q0;
    int32_t* q1 = r.q1;
    void* args[] = {&aa, &sa, &buf_a, &buf_b, &q0, &q1, &cap, &bar, &status, &limit};
    e = hipLaunchCooperativeKernel(fn, dim3((unsigned)grid), dim3(kPersistentWaves * kC), args,
                                   lds, st);
  } else {
    void* args[] = {&aa, &buf_a, &buf_b, &cap, &bar, &status, &limit};
    e = hipLaunchCooperativeKernel(fn, dim3((unsigned)grid), dim3(kPersistentWaves * kC), args,
                                   lds, st);
  }
  if (e != hipSuccess)
    return set_error(SS_EHIP, std::string("cooperative launch: ") + hipGetErrorString(e));
  return SS_OK;
}

int launch_persistent(int semiring, int unroll, const LevelArgs& a, void* buf_a, void* buf_b,
                      const PersistentRun& r, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
#define SS_PERS(S)                                                                \
  return level_lds(a) ? launch_persistent_u<S, true>(unroll, a, buf_a, buf_b, r, st) \
                     : launch_persistent_u<S, false>(unroll, a, buf_a, buf_b, r, st);
  switch (semiring) {
    case SS_TROPICAL: SS_PERS(Tropical)
    case SS_REAL: SS_PERS(Real)
    case SS_BOOLEAN: SS_PERS(Boolean)
    case SS_SELMAX: SS_PERS(SelMax)
    case kBatchSemiring: SS_PERS(Batch)
    default: return set_error(SS_EINVAL, "unknown semiring");
  }
#undef SS_PERS
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

int launch_batch_init(const Graph& g, const BatchWorkspace& b, int32_t count, bool summary,
                      void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  uint32_t* summ = summary ? g.ws.summ : nullptr;
  batch_init_kernel<<<blocks_for(g.n_pad, 256), 256, 0, st>>>(g.n_pad, g.n_chunks, g.d_v, b.vis,
                                                              b.fa, b.acc64, g.ws.arrive, summ,
                                                              g.ws.summ_words, g.ws.done);
  int rc = check_launch("batch_init_kernel");
  if (rc || count == 0) return rc;
  batch_roots_kernel<<<blocks_for(count, 256), 256, 0, st>>>(count, b.root_rows, b.slots, b.vis,
                                                             b.fa, b.lvl, summ);
  return check_launch("batch_roots_kernel");
}

int launch_batch_finalise(const Graph& g, const BatchWorkspace& b, int32_t rpg, int32_t* dist,
                          void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  batch_finalise_kernel<<<blocks_for(g.n, 256), 256, 0, st>>>(
      g.n, g.num_graphs, g.d_voff, g.d_perm, b.vis, b.lvl, rpg, dist);
  return check_launch("batch_finalise_kernel");
}

__global__ void sell_build_kernel(const int32_t* col, int64_t cells, int32_t* scol,
                                  int32_t* sval) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cells;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t c = col[i];
    scol[i] = c >= 0 ? c : 0;
    sval[i] = c >= 0 ? 1 : 0;
  }
}

int launch_sell_build(const int32_t* col, int64_t cells, int32_t* scol, int32_t* sval,
                      void* stream) {
  if (cells <= 0) return SS_OK;
  unsigned blocks = blocks_for(cells, 256);
  if (blocks > 8192) blocks = 8192;
  sell_build_kernel<<<blocks, 256, 0, static_cast<hipStream_t>(stream)>>>(col, cells, scol, sval);
  return check_launch("sell_build_kernel");
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
