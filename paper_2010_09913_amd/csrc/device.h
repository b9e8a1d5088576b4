// Device helpers shared by the HIP sources: raw buffer loads and wavefront
// reductions for gfx950 (64-lane wavefronts).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace ss {

// A raw buffer load whose offset is at or past the buffer's size returns
// zero without touching memory, so a gather of a padding cell (-1) or of a
// miss needs no branch and every load of an unrolled block can be in flight
// before the first wait.
using Rsrc = __amdgpu_buffer_rsrc_t;
constexpr uint32_t kOob = 0x80000000u;  // any offset >= the buffer size reads as 0
constexpr int kRsrcWord3 = 0x00020000;  // raw buffer, gfx9 family

__device__ __forceinline__ Rsrc make_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, kRsrcWord3);
}

// Returning atomics are passed through keep(), so that wait_memory() (all of
// this wavefront's vector memory operations done) covers their completion.
__device__ __forceinline__ void keep(int32_t v) { asm volatile("" ::"v"(v)); }
__device__ __forceinline__ void wait_memory() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// LDS-staged prefix of the gathered vector.  With a full sort the rows of
// highest degree (the most gathered) come first, so each workgroup copies the
// first `bytes` of the vector into LDS once per level; a gather whose byte
// offset falls inside reads LDS, any other reads global memory.  The two
// loads are issued branch-free: the LDS read uses a clamped address and is
// masked, the buffer load gets an out-of-range offset when LDS serves it.
struct Stage {
  const uint8_t* lds;
  uint32_t bytes;  // 0 = nothing staged
  // filter: the frontier summary sits in LDS at byte `summ` (right behind
  // the largest prefix), one bit per 64-row chunk, and this level uses it
  bool filter = false;
  uint32_t summ = 0;
};

// The product terms of one block of U columns: element c[t] of the gathered
// vector for each lane (c[t] = -1 is padding).  KIND 0: one byte per row;
// 1: four bytes per row; 2: the 32-bit word of a one-bit-per-row bitmap that
// holds row c; 3: the byte of a two-bits-per-row code that holds row c.  A
// term is read from LDS when the staged prefix holds it.
// With the filter on, a term outside the prefix is read from memory only
// when its row's chunk had a row enter the frontier in the previous level;
// otherwise it is left unread (got[t] false, y[t] 0).  If no lane of the
// block needs memory, no load instruction is issued at all: this is what
// makes levels with a small frontier cheap, since every other term of the
// product is then the semiring's identity.  The filter costs an LDS round
// trip before the memory gathers, so levels whose frontier touches many
// chunks run without it.
template <int KIND>
__device__ __forceinline__ uint32_t row_offset(int32_t c) {  // byte offset of row c's element
  const uint32_t cu = (uint32_t)c;
  return c < 0 ? kOob
               : KIND == 0 ? cu : KIND == 1 ? (cu << 2) : KIND == 2 ? ((cu >> 5) << 2) : (cu >> 2);
}
template <int KIND>
constexpr bool byte_kind() { return KIND == 0 || KIND == 3; }  // elements read one byte at a time
template <int U, bool STAGED, int KIND>
__device__ __forceinline__ void gather_rows(Rsrc r, Stage st, const int32_t (&c)[U],
                                            uint32_t (&y)[U], bool (&got)[U]) {
  if (!STAGED || !st.filter) {
    // every term: LDS if the prefix holds it, else memory; both loads are
    // issued without a branch (the LDS address is clamped and its value
    // masked, the buffer load gets an out-of-range offset when LDS serves it)
    uint32_t l[U], g[U];
#pragma unroll
    for (int t = 0; t < U; ++t) {
      const uint32_t off = row_offset<KIND>(c[t]);
      const bool in = STAGED && off < st.bytes;
      l[t] = 0u;
      if (STAGED) {
        const uint32_t v = *reinterpret_cast<const uint32_t*>(st.lds + (in ? (off & ~3u) : 0u));
        l[t] = !in ? 0u : byte_kind<KIND>() ? (v >> ((off & 3u) * 8u)) & 0xFFu : v;
      }
      const uint32_t o = in ? kOob : off;
      g[t] = byte_kind<KIND>() ? (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(r, o, 0, 0)
                               : __builtin_amdgcn_raw_buffer_load_b32(r, o, 0, 0);
    }
    // every load of the block is issued before the first use: without this
    // fence a register-limited schedule waits for each load before issuing
    // the next (and, waiting for all, for the next block's prefetch too)
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < U; ++t) {
      y[t] = l[t] | g[t];
      got[t] = c[t] >= 0;
    }
    return;
  }
  uint32_t o[U];  // memory offset of the term, kOob when LDS serves it or it is skipped
  bool some = false;
  // one LDS read per term: the staged element if the prefix holds it, else
  // the summary word of its chunk (all U reads in flight before the first use)
  uint32_t lv[U];
#pragma unroll
  for (int t = 0; t < U; ++t) {
    const uint32_t cu = c[t] >= 0 ? (uint32_t)c[t] : 0u;
    const uint32_t off = row_offset<KIND>(c[t]);
    const bool in = off < st.bytes;
    const uint32_t sw = st.summ + ((cu >> 11) << 2);
    lv[t] = *reinterpret_cast<const uint32_t*>(st.lds + (in ? (off & ~3u) : sw));
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int t = 0; t < U; ++t) {
    const bool valid = c[t] >= 0;
    const uint32_t cu = valid ? (uint32_t)c[t] : 0u;
    const uint32_t off = row_offset<KIND>(c[t]);
    const bool in = off < st.bytes;
    const uint32_t v = lv[t];
    y[t] = !in ? 0u : byte_kind<KIND>() ? (v >> ((off & 3u) * 8u)) & 0xFFu : v;
    const uint32_t need = (valid && !in ? 1u : 0u) & (v >> ((cu >> 6) & 31u));
    o[t] = need ? off : kOob;
    some = some || need;
  }
  uint32_t g[U];
#pragma unroll
  for (int t = 0; t < U; ++t) g[t] = 0u;
  if (__any(some)) {
#pragma unroll
    for (int t = 0; t < U; ++t)
      g[t] = byte_kind<KIND>() ? (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(r, o[t], 0, 0)
                               : __builtin_amdgcn_raw_buffer_load_b32(r, o[t], 0, 0);
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int t = 0; t < U; ++t) {
    y[t] |= g[t];
    got[t] = o[t] != kOob || row_offset<KIND>(c[t]) < st.bytes;
  }
}

// The same for the batched SpMM's 64-bit masks (8 bytes per row): with the
// filter on, a mask outside the prefix is read only when its row's chunk
// gained frontier bits in the previous level; unread masks are 0.
template <int U, bool STAGED>
__device__ __forceinline__ void gather_masks(Rsrc r, Stage st, const int32_t (&c)[U],
                                             unsigned long long (&y)[U]) {
  if (!STAGED || !st.filter) {
    unsigned long long l[U], g[U];
#pragma unroll
    for (int t = 0; t < U; ++t) {
      const uint32_t off = c[t] >= 0 ? (uint32_t)c[t] << 3 : kOob;
      const bool in = STAGED && off < st.bytes;
      l[t] = STAGED ? *reinterpret_cast<const unsigned long long*>(st.lds + (in ? off : 0u)) : 0ull;
      if (!in) l[t] = 0ull;
      const auto w = __builtin_amdgcn_raw_buffer_load_b64(r, in ? kOob : off, 0, 0);
      g[t] = ((unsigned long long)w[1] << 32) | (unsigned long long)w[0];
    }
    __builtin_amdgcn_sched_barrier(0);  // every load of the block in flight first
#pragma unroll
    for (int t = 0; t < U; ++t) y[t] = l[t] | g[t];
    return;
  }
  uint32_t o[U];
  bool some = false;
  // the staged mask, or (as its low word) the summary word of the chunk:
  // all U LDS reads in flight before the first use
  unsigned long long lv[U];
#pragma unroll
  for (int t = 0; t < U; ++t) {
    const uint32_t cu = c[t] >= 0 ? (uint32_t)c[t] : 0u;
    const uint32_t off = c[t] >= 0 ? cu << 3 : kOob;
    const uint32_t sw = st.summ + ((cu >> 11) << 2);
    if (off < st.bytes) {
      lv[t] = *reinterpret_cast<const unsigned long long*>(st.lds + off);
    } else {
      lv[t] = *reinterpret_cast<const uint32_t*>(st.lds + sw);
    }
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int t = 0; t < U; ++t) {
    const bool valid = c[t] >= 0;
    const uint32_t cu = valid ? (uint32_t)c[t] : 0u;
    const uint32_t off = valid ? cu << 3 : kOob;
    const bool in = off < st.bytes;
    const unsigned long long v = lv[t];
    y[t] = in ? v : 0ull;
    const uint32_t need = (valid && !in ? 1u : 0u) & ((uint32_t)v >> ((cu >> 6) & 31u));
    o[t] = need ? off : kOob;
    some = some || need;
  }
  if (__any(some)) {
    unsigned long long g[U];
#pragma unroll
    for (int t = 0; t < U; ++t) {
      const auto w = __builtin_amdgcn_raw_buffer_load_b64(r, o[t], 0, 0);
      g[t] = ((unsigned long long)w[1] << 32) | (unsigned long long)w[0];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < U; ++t) y[t] |= g[t];
  }
}

__device__ __forceinline__ int32_t wave_max(int32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const int32_t o = __shfl_xor(v, off);
    v = o > v ? o : v;
  }
  return v;
}

}  // namespace ss
