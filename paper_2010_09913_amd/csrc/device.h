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
__device__ __forceinline__ uint32_t off_of(int32_t c, int shift) {
  return c >= 0 ? ((uint32_t)c << shift) : kOob;
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
};

template <bool STAGED>
__device__ __forceinline__ uint32_t gather_b32(Rsrc r, Stage st, uint32_t off) {
  if (!STAGED) return __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
  const bool in = off < st.bytes;
  uint32_t l = *reinterpret_cast<const uint32_t*>(st.lds + (in ? off : 0u));
  const uint32_t g = __builtin_amdgcn_raw_buffer_load_b32(r, in ? kOob : off, 0, 0);
  return (in ? l : 0u) | g;
}
template <bool STAGED>
__device__ __forceinline__ uint32_t gather_b8(Rsrc r, Stage st, uint32_t off) {
  if (!STAGED) return __builtin_amdgcn_raw_buffer_load_b8(r, off, 0, 0);
  const bool in = off < st.bytes;
  const uint32_t l = st.lds[in ? off : 0u];
  const uint32_t g = __builtin_amdgcn_raw_buffer_load_b8(r, in ? kOob : off, 0, 0);
  return (in ? l : 0u) | g;
}
template <bool STAGED>
__device__ __forceinline__ unsigned long long gather_b64(Rsrc r, Stage st, uint32_t off) {
  unsigned long long l = 0ull;
  bool in = false;
  if (STAGED) {
    in = off < st.bytes;
    l = *reinterpret_cast<const unsigned long long*>(st.lds + (in ? off : 0u));
  }
  const auto w = __builtin_amdgcn_raw_buffer_load_b64(r, in ? kOob : off, 0, 0);
  const unsigned long long g = ((unsigned long long)w[1] << 32) | (unsigned long long)w[0];
  return (in ? l : 0ull) | g;
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
