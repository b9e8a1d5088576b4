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

__device__ __forceinline__ int32_t wave_max(int32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const int32_t o = __shfl_xor(v, off);
    v = o > v ? o : v;
  }
  return v;
}

}  // namespace ss
