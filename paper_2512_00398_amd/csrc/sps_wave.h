// sps_wave.h - wave64 building blocks for gfx950 (CDNA4).
//
// Every helper that exchanges data between lanes must be called with all 64
// lanes of the wave active (wave-uniform control flow).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sps {

__device__ __forceinline__ int lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ int popc(uint64_t m) { return __popcll(m); }

// index of the lowest set bit; m must be nonzero
__device__ __forceinline__ int ctz(uint64_t m) { return __builtin_ctzll(m); }

// index of the highest set bit; m must be nonzero
__device__ __forceinline__ int msb(uint64_t m) { return 63 - __builtin_clzll(m); }

// value of v in lane l (l wave-uniform)
__device__ __forceinline__ int readlane(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

__device__ __forceinline__ int readfirst(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Orders this wave's LDS accesses: everything before is complete before
// anything after is issued.
__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Inclusive prefix sum over the 64 lanes.
__device__ __forceinline__ int wave_scan_incl(int v) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int t = __shfl_up(v, o, 64);
    v += (l >= o) ? t : 0;
  }
  return v;
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

}  // namespace sps
