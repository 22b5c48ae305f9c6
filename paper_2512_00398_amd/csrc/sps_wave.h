// sps_wave.h - wave64 building blocks for gfx950 (CDNA4).
//
// Every helper that exchanges data between lanes must be called with all 64
// lanes of the wave active (wave-uniform control flow).
#pragma once

#include <climits>

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sps {

__device__ __forceinline__ int lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// Lanes where p holds; compiles to the compare's own lane mask.
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

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

// DPP lane move: lanes whose source is outside the row, or whose row/bank is
// masked off, receive `old`. Controls (GFX9 encoding): row_shr:n = 0x110+n,
// row_mirror = 0x140, row_half_mirror = 0x141, row_bcast:15 = 0x142,
// row_bcast:31 = 0x143, quad_perm = 0x00..0xff.
template <int CTRL, int ROW_MASK = 0xf, int BANK_MASK = 0xf>
__device__ __forceinline__ int dpp(int old, int src) {
  return __builtin_amdgcn_update_dpp(old, src, CTRL, ROW_MASK, BANK_MASK, false);
}

// Inclusive prefix sum over the 64 lanes (Hillis-Steele within rows of 16,
// then row broadcasts).
__device__ __forceinline__ int wave_scan_incl(int v) {
  v += dpp<0x111>(0, v);
  v += dpp<0x112>(0, v);
  v += dpp<0x114>(0, v);
  v += dpp<0x118>(0, v);
  v += dpp<0x142, 0xa>(0, v);
  v += dpp<0x143, 0xc>(0, v);
  return v;
}

// One level of a max-reduction: max(v, v moved by CTRL). Masked-off rows
// receive INT_MIN, the identity of max, which lets the compiler fold the lane
// move into the max itself (one DPP instruction per level).
template <int CTRL, int RM = 0xf>
__device__ __forceinline__ int max_step(int v) {
  return max(v, dpp<CTRL, RM>(INT_MIN, v));
}

template <int CTRL, int RM = 0xf>
__device__ __forceinline__ int min_step(int v) {
  return min(v, dpp<CTRL, RM>(INT_MAX, v));
}

// Maximum over the 64 lanes, returned wave-uniform.
__device__ __forceinline__ int wave_max_u(int v) {
  v = max_step<0xb1>(v);        // quad_perm [1,0,3,2]
  v = max_step<0x4e>(v);        // quad_perm [2,3,0,1]
  v = max_step<0x141>(v);       // row_half_mirror
  v = max_step<0x140>(v);       // row_mirror
  v = max_step<0x142, 0xa>(v);  // row_bcast:15
  v = max_step<0x143, 0xc>(v);  // row_bcast:31
  return readlane(v, 63);
}

// Minimum over the 64 lanes, returned wave-uniform.
__device__ __forceinline__ int wave_min_u(int v) {
  v = min_step<0xb1>(v);
  v = min_step<0x4e>(v);
  v = min_step<0x141>(v);
  v = min_step<0x140>(v);
  v = min_step<0x142, 0xa>(v);
  v = min_step<0x143, 0xc>(v);
  return readlane(v, 63);
}

template <int CTRL, int RM>
__device__ __forceinline__ void max_step4(int& a, int& b, int& c, int& d) {
  a = max_step<CTRL, RM>(a);
  b = max_step<CTRL, RM>(b);
  c = max_step<CTRL, RM>(c);
  d = max_step<CTRL, RM>(d);
}

// wave_max_u of four values at once, interleaved so that the DPP latencies
// of the four reductions overlap.
__device__ __forceinline__ void wave_max4_u(int& a, int& b, int& c, int& d) {
  max_step4<0xb1, 0xf>(a, b, c, d);
  max_step4<0x4e, 0xf>(a, b, c, d);
  max_step4<0x141, 0xf>(a, b, c, d);
  max_step4<0x140, 0xf>(a, b, c, d);
  max_step4<0x142, 0xa>(a, b, c, d);
  max_step4<0x143, 0xc>(a, b, c, d);
  a = readlane(a, 63);
  b = readlane(b, 63);
  c = readlane(c, 63);
  d = readlane(d, 63);
}

// Sum over the 64 lanes, returned wave-uniform.
__device__ __forceinline__ int wave_sum_u(int v) { return readlane(wave_scan_incl(v), 63); }

// Lanes lo..hi (inclusive, clipped to 0..63) as a mask; empty if lo > hi.
// Branch-free (selects only).
__device__ __forceinline__ uint64_t lane_range(int lo, int hi) {
  const int l = lo < 0 ? 0 : (lo > 63 ? 63 : lo);
  const int h = hi > 63 ? 63 : (hi < 0 ? 0 : hi);
  const uint64_t upto = (2ull << h) - 1ull;  // h = 63: 2^64 wraps to 0, minus 1 = all lanes
  const uint64_t m = upto & (~0ull << l);
  return (lo > hi || hi < 0 || lo > 63) ? 0ull : m;
}

// Inclusive prefix sum within each row of 16 lanes.
__device__ __forceinline__ int row_scan_incl(int v) {
  v += dpp<0x111>(0, v);
  v += dpp<0x112>(0, v);
  v += dpp<0x114>(0, v);
  v += dpp<0x118>(0, v);
  return v;
}

// Value of lane i + D of the same row of 16 lanes (DPP row_shl:D); lanes
// whose source lies past the row end receive `old`.
template <int D>
__device__ __forceinline__ int row_down(int old, int v) {
  static_assert(D >= 1 && D <= 15, "row_shl range");
  return dpp<0x100 + D>(old, v);
}

template <int D>
__device__ __forceinline__ double row_down(double old, double v) {
  const long long o = __double_as_longlong(old), x = __double_as_longlong(v);
  const int lo = row_down<D>((int)(uint32_t)o, (int)(uint32_t)x);
  const int hi = row_down<D>((int)(o >> 32), (int)(x >> 32));
  return __longlong_as_double(((long long)hi << 32) | (uint32_t)lo);
}

// Value of lane i - D of the same row of 16 lanes (DPP row_shr:D); lanes
// whose source lies before the row start receive `old`.
template <int D>
__device__ __forceinline__ int row_up(int old, int v) {
  static_assert(D >= 1 && D <= 15, "row_shr range");
  return dpp<0x110 + D>(old, v);
}

template <int D>
__device__ __forceinline__ double row_up(double old, double v) {
  const long long o = __double_as_longlong(old), x = __double_as_longlong(v);
  const int lo = row_up<D>((int)(uint32_t)o, (int)(uint32_t)x);
  const int hi = row_up<D>((int)(o >> 32), (int)(x >> 32));
  return __longlong_as_double(((long long)hi << 32) | (uint32_t)lo);
}

// Bitwise or over each row of 16 lanes, in every lane of the row.
__device__ __forceinline__ int row_or(int v) {
  v |= dpp<0xb1>(0, v);   // quad_perm [1,0,3,2]
  v |= dpp<0x4e>(0, v);   // quad_perm [2,3,0,1]
  v |= dpp<0x141>(0, v);  // row_half_mirror
  v |= dpp<0x140>(0, v);  // row_mirror
  return v;
}

// Maximum over each row of 16 lanes, in every lane of the row.
__device__ __forceinline__ int row_max(int v) {
  v = max_step<0xb1>(v);
  v = max_step<0x4e>(v);
  v = max_step<0x141>(v);
  v = max_step<0x140>(v);
  return v;
}

// Value of v in lane l (per-lane l, 0..63).
__device__ __forceinline__ int lane_read(int v, int l) { return __builtin_amdgcn_ds_bpermute(l << 2, v); }

__device__ __forceinline__ double lane_read(double v, int l) {
  const long long x = __double_as_longlong(v);
  const int lo = lane_read((int)(uint32_t)x, l), hi = lane_read((int)(x >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (uint32_t)lo);
}

}  // namespace sps
