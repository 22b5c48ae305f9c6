// sps_rownorm.hip - one noise scale per DM row (Heimdall++, Section II-B's
// normalisation, read as one scale per trial and chunk): with the block
// medians m_k already computed, the residual r_t = x_t - m_{floor(t/64)} of
// the whole row is formed on the fly, c = its lower median and
// MAD_row = the lower median of |r_t - c|; every block of the row then takes
// MAD_row as its scale. Exact integer order statistics.
//
// One 1024-thread workgroup per row. One pass histograms the residuals in a
// 4096-value LDS window around 0 (where the median of a baseline-removed row
// sits) and counts those below it. When c falls inside the window, the same
// histogram, prefix-summed, gives #{|r - c| <= d} = P(c + d) - P(c - d - 1)
// for every d with [c - d, c + d] inside the window, and MAD_row is the
// smallest d whose count exceeds the rank: one read of the row. Otherwise
// each statistic is an exact select of rank (N-1)/2 of its own: the window
// pass (from 0 for the deviations), then, if the rank lies outside, a radix
// select (digits of 12, 12 and 8 bits, most significant first). HBM traffic
// in the common case: 4 B per sample.
#include <hip/hip_runtime.h>

#include "sps_internal.h"
#include "sps_wave.h"

namespace sps {
namespace {

constexpr int kThreads = 1024;
constexpr int kWaves = kThreads / 64;
constexpr int kBins = 4096;

struct RowShared {
  uint32_t H[kBins];
  int part[kWaves];
  uint32_t found;  // bin index of the answer (kBins: not in the histogram)
  uint32_t below;  // values of the matching prefix below the found bin
};

// Residual of sample i of the row (block median of its 64-sample block).
__device__ __forceinline__ int resid(const float* x, const int32_t* m, int i) { return (int)x[i] - m[i >> 6]; }

// Block sum of one value per thread (every thread gets the total).
__device__ int block_sum(int v, RowShared& S) {
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  v = wave_sum_u(v);
  if (lane == 0) S.part[wave] = v;
  __syncthreads();
  int t = 0;
#pragma unroll
  for (int k = 0; k < kWaves; ++k) t += S.part[k];
  __syncthreads();
  return t;
}

// Find the bin holding rank `rho` of the histogram (each thread owns 4 bins).
// Leaves S.found / S.below (S.found = kBins when rho >= total); returns total.
__device__ int find_bin(RowShared& S, uint32_t rho) {
  const int lane = lane_id(), wave = threadIdx.x >> 6, t = threadIdx.x;
  const uint32_t h0 = S.H[4 * t], h1 = S.H[4 * t + 1], h2 = S.H[4 * t + 2], h3 = S.H[4 * t + 3];
  const int c = (int)(h0 + h1 + h2 + h3);
  const int incl = wave_scan_incl(c);
  if (lane == 63) S.part[wave] = incl;
  if (t == 0) S.found = kBins;
  __syncthreads();
  int base = 0, total = 0;
#pragma unroll
  for (int k = 0; k < kWaves; ++k) {
    const int p = S.part[k];
    base += k < wave ? p : 0;
    total += p;
  }
  const uint32_t ex = (uint32_t)(base + incl - c);
  if (ex <= rho && rho < ex + (uint32_t)c) {
    uint32_t r = rho - ex, b = 0, acc = ex;
    if (r >= h0) { r -= h0; acc += h0; b = 1;
      if (r >= h1) { r -= h1; acc += h1; b = 2;
        if (r >= h2) { r -= h2; acc += h2; b = 3; } } }
    S.found = 4 * t + b;
    S.below = acc;
  }
  __syncthreads();
  return total;
}

// H[b] <- H[0] + ... + H[b] (every thread owns 4 bins).
__device__ void prefix_hist(RowShared& S) {
  const int lane = lane_id(), wave = threadIdx.x >> 6, t = threadIdx.x;
  const uint32_t h0 = S.H[4 * t], h1 = S.H[4 * t + 1], h2 = S.H[4 * t + 2], h3 = S.H[4 * t + 3];
  const int c = (int)(h0 + h1 + h2 + h3);
  const int incl = wave_scan_incl(c);
  if (lane == 63) S.part[wave] = incl;
  __syncthreads();
  int base = 0;
#pragma unroll
  for (int k = 0; k < kWaves; ++k) base += k < wave ? S.part[k] : 0;
  const uint32_t ex = (uint32_t)(base + incl - c);
  S.H[4 * t] = ex + h0;
  S.H[4 * t + 1] = ex + h0 + h1;
  S.H[4 * t + 2] = ex + h0 + h1 + h2;
  S.H[4 * t + 3] = ex + h0 + h1 + h2 + h3;
  __syncthreads();
}

__device__ __forceinline__ void clear_hist(RowShared& S) {
  for (int b = threadIdx.x; b < kBins; b += kThreads) S.H[b] = 0;
  __syncthreads();
}

// Exact key of rank rho among key(i), i in [0, n); keys are uint32 and the
// first pass looks in [base, base + 4096).
template <class Key>
__device__ uint32_t select_rank(const Key& key, int n, uint32_t rho, uint32_t base, RowShared& S) {
  clear_hist(S);
  int below = 0;
  for (int i = threadIdx.x; i < n; i += kThreads) {
    const uint32_t k = key(i);
    const uint32_t d = k - base;
    if (d < (uint32_t)kBins) atomicAdd(&S.H[d], 1u);
    else below += k < base ? 1 : 0;
  }
  __syncthreads();
  const uint32_t B = (uint32_t)block_sum(below, S);
  if (rho >= B) {
    find_bin(S, rho - B);
    if (S.found < (uint32_t)kBins) return base + S.found;
  }
  // radix select: digits [31:20], [19:8], [7:0]
  uint32_t prefix = 0, r = rho;
#pragma unroll 1
  for (int p = 0; p < 3; ++p) {
    const int bits = p == 2 ? 8 : 12, sh = p == 0 ? 20 : (p == 1 ? 8 : 0), hi = sh + bits;
    const uint32_t dmask = (1u << bits) - 1u;
    clear_hist(S);
    for (int i = threadIdx.x; i < n; i += kThreads) {
      const uint32_t k = key(i);
      const bool match = hi >= 32 || (k >> hi) == (prefix >> hi);
      if (match) atomicAdd(&S.H[(k >> sh) & dmask], 1u);
    }
    __syncthreads();
    find_bin(S, r);
    // the rank is always inside the matching keys' histogram
    r -= S.below;
    prefix |= S.found << sh;
  }
  return prefix;
}

__global__ __launch_bounds__(kThreads) void k_row_mad(RowMadArgs a) {
  __shared__ RowShared S;
  const int row = blockIdx.x;
  const float* x = a.x + (int64_t)row * a.ld;
  const int32_t* m = a.med + (int64_t)row * a.ldm;
  const int n = a.N;
  const uint32_t rho = (uint32_t)((n - 1) / 2);
  constexpr int kHalf = kBins / 2;

  // residual histogram over [-2048, 2048), 4 consecutive samples per thread
  clear_hist(S);
  int below = 0;
  auto add = [&](int r) {
    const uint32_t b = (uint32_t)(r + kHalf);
    if (b < (uint32_t)kBins) atomicAdd(&S.H[b], 1u);
    else below += r < -kHalf ? 1 : 0;
  };
  const bool vec = (reinterpret_cast<uintptr_t>(x) & 15u) == 0;
  for (int i = 4 * (int)threadIdx.x; i < n; i += 4 * kThreads) {
    const int mk = m[i >> 6];  // the 4 samples share one 64-sample block
    if (vec && i + 3 < n) {
      const float4 v = *reinterpret_cast<const float4*>(x + i);
      add((int)v.x - mk);
      add((int)v.y - mk);
      add((int)v.z - mk);
      add((int)v.w - mk);
    } else {
      for (int q = 0; q < 4; ++q)
        if (i + q < n) add((int)x[i + q] - mk);
    }
  }
  __syncthreads();
  const uint32_t B = (uint32_t)block_sum(below, S);
  int c = 0;
  bool cwin = false;
  if (rho >= B) {
    find_bin(S, rho - B);
    cwin = S.found < (uint32_t)kBins;
    c = (int)S.found - kHalf;
  }
  uint32_t d = 0;
  bool dwin = false;
  if (cwin) {
    // smallest d with #{|r - c| <= d} > rho, over the d whose interval stays in the window
    prefix_hist(S);
    const int cb = c + kHalf, dmax = min(cb, kBins - 1 - cb);
    if (threadIdx.x == 0) S.found = kBins;
    __syncthreads();
    auto cnt = [&](int dd) { return S.H[cb + dd] - (cb - dd - 1 >= 0 ? S.H[cb - dd - 1] : 0u); };
    for (int dd = threadIdx.x; dd <= dmax; dd += kThreads)
      if (cnt(dd) > rho && (dd == 0 || cnt(dd - 1) <= rho)) S.found = (uint32_t)dd;
    __syncthreads();
    dwin = S.found < (uint32_t)kBins;
    d = S.found;
  } else {
    // residual keys: two's complement with the sign bit flipped orders as unsigned
    const uint32_t kc = select_rank([&](int i) { return (uint32_t)resid(x, m, i) ^ 0x80000000u; }, n, rho,
                                    0x80000000u - kHalf, S);
    c = (int)(kc ^ 0x80000000u);
  }
  if (!dwin)
    d = select_rank([&](int i) { const int v = resid(x, m, i) - c; return (uint32_t)(v < 0 ? -v : v); }, n, rho, 0u,
                    S);
  int32_t* out = a.mad + (int64_t)row * a.ldm;
  for (int k = threadIdx.x; k < a.nblocks; k += kThreads) out[k] = (int32_t)d;
}

}  // namespace

hipError_t launch_row_mad(const RowMadArgs& a, hipStream_t s) {
  if (a.rows <= 0 || a.N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_row_mad, dim3(a.rows), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace sps
