// sps_rownorm.hip - one noise scale per DM row (Heimdall++, Section II-B's
// normalisation, read as one scale per trial and chunk): with the block
// medians m_k already computed, the residual r_t = x_t - m_{floor(t/64)} of
// the whole row is formed on the fly, c = its lower median and
// MAD_row = the lower median of |r_t - c|; every block of the row then takes
// MAD_row as its scale. Exact integer order statistics.
//
// One 1024-thread workgroup per row. Each order statistic is an exact select
// of rank (N-1)/2: a first pass histograms a 4096-value window in LDS (around
// 0 for the residual, from 0 for the deviations, where these statistics sit
// for any baseline-removed row) and counts the values below it; if the rank
// falls inside, a block scan of the histogram gives the answer. Otherwise a
// radix select (digits of 12, 12 and 8 bits, most significant first) over
// the same keys finds it. Each pass reads the row once, coalesced; HBM
// traffic is 2 x 4 B per sample in the common case.
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
  const int32_t* m = a.med + (int64_t)row * a.nblocks;
  const int n = a.N;
  const uint32_t rho = (uint32_t)((n - 1) / 2);
  // residual keys: two's complement with the sign bit flipped orders as unsigned
  const uint32_t kc = select_rank([&](int i) { return (uint32_t)resid(x, m, i) ^ 0x80000000u; }, n, rho,
                                  0x80000000u - kBins / 2, S);
  const int c = (int)(kc ^ 0x80000000u);
  const uint32_t d = select_rank([&](int i) { const int v = resid(x, m, i) - c; return (uint32_t)(v < 0 ? -v : v); },
                                 n, rho, 0u, S);
  int32_t* out = a.mad + (int64_t)row * a.nblocks;
  for (int k = threadIdx.x; k < a.nblocks; k += kThreads) out[k] = (int32_t)d;
}

}  // namespace

hipError_t launch_row_mad(const RowMadArgs& a, hipStream_t s) {
  if (a.rows <= 0 || a.N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_row_mad, dim3(a.rows), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace sps
