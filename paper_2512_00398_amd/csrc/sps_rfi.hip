// sps_rfi.hip - RFI excision (Heimdall++, Section II-B, "RFI Mitigation").
// Narrowband: channels whose lower MAD over the chunk exceeds the median of
// the channels' MADs by k MADs of those MADs are replaced by their median
// (exact byte order statistics from 256-bin histograms).
// Broadband (zero-DM): interference present in every channel at once is
// undispersed; each time sample's level across the band,
// z_t = floor((2 * sum_f I[f][t] + nchan) / (2 * nchan)) (the channel mean
// rounded half up), is subtracted from every channel and the caller's offset
// added, clamped to [0, 255]. Exact integer arithmetic.
//
// Design (gfx950, wave64): a workgroup covers 256 consecutive samples; lane
// l of every wave owns samples 4l .. 4l+3 of that range (one 4-byte word per
// channel row, 256 contiguous bytes per wave and channel), and the 16 waves
// split the channels (wave w takes f = w, w+16, ...), so many rows' loads are
// in flight at once. Partial sums meet in LDS, every wave forms the same
// levels, then each wave rewrites its own channels. Traffic: the filterbank read twice (the second read mostly from
// L2) and written once.
#include <hip/hip_runtime.h>

#include "sps_internal.h"

namespace sps {
namespace {

constexpr int kZdWaves = 16;
constexpr int kZdSpan = 256;  // samples per workgroup: 4 per lane

__device__ __forceinline__ uint32_t clamp8(int v) { return (uint32_t)min(255, max(0, v)); }

__global__ __launch_bounds__(64 * kZdWaves) void k_zero_dm(ZeroDmArgs a) {
  __shared__ uint32_t part[kZdWaves][64][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t t = (int64_t)blockIdx.x * kZdSpan + 4 * lane;  // first of this lane's samples
  const int n = t < a.nsamp ? (int)min<int64_t>(4, a.nsamp - t) : 0;
  const bool word = a.aligned4 && n == 4;
  uint32_t s0 = 0, s1 = 0, s2 = 0, s3 = 0;
#pragma unroll 4
  for (int f = wave; f < a.nchan; f += kZdWaves) {
    const uint8_t* p = a.in + (int64_t)f * a.nsamp + t;
    if (word) {
      const uint32_t w = *reinterpret_cast<const uint32_t*>(p);
      s0 += w & 0xFFu;
      s1 += (w >> 8) & 0xFFu;
      s2 += (w >> 16) & 0xFFu;
      s3 += w >> 24;
    } else if (n > 0) {
      s0 += p[0];
      if (n > 1) s1 += p[1];
      if (n > 2) s2 += p[2];
      if (n > 3) s3 += p[3];
    }
  }
  part[wave][lane][0] = s0;
  part[wave][lane][1] = s1;
  part[wave][lane][2] = s2;
  part[wave][lane][3] = s3;
  __syncthreads();
  // sums < 255 * 65536 < 2^24: the level fits 32-bit arithmetic
  const uint32_t c = (uint32_t)a.nchan;
  int z[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    uint32_t sum = 0;
#pragma unroll
    for (int w = 0; w < kZdWaves; ++w) sum += part[w][lane][q];
    z[q] = (int)((2u * sum + c) / (2u * c)) - a.offset;
  }
#pragma unroll 4
  for (int f = wave; f < a.nchan; f += kZdWaves) {
    const int64_t at = (int64_t)f * a.nsamp + t;
    if (word) {
      const uint32_t w = *reinterpret_cast<const uint32_t*>(a.in + at);
      const uint32_t o = clamp8((int)(w & 0xFFu) - z[0]) | (clamp8((int)((w >> 8) & 0xFFu) - z[1]) << 8) |
                         (clamp8((int)((w >> 16) & 0xFFu) - z[2]) << 16) | (clamp8((int)(w >> 24) - z[3]) << 24);
      *reinterpret_cast<uint32_t*>(a.out + at) = o;
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (q < n) a.out[at + q] = (uint8_t)clamp8((int)a.in[at + q] - z[q]);
    }
  }
}

// ---- narrowband: per-channel statistics, flags, replacement -----------------
// Exact order statistics of bytes from a 256-bin histogram H with n values:
// the lower median (rank (n-1)/2) and the lower MAD about it, found by
// widening [mu - D, mu + D] until it holds more than the rank.
__device__ void hist_median_mad(const uint32_t* H, uint32_t n, int& mu, int& mad) {
  const uint32_t r = (n - 1) / 2;
  uint32_t acc = 0;
  int m = 0;
  for (; m < 256; ++m) {
    acc += H[m];
    if (acc > r) break;
  }
  uint32_t cnt = H[m];
  int d = 0;
  while (cnt <= r) {
    ++d;
    if (m - d >= 0) cnt += H[m - d];
    if (m + d <= 255) cnt += H[m + d];
  }
  mu = m;
  mad = d;
}

// One workgroup per channel: byte histogram of the row (one sub-histogram
// per wave against same-bin contention), then its median and MAD.
__global__ __launch_bounds__(256) void k_chan_stats(ChanMaskArgs a) {
  __shared__ uint32_t h[4][256];
  const int tid = threadIdx.x, wave = tid >> 6;
  const int f = blockIdx.x;
  for (int b = tid; b < 4 * 256; b += 256) (&h[0][0])[b] = 0;
  __syncthreads();
  const uint8_t* row = a.in + (int64_t)f * a.nsamp;
  for (int64_t i = 4 * (int64_t)tid; i < a.nsamp; i += 1024) {
    if (a.aligned4 && i + 3 < a.nsamp) {
      const uint32_t w = *reinterpret_cast<const uint32_t*>(row + i);
      atomicAdd(&h[wave][w & 0xFFu], 1u);
      atomicAdd(&h[wave][(w >> 8) & 0xFFu], 1u);
      atomicAdd(&h[wave][(w >> 16) & 0xFFu], 1u);
      atomicAdd(&h[wave][w >> 24], 1u);
    } else {
      for (int q = 0; q < 4; ++q)
        if (i + q < a.nsamp) atomicAdd(&h[wave][row[i + q]], 1u);
    }
  }
  __syncthreads();
  h[0][tid] += h[1][tid] + h[2][tid] + h[3][tid];
  __syncthreads();
  if (tid == 0) {
    int mu, mad;
    hist_median_mad(h[0], (uint32_t)a.nsamp, mu, mad);
    a.stats[3 * (int64_t)f] = (uint8_t)mu;
    a.stats[3 * (int64_t)f + 1] = (uint8_t)mad;
  }
}

// One workgroup: median M and MAD S of the channels' MADs (bytes again),
// then the flags sigma_f > M + k * S.
__global__ __launch_bounds__(256) void k_chan_flags(ChanMaskArgs a) {
  __shared__ uint32_t h[256];
  __shared__ int ms[2];
  const int tid = threadIdx.x;
  h[tid] = 0;
  __syncthreads();
  for (int f = tid; f < a.nchan; f += 256) atomicAdd(&h[a.stats[3 * (int64_t)f + 1]], 1u);
  __syncthreads();
  if (tid == 0) hist_median_mad(h, (uint32_t)a.nchan, ms[0], ms[1]);
  __syncthreads();
  const int64_t lim = (int64_t)ms[0] + (int64_t)a.k * ms[1];
  for (int f = tid; f < a.nchan; f += 256) a.stats[3 * (int64_t)f + 2] = (int64_t)a.stats[3 * (int64_t)f + 1] > lim;
}

// Flagged channels take their median; the others are copied (nothing to do in place).
__global__ __launch_bounds__(256) void k_chan_apply(ChanMaskArgs a) {
  const int64_t i = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
  if (i >= a.nsamp) return;
  for (int f = blockIdx.y; f < a.nchan; f += gridDim.y) {
    const bool flag = a.stats[3 * (int64_t)f + 2] != 0;
    if (!flag && a.in == a.out) continue;
    const int64_t at = (int64_t)f * a.nsamp + i;
    const uint8_t mu = a.stats[3 * (int64_t)f];
    if (a.aligned4 && i + 3 < a.nsamp) {
      const uint32_t v = flag ? 0x01010101u * mu : *reinterpret_cast<const uint32_t*>(a.in + at);
      *reinterpret_cast<uint32_t*>(a.out + at) = v;
    } else {
      for (int q = 0; q < 4; ++q)
        if (i + q < a.nsamp) a.out[at + q] = flag ? mu : a.in[at + q];
    }
  }
}

}  // namespace

hipError_t launch_chan_mask(const ChanMaskArgs& a, hipStream_t s) {
  if (a.nsamp <= 0 || a.nchan <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_chan_stats, dim3((unsigned)a.nchan), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_chan_flags, dim3(1), dim3(256), 0, s, a);
  const unsigned gx = (unsigned)((a.nsamp + 1023) / 1024), gy = (unsigned)min(a.nchan, 65535);
  hipLaunchKernelGGL(k_chan_apply, dim3(gx, gy), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_zero_dm(const ZeroDmArgs& a, hipStream_t s) {
  if (a.nsamp <= 0 || a.nchan <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_dm, dim3((unsigned)((a.nsamp + kZdSpan - 1) / kZdSpan)), dim3(64 * kZdWaves), 0, s, a);
  return hipGetLastError();
}

}  // namespace sps
