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
// l of every wave owns samples 4l .. 4l+3 of that range (256 contiguous bytes
// per wave and channel), and the 16 waves split the channels (wave w takes
// f = w, w+16, ...), so many rows' loads are in flight at once. Rows of an
// odd length start anywhere in a 4-byte word, so every access is made on
// aligned words: a lane's 4 bytes are one or two aligned loads and a
// v_alignbyte, and the rewrite stores whole aligned words, byte stores only
// for the one or two words at the ends of a row's stretch. Partial sums meet
// in LDS, one wave forms the levels, then each wave rewrites its own
// channels. Traffic: the filterbank read twice (the second read mostly from
// L2) and written once.
#include <hip/hip_runtime.h>

#include "sps_internal.h"

namespace sps {
namespace {

constexpr int kZdWaves = 16;
constexpr int kZdSpan = 256;  // samples per workgroup: 4 per lane

__device__ __forceinline__ uint32_t clamp8(int v) { return (uint32_t)min(255, max(0, v)); }

// n (1..4) bytes from p, in the low bytes (higher bytes undefined), read as
// the aligned 4-byte words that hold them: rows of an odd length start
// anywhere in a word. The second word is read only when one of the n bytes
// lies in it, so every word read holds a wanted byte (same page: no read
// leaves mapped memory).
__device__ __forceinline__ uint32_t load4(const uint8_t* p, int n) {
  const uintptr_t ap = reinterpret_cast<uintptr_t>(p);
  const uint32_t il = (uint32_t)(ap & 3u);
  const uint32_t* w = reinterpret_cast<const uint32_t*>(ap - il);
  const uint32_t lo = w[0];
  if (il == 0u) return lo;
  const uint32_t hi = (int)il + n > 4 ? w[1] : 0u;
  return __builtin_amdgcn_alignbyte(hi, lo, il);
}

__global__ __launch_bounds__(64 * kZdWaves) void k_zero_dm(ZeroDmArgs a) {
  __shared__ uint32_t part[kZdWaves][64][4];
  __shared__ int zs[kZdSpan];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t t0 = (int64_t)blockIdx.x * kZdSpan;
  const int tv = (int)min<int64_t>(kZdSpan, a.nsamp - t0);  // samples of this tile
  const int tl = 4 * lane;                                  // this lane's first sample in the tile
  const int n = max(0, min(4, tv - tl));
  const uint32_t keep = n >= 4 ? 0xFFFFFFFFu : ((1u << (8 * n)) - 1u);
  uint32_t s0 = 0, s1 = 0, s2 = 0, s3 = 0;
#pragma unroll 4
  for (int f = wave; f < a.nchan; f += kZdWaves) {
    if (n > 0) {
      const uint32_t w = load4(a.in + (int64_t)f * a.nsamp + t0 + tl, n) & keep;
      s0 += w & 0xFFu;
      s1 += (w >> 8) & 0xFFu;
      s2 += (w >> 16) & 0xFFu;
      s3 += w >> 24;
    }
  }
  part[wave][lane][0] = s0;
  part[wave][lane][1] = s1;
  part[wave][lane][2] = s2;
  part[wave][lane][3] = s3;
  __syncthreads();
  // sums < 255 * 65536 < 2^24: the level fits 32-bit arithmetic
  if (wave == 0) {
    const uint32_t c = (uint32_t)a.nchan;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      uint32_t sum = 0;
#pragma unroll
      for (int w = 0; w < kZdWaves; ++w) sum += part[w][lane][q];
      zs[tl + q] = (int)((2u * sum + c) / (2u * c)) - a.offset;
    }
  }
  __syncthreads();
  // Rewrite, one row at a time: the aligned output words over the tile's
  // bytes. Word k holds tile bytes 4k - lead .. 4k - lead + 3; words wholly
  // inside the tile are read (aligned, realigned) and stored whole, the one
  // or two at its ends byte by byte, only the tile's own bytes.
  for (int f = wave; f < a.nchan; f += kZdWaves) {
    const int64_t row = (int64_t)f * a.nsamp + t0;
    const int lead = (int)((reinterpret_cast<uintptr_t>(a.out + row)) & 3u);
    for (int k = lane; k <= kZdSpan / 4; k += 64) {
      const int j0 = 4 * k - lead;
      if (j0 >= tv || j0 + 4 <= 0) continue;
      if (j0 >= 0 && j0 + 4 <= tv) {
        const uint32_t v = load4(a.in + row + j0, 4);
        const uint32_t o = clamp8((int)(v & 0xFFu) - zs[j0]) | (clamp8((int)((v >> 8) & 0xFFu) - zs[j0 + 1]) << 8) |
                           (clamp8((int)((v >> 16) & 0xFFu) - zs[j0 + 2]) << 16) |
                           (clamp8((int)(v >> 24) - zs[j0 + 3]) << 24);
        *reinterpret_cast<uint32_t*>(a.out + row + j0) = o;
      } else {
        for (int q = 0; q < 4; ++q) {
          const int j = j0 + q;
          if (j >= 0 && j < tv) a.out[row + j] = (uint8_t)clamp8((int)a.in[row + j] - zs[j]);
        }
      }
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
  // The row read as the aligned 4-byte words that cover it, whatever its
  // alignment (rows of an odd length start anywhere in a word): bytes of a
  // word outside the row are skipped. A word holding one byte of the row
  // lies in the same page as that byte, so the reads stay in mapped memory.
  const uintptr_t start = reinterpret_cast<uintptr_t>(a.in + (int64_t)f * a.nsamp);
  const int lead = (int)(start & 3u);
  const uint32_t* words = reinterpret_cast<const uint32_t*>(start - (uintptr_t)lead);
  const int64_t nw = (lead + a.nsamp + 3) >> 2;
  const int64_t last = lead + a.nsamp;  // one past the row's last byte, in word-byte units
  for (int64_t k = tid; k < nw; k += 256) {
    const uint32_t w = words[k];
    const int64_t b0 = 4 * k;
    if (b0 >= lead && b0 + 4 <= last) {
      atomicAdd(&h[wave][w & 0xFFu], 1u);
      atomicAdd(&h[wave][(w >> 8) & 0xFFu], 1u);
      atomicAdd(&h[wave][(w >> 16) & 0xFFu], 1u);
      atomicAdd(&h[wave][w >> 24], 1u);
    } else {
      for (int q = 0; q < 4; ++q)
        if (b0 + q >= lead && b0 + q < last) atomicAdd(&h[wave][(w >> (8 * q)) & 0xFFu], 1u);
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

// Flagged channels take their median; the others are copied (nothing to do
// in place). Thread k writes the row's aligned output word k (the row read
// as aligned words too, realigned); the one or two words at the row's ends
// are written byte by byte, only the row's own bytes.
__global__ __launch_bounds__(256) void k_chan_apply(ChanMaskArgs a) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  for (int f = blockIdx.y; f < a.nchan; f += gridDim.y) {
    const bool flag = a.stats[3 * (int64_t)f + 2] != 0;
    if (!flag && a.in == a.out) continue;
    const int64_t row = (int64_t)f * a.nsamp;
    const int lead = (int)((reinterpret_cast<uintptr_t>(a.out + row)) & 3u);
    const int64_t j0 = 4 * k - lead;
    if (j0 >= a.nsamp || j0 + 4 <= 0) continue;
    const uint8_t mu = a.stats[3 * (int64_t)f];
    if (j0 >= 0 && j0 + 4 <= a.nsamp) {
      const uint32_t v = flag ? 0x01010101u * mu : load4(a.in + row + j0, 4);
      *reinterpret_cast<uint32_t*>(a.out + row + j0) = v;
    } else {
      for (int q = 0; q < 4; ++q) {
        const int64_t j = j0 + q;
        if (j >= 0 && j < a.nsamp) a.out[row + j] = flag ? mu : a.in[row + j];
      }
    }
  }
}

}  // namespace

hipError_t launch_chan_mask(const ChanMaskArgs& a, hipStream_t s) {
  if (a.nsamp <= 0 || a.nchan <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_chan_stats, dim3((unsigned)a.nchan), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_chan_flags, dim3(1), dim3(256), 0, s, a);
  const unsigned gx = (unsigned)((a.nsamp / 4 + 2 + 255) / 256), gy = (unsigned)min(a.nchan, 65535);
  hipLaunchKernelGGL(k_chan_apply, dim3(gx, gy), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_zero_dm(const ZeroDmArgs& a, hipStream_t s) {
  if (a.nsamp <= 0 || a.nchan <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_dm, dim3((unsigned)((a.nsamp + kZdSpan - 1) / kZdSpan)), dim3(64 * kZdWaves), 0, s, a);
  return hipGetLastError();
}

}  // namespace sps
