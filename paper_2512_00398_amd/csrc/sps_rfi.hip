// sps_rfi.hip - broadband (zero-DM) RFI excision (Heimdall++, Section II-B,
// "RFI Mitigation"): interference present in every channel at once is
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

}  // namespace

hipError_t launch_zero_dm(const ZeroDmArgs& a, hipStream_t s) {
  if (a.nsamp <= 0 || a.nchan <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_dm, dim3((unsigned)((a.nsamp + kZdSpan - 1) / kZdSpan)), dim3(64 * kZdWaves), 0, s, a);
  return hipGetLastError();
}

}  // namespace sps
