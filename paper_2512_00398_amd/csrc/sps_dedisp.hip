// sps_dedisp.hip - incoherent dedispersion on the device (Heimdall++,
// Section II-B, "Incoherent Dedispersion"; the DM of Eq. 1): for every trial
// d, out[d][t] = sum over channels f of fil[f][t + delay[d][f]], from an 8-bit
// channel-major filterbank to the FP32 [ndm][nsamp_out] block the search
// consumes. Exact integer sums.
//
// Design (gfx950, wave64). A workgroup of 256 threads owns 1024 output
// samples of DD consecutive trials (DD = 16 unless the trials' delays spread
// too far for the LDS staging). For each channel it stages, with aligned
// 4-byte loads, the bytes from t0 + min delay to t0 + 1024 + max delay of the
// channel row into LDS, two channels per stage (two stages: the next pair's
// loads are in flight while this pair is summed, one barrier per pair); each
// thread then takes, for every trial, the 4 bytes
// of its 4 consecutive output samples from there (two LDS words and one
// v_alignbyte, then two v_perm_b32 that place bytes 0 and 2, and bytes 1 and
// 3, in the low bytes of two 16-bit lanes) and adds them as two pairs of
// 16-bit sums, flushing the pairs into 32-bit sums every 256 channels
// (256 x 255 < 2^16). The arithmetic is one add per (trial, channel, output
// sample); the data are re-read from L2 by each trial group, so workgroups
// are ordered XCD by XCD over time tiles, all trial groups of a time tile on
// one XCD, sharing its L2.
#include <hip/hip_runtime.h>

#include "sps_internal.h"

namespace sps {
namespace {

constexpr int kDT = 1024;  // output samples per workgroup

__device__ __forceinline__ uint32_t load_word(const DedispArgs& a, int64_t w) {
  if (w < a.nfull) return a.fil32[w];
  // the last, partial word of the filterbank: bytes past its end read as 0
  const uint8_t* b = reinterpret_cast<const uint8_t*>(a.fil32);
  uint32_t v = 0;
  for (int q = 0; q < 4; ++q)
    if (4 * w + q < a.total_bytes) v |= (uint32_t)b[4 * w + q] << (8 * q);
  return v;
}

// Sums of one staged channel into the 16-bit pairs (B: this thread's view of
// the span; bf: the trials' byte offsets into it).
template <int DD>
__device__ __forceinline__ void add_channel(const uint32_t* B, const int32_t* bf, uint32_t (&lo)[DD],
                                            uint32_t (&hi)[DD]) {
#pragma unroll
  for (int j = 0; j < DD; ++j) {
    // this thread's 4 bytes start at byte 4*tid + base of the staged span;
    // v_alignbyte takes the shift from the low 2 bits of base (the same in
    // every lane), and two constant byte selectors place samples 0 and 2,
    // then 1 and 3, in the low bytes of two 16-bit lanes (0x0c gives zero)
    const int base = bf[j];
    const uint32_t x0 = B[base >> 2], x1 = B[(base >> 2) + 1];
    const uint32_t v = __builtin_amdgcn_alignbyte(x1, x0, (uint32_t)base);
    lo[j] += __builtin_amdgcn_perm(0u, v, 0x0c020c00u);  // samples 0 and 2
    hi[j] += __builtin_amdgcn_perm(0u, v, 0x0c030c01u);  // samples 1 and 3
  }
}

template <int DD>
__global__ __launch_bounds__(256) void k_dedisp(DedispArgs a) {
  // Channels go in pairs: one stage holds two channel spans; stage s is
  // summed from one buffer while stage s+1 is written to the other, one
  // barrier per two channels.
  __shared__ uint32_t buf[2][2][kDedispSpanWords];
  // XCD-aware order: block b runs on XCD b % 8; give each XCD a contiguous
  // range of tiles, trial groups fastest, so one time tile stays on one XCD
  const int b = blockIdx.x;
  const int tile = (b & 7) * a.per_xcd + (b >> 3);
  if (tile >= a.ntiles) return;  // whole workgroup leaves; no barrier passed yet
  const int dg = tile % a.ngroups, tt = tile / a.ngroups;
  const int t0 = tt * kDT, d0 = dg * DD;
  const int tid = threadIdx.x;
  // spans and offsets were laid out on the host (t0 is a multiple of 4, so a
  // tile only moves the span by whole words): the channel loop reads them
  // with scalar loads and does no delay arithmetic
  const DedispSpan* sp = a.span + dg;
  const int32_t* bs = a.base + d0;
  const int64_t tw = t0 >> 2;
  const int nchan = a.nchan;

  uint32_t lo[DD], hi[DD], acc[DD][4];
#pragma unroll
  for (int j = 0; j < DD; ++j) {
    lo[j] = hi[j] = 0u;
    acc[j][0] = acc[j][1] = acc[j][2] = acc[j][3] = 0u;
  }
  // stage 0: channels 0 and 1 (if any)
  for (int c = 0; c < 2 && c < nchan; ++c) {
    const DedispSpan s0 = sp[(int64_t)c * a.ngroups];
    for (int k = tid; k < s0.nw; k += 256) buf[0][c][k] = load_word(a, s0.w0 + tw + k);
  }
  __syncthreads();
  for (int f = 0; f < nchan; f += 2) {
    const int pb = (f >> 1) & 1;
    const bool two = f + 1 < nchan;
    // next stage's spans: the first two words per thread of each are loaded
    // now and stored after this stage's sums, so the loads overlap them
    const bool m0 = f + 2 < nchan, m1 = f + 3 < nchan;
    const DedispSpan n0 = sp[(int64_t)(m0 ? f + 2 : f) * a.ngroups];
    const DedispSpan n1 = sp[(int64_t)(m1 ? f + 3 : f) * a.ngroups];
    const int nw0 = m0 ? n0.nw : 0, nw1 = m1 ? n1.nw : 0;
    const int64_t w0 = n0.w0 + tw, w1 = n1.w0 + tw;
    const uint32_t q00 = tid < nw0 ? load_word(a, w0 + tid) : 0u;
    const uint32_t q01 = tid + 256 < nw0 ? load_word(a, w0 + tid + 256) : 0u;
    const uint32_t q10 = tid < nw1 ? load_word(a, w1 + tid) : 0u;
    const uint32_t q11 = tid + 256 < nw1 ? load_word(a, w1 + tid + 256) : 0u;
    add_channel<DD>(buf[pb][0] + tid, bs + (int64_t)f * a.ndm_pad, lo, hi);
    if (two) add_channel<DD>(buf[pb][1] + tid, bs + (int64_t)(f + 1) * a.ndm_pad, lo, hi);
    // 256 is even: a flush point (every 256 channels) always ends a pair
    if (((f + 1) & 255) == 255 || f + 2 >= nchan) {
#pragma unroll
      for (int j = 0; j < DD; ++j) {
        acc[j][0] += lo[j] & 0xFFFFu;
        acc[j][2] += lo[j] >> 16;
        acc[j][1] += hi[j] & 0xFFFFu;
        acc[j][3] += hi[j] >> 16;
        lo[j] = hi[j] = 0u;
      }
    }
    uint32_t* N0 = buf[pb ^ 1][0];
    uint32_t* N1 = buf[pb ^ 1][1];
    if (tid < nw0) N0[tid] = q00;
    if (tid + 256 < nw0) N0[tid + 256] = q01;
    if (tid < nw1) N1[tid] = q10;
    if (tid + 256 < nw1) N1[tid + 256] = q11;
    for (int k = tid + 512; k < nw0; k += 256) N0[k] = load_word(a, w0 + k);  // wide spreads only
    for (int k = tid + 512; k < nw1; k += 256) N1[k] = load_word(a, w1 + k);
    __syncthreads();
  }
  const int t = t0 + 4 * tid;
#pragma unroll
  for (int j = 0; j < DD; ++j) {
    const int d = d0 + j;
    if (d >= a.ndm) break;
    float* o = a.out + (int64_t)d * a.nsamp_out;
    if (t + 3 < a.nsamp_out && ((reinterpret_cast<uintptr_t>(o + t) & 15u) == 0)) {
      *reinterpret_cast<float4*>(o + t) = make_float4((float)acc[j][0], (float)acc[j][1], (float)acc[j][2],
                                                      (float)acc[j][3]);
    } else {
      for (int q = 0; q < 4; ++q)
        if (t + q < a.nsamp_out) o[t + q] = (float)acc[j][q];
    }
  }
}

}  // namespace

hipError_t launch_dedisp(const DedispArgs& a, hipStream_t s) {
  if (a.ntiles <= 0) return hipSuccess;
  const dim3 g(8 * a.per_xcd), b(256);
  switch (a.dd) {
    case 16: hipLaunchKernelGGL(k_dedisp<16>, g, b, 0, s, a); break;
    case 8: hipLaunchKernelGGL(k_dedisp<8>, g, b, 0, s, a); break;
    case 4: hipLaunchKernelGGL(k_dedisp<4>, g, b, 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_dedisp<2>, g, b, 0, s, a); break;
    case 1: hipLaunchKernelGGL(k_dedisp<1>, g, b, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace sps
