// sps_plain.hip - the search as plain per-stage kernels (the comparison path).
//
// The same arithmetic as the fused path, run the way the DM-trial loop of
// Heimdall (Section II-B) stages it: one kernel per stage and per boxcar
// width, every intermediate materialised in device memory and re-read by the
// next stage. Only the launch granularity differs from the paper's loop: each
// launch covers all DM rows at once. Stages: baseline/normalisation
// (k_block_stats, shared with the fused path) -> residual -> prefix sum ->
// per width: boxcar -> threshold -> peaks per strip -> stitch strips.
#include "sps_internal.h"
#include "sps_runs.h"
#include "sps_wave.h"

namespace sps {

namespace {

// r[row][t] = x - m_{t/64}
__global__ __launch_bounds__(256) void k_plain_residual(PlainArgs A) {
  const int row = blockIdx.y;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= A.N) return;
  const float* xr = A.x + (int64_t)row * A.N;
  A.r[(int64_t)row * A.N + t] = (int)xr[t] - A.med[(int64_t)row * A.nblocks + (t >> 6)];
}

// P[row][0] = 0, P[row][t + 1] = P[row][t] + r[row][t] (uint32, wrapping);
// one workgroup per row walks it in chunks of 1024.
__global__ __launch_bounds__(256) void k_plain_prefix(PlainArgs A) {
  __shared__ uint32_t wt[4];
  const int row = blockIdx.x;
  const int tid = threadIdx.x, wave = tid >> 6, lane = lane_id();
  const int32_t* rr = A.r + (int64_t)row * A.N;
  uint32_t* pr = A.P + (int64_t)row * (A.N + 1);
  if (tid == 0) pr[0] = 0u;
  uint32_t carry = 0;
  for (int c0 = 0; c0 < A.N; c0 += 1024) {
    const int t = c0 + 4 * tid;
    const uint32_t v0 = t < A.N ? (uint32_t)rr[t] : 0u;
    const uint32_t v1 = t + 1 < A.N ? (uint32_t)rr[t + 1] : 0u;
    const uint32_t v2 = t + 2 < A.N ? (uint32_t)rr[t + 2] : 0u;
    const uint32_t v3 = t + 3 < A.N ? (uint32_t)rr[t + 3] : 0u;
    const uint32_t q0 = v0, q1 = q0 + v1, q2 = q1 + v2, q3 = q2 + v3;
    const uint32_t inc = (uint32_t)wave_scan_incl((int)q3);
    if (lane == 63) wt[wave] = inc;
    __syncthreads();
    uint32_t off = carry;
    for (int v = 0; v < wave; ++v) off += wt[v];
    const uint32_t tot = wt[0] + wt[1] + wt[2] + wt[3];
    const uint32_t base = off + inc - q3;
    if (t < A.N) pr[t + 1] = base + q0;
    if (t + 1 < A.N) pr[t + 2] = base + q1;
    if (t + 2 < A.N) pr[t + 3] = base + q2;
    if (t + 3 < A.N) pr[t + 4] = base + q3;
    carry += tot;
    __syncthreads();
  }
}

// S[row][i] = P[i + w] - P[i], i = 0 .. N - w
__global__ __launch_bounds__(256) void k_plain_boxcar(PlainArgs A) {
  const int row = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > A.N - A.w) return;
  const uint32_t* pr = A.P + (int64_t)row * (A.N + 1);
  A.S[(int64_t)row * A.N + i] = (int)(pr[i + A.w] - pr[i]);
}

// flag[row][i] = S/N of position i at width w above the threshold
__global__ __launch_bounds__(256) void k_plain_threshold(PlainArgs A) {
  const int row = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > A.N - A.w) return;
  const int mad = A.mad[(int64_t)row * A.nblocks + ((i + (A.w >> 1)) >> 6)];
  const Bound b = make_bound(mad, A.sqrtw, A.theta);
  A.flag[(int64_t)row * A.N + i] = above(A.S[(int64_t)row * A.N + i], b, A.theta) ? 1 : 0;
}

__device__ __forceinline__ double wave_max_f64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// One wave per strip of positions, 64 at a time: the group's threshold
// decisions come from memory, each run's best position is the first lane
// holding the run's largest double S/N. Runs inside the strip are emitted;
// runs touching its ends are summarised for the stitch kernel.
__global__ __launch_bounds__(256) void k_plain_peaks(PlainArgs A) {
  const int row = blockIdx.y;
  const int lane = lane_id();
  const int s = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (s >= A.nstrip) return;  // whole wave
  const int npos = A.N - A.w + 1;
  const int i0 = s * A.strip, i1 = min(npos, i0 + A.strip);
  const Emitter em{nullptr, nullptr, A.cands, A.ncand, A.cap, (uint32_t)row, (uint32_t)A.w, lane == 0, 0};
  const int32_t* Sr = A.S + (int64_t)row * A.N;
  const uint8_t* fr = A.flag + (int64_t)row * A.N;
  const int32_t* mr = A.mad + (int64_t)row * A.nblocks;
  RunSum acc = rs_empty();
  for (int g = i0; g < i1; g += 64) {
    const int i = g + lane;
    const bool valid = i < i1;
    const bool f = valid && fr[i] != 0;
    const uint64_t V = ballot(valid), M = ballot(f);
    RunSum gs = rs_empty();
    gs.flags = kNonEmpty;
    if (M) {
      const int S = f ? Sr[i] : 0;
      const double d = f ? (kMadToSigma * (double)mr[(i + (A.w >> 1)) >> 6]) * A.sqrtw : 1.0;
      const double key = f ? (double)S / d : -1.0;
      const int fv = ctz(V), lv = msb(V);
      uint64_t m = M;
      while (m) {
        const int a0 = ctz(m);
        const uint64_t gap = ~m & (~0ull << a0);
        const int b0 = gap ? ctz(gap) : 64;
        const uint64_t run = (b0 == 64 ? ~0ull : ((1ull << b0) - 1ull)) & (~0ull << a0);
        const bool in = (run >> lane) & 1ull;
        const double km = wave_max_f64(in ? key : -1.0);
        const int j = ctz(ballot(in && key == km));
        const double bq = km;  // the run's best S/N, S / den at lane j
        if (a0 == fv && b0 - 1 == lv) { gs.flags |= kFull | kHead; gs.hi = g + j; gs.hq = bq; }
        else if (a0 == fv) { gs.flags |= kHead; gs.hi = g + j; gs.hq = bq; }
        else if (b0 - 1 == lv) { gs.flags |= kTail; gs.ti = g + j; gs.tq = bq; }
        else emit(em, g + j, bq);
        m &= ~run;
      }
    }
    acc = rs_combine(acc, gs, em);
  }
  if (lane == 0) A.frag[(int64_t)row * A.nstrip + s] = acc;
}

// One thread per row: stitch the strips in order; runs at the row ends close.
__global__ __launch_bounds__(256) void k_plain_stitch(PlainArgs A) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= A.rows) return;
  const Emitter em{nullptr, nullptr, A.cands, A.ncand, A.cap, (uint32_t)row, (uint32_t)A.w, true, 0};
  RunSum acc = rs_empty();
  for (int s = 0; s < A.nstrip; ++s) acc = rs_combine(acc, A.frag[(int64_t)row * A.nstrip + s], em);
  rs_close(acc, em);
}

}  // namespace

hipError_t launch_plain_width(const PlainArgs& a, hipStream_t s) {
  const int npos = a.N - a.w + 1;
  if (npos <= 0 || a.rows <= 0) return hipSuccess;
  const dim3 g((npos + 255) / 256, a.rows), b(256);
  hipLaunchKernelGGL(k_plain_boxcar, g, b, 0, s, a);
  hipLaunchKernelGGL(k_plain_threshold, g, b, 0, s, a);
  hipLaunchKernelGGL(k_plain_peaks, dim3((a.nstrip + 3) / 4, a.rows), b, 0, s, a);
  hipLaunchKernelGGL(k_plain_stitch, dim3((a.rows + 255) / 256), b, 0, s, a);
  return hipGetLastError();
}

hipError_t launch_plain_prepare(const PlainArgs& a, hipStream_t s) {
  if (a.rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_plain_residual, dim3((a.N + 255) / 256, a.rows), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_plain_prefix, dim3(a.rows), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace sps
