// sps_detect.hip - matched filtering and peak detection stages (Heimdall++,
// Section II-B), fused: residuals, boxcar sums at every power-of-two width,
// the S/N threshold and run-based peak picking in one pass over the block.
//
// Arithmetic (exact): r_t = x_t - m_{t/64}; prefix P[E] = sum of r over the
// first E samples of the segment (uint32, wrapping; differences are exact
// while |S| < 2^31); S_w(i) = P[E] - P[E - w] with E = i - s0 + w. The S/N
// test "S / den > theta", den = (K * MAD_{k*}) * sqrt(w), is decided by
// integer bounds lo < S < hi per (centre block, width) and, inside that
// 3-integer band only, by the IEEE double division itself. Within one centre
// block S/N is strictly increasing in S, so the best of a run inside a group
// is found on S; each group best is then divided once, and bests are compared
// across groups, steps and segments on those exact double S/N values.
//
// Layout (gfx950, wave64). One 256-thread workgroup streams one segment of a
// row in steps of 1024 samples: coalesced float4 loads, residuals, a
// workgroup scan into an 8192-entry LDS ring of P (max_width of history).
// For width w the step's positions are grouped 64 per (wave, q) so that each
// group shares one centre block k* (window ends E with E - ceil(w/2) = 0 mod
// 64): the group's bound is one scalar. Fast pass: per lane and width two LDS
// reads, a subtract and a compare folded into a ballot; groups whose every
// position is above for sure are summarised there. Widths with any other
// position beyond the bound take the run pass: per group a DPP max-reduction
// and a packed summary in LDS, then a segmented max-scan over the 16 groups
// of each flagged width in one DPP row, folded into the carried run
// summaries that stitch runs across steps and, through the fix-up kernel,
// segments.
// Candidates are staged in LDS and flushed with one global atomic per step.
#include "sps_detect_body.h"

namespace sps {

namespace {

template <int NW, bool VIRT>
__global__ __launch_bounds__(256) void k_detect(DetectArgs A) {
  detect_body<NW, VIRT>(A, blockIdx.x);
}

// Persistent form over a batch of blocks: workgroups take (item, segment)
// tasks from a queue (items ordered by segment length, longest first) until
// none is left; every workgroup leaves once the counter passes the total.
// Four waves per SIMD (at most 128 VGPRs): reading each item's arguments from
// memory costs registers, and the kernel is faster at this occupancy even
// with the two spilled registers it takes.
template <int NW, bool VIRT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_detect_batch(BatchDetect B) {
  __shared__ int s_task;
  while (true) {
    if (threadIdx.x == 0) s_task = (int)atomicAdd(B.counter, 1u);
    __syncthreads();
    const int task = __builtin_amdgcn_readfirstlane(s_task);
    __syncthreads();
    if (task >= B.total) break;
    int it = 0;
    while (it + 1 < B.nitems && B.offs[it + 1] <= task) ++it;
    detect_body<NW, VIRT>(B.items[it], task - B.offs[it]);
    __syncthreads();
  }
}

// Stitch the segment summaries of each (row, width) in order.
__device__ __forceinline__ void fixup_one(const DetectArgs& A, const int t) {
  const int row = t / A.nw, j = t - row * A.nw;
  const Emitter em{nullptr, nullptr, A.cands, A.ncand, A.cap, (uint32_t)row + A.row_offset, (uint32_t)(1 << j),
                   true, A.sample_offset};
  const RunSum* f = A.frag + (int64_t)t * A.nseg;
  RunSum acc = rs_empty();
  for (int s = 0; s < A.nseg; ++s) acc = rs_combine(acc, f[s], em);
  rs_close(acc, em);
}

__global__ __launch_bounds__(256) void k_fixup(DetectArgs A) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= A.rows * A.nw) return;
  fixup_one(A, t);
}

// Batch: thread t -> (item, row, width); items with one segment per row
// contribute no threads (their runs were closed by the detect kernel).
__global__ __launch_bounds__(256) void k_fixup_batch(BatchDetect B, const int32_t* offs) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= offs[B.nitems]) return;
  int lo = 0, hi = B.nitems - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (offs[mid] <= t) lo = mid; else hi = mid - 1;
  }
  fixup_one(B.items[lo], t - offs[lo]);
}

// Batch prologue: zero every item's candidate counter and both queue heads.
__global__ __launch_bounds__(256) void k_batch_zero(uint32_t* const* ncand, int n, uint32_t* counters) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) *ncand[t] = 0u;
  if (t < 2) counters[t] = 0u;
}

__device__ __forceinline__ RunSum rs_shift(RunSum r, int d) {
  r.hi += d;
  r.ti += d;
  return r;
}

// Streaming, one (row, width) per thread: append this push's segment
// summaries to the carried one. A run that touches the stream's first
// position and has ended is reported here; everything still open is carried
// with positions re-based on the next gulp.
__global__ __launch_bounds__(256) void k_stream_fold(StreamArgs A) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= A.rows * A.nw) return;
  const int row = t / A.nw, j = t - row * A.nw;
  const Emitter em{nullptr, nullptr, A.cands, A.ncand, A.cap, (uint32_t)row + A.row_offset, (uint32_t)(1 << j),
                   true, 0};
  RunSum acc = A.carry[t];
  const RunSum* f = A.frag + (int64_t)t * A.nseg;
  for (int s = 0; s < A.nseg; ++s) acc = rs_combine(acc, rs_shift(f[s], -A.Hx), em);
  if ((acc.flags & kHead) && !(acc.flags & kFull)) {
    emit(em, acc.hi, acc.hq);
    acc.flags &= ~kHead;
  }
  A.carry[t] = rs_shift(acc, -A.ngulp);
}

// Streaming flush: the stream has ended, so every carried run is closed.
__global__ __launch_bounds__(256) void k_stream_close(StreamArgs A) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= A.rows * A.nw) return;
  const int row = t / A.nw, j = t - row * A.nw;
  const Emitter em{nullptr, nullptr, A.cands, A.ncand, A.cap, (uint32_t)row + A.row_offset, (uint32_t)(1 << j),
                   true, 0};
  rs_close(A.carry[t], em);
  A.carry[t] = rs_empty();
}

// Streaming: the next push's history is the last Hx samples (and Hb block
// statistics) of this push's virtual row; the stream start moves down by
// the gulp length. Grid: (chunks, rows).
__global__ __launch_bounds__(256) void k_stream_advance(StreamArgs A) {
  const int row = blockIdx.y;
  const int nbg = A.nbv - A.Hb;
  const float* hin = A.hist_in + (int64_t)row * A.Hx;
  const float* gin = A.gulp + (int64_t)row * A.ngulp;
  float* hout = A.hist_out + (int64_t)row * A.Hx;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < A.Hx; t += gridDim.x * blockDim.x) {
    const int v = t + A.ngulp;
    hout[t] = v < A.Hx ? hin[v] : gin[v - A.Hx];
  }
  const int32_t* mi = A.med_in + (int64_t)row * A.nbv;
  const int32_t* di = A.mad_in + (int64_t)row * A.nbv;
  int32_t* mo = A.med_out + (int64_t)row * A.nbv;
  int32_t* dout = A.mad_out + (int64_t)row * A.nbv;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < A.Hb; k += gridDim.x * blockDim.x) {
    mo[k] = mi[k + nbg];
    dout[k] = di[k + nbg];
  }
  if (row == 0 && blockIdx.x == 0 && threadIdx.x == 0) *A.tmin = max(0, *A.tmin - A.ngulp);
}

// Domain check: *bad = 1 if a sample is not an integer or |x| > bound
// (NaN and infinities fail both tests).
__global__ __launch_bounds__(256) void k_validate(const float* x, int64_t n, float bound, uint32_t* bad) {
  bool ok = true;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float v = x[i];
    ok = ok && fabsf(v) <= bound && v == rintf(v);
  }
  if (!ok) *bad = 1u;
}

__global__ void k_zero_u32(uint32_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

}  // namespace

hipError_t launch_detect(const DetectArgs& a, hipStream_t s) {
  const int64_t grid = (int64_t)a.rows * a.nseg;
  if (grid <= 0) return hipSuccess;
  const dim3 g((unsigned)grid), b(256);
  if (a.Hx > 0) {
    if (a.nw == 13) hipLaunchKernelGGL((k_detect<13, true>), g, b, 0, s, a);
    else hipLaunchKernelGGL((k_detect<0, true>), g, b, 0, s, a);
  } else {
    if (a.nw == 13) hipLaunchKernelGGL((k_detect<13, false>), g, b, 0, s, a);
    else if (a.nw == 7) hipLaunchKernelGGL((k_detect<7, false>), g, b, 0, s, a);
    else hipLaunchKernelGGL((k_detect<0, false>), g, b, 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_fixup(const DetectArgs& a, hipStream_t s) {
  const int n = a.rows * a.nw;
  if (n <= 0 || a.nseg <= 1) return hipSuccess;
  hipLaunchKernelGGL(k_fixup, dim3((n + 255) / 256), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_stream_fold(const StreamArgs& a, hipStream_t s) {
  const int n = a.rows * a.nw;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_stream_fold, dim3((n + 255) / 256), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_stream_close(const StreamArgs& a, hipStream_t s) {
  const int n = a.rows * a.nw;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_stream_close, dim3((n + 255) / 256), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_stream_advance(const StreamArgs& a, hipStream_t s) {
  if (a.rows <= 0) return hipSuccess;
  const int chunks = (a.Hx + 4095) / 4096;
  hipLaunchKernelGGL(k_stream_advance, dim3(chunks > 0 ? chunks : 1, a.rows), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_detect_batch(const BatchDetect& b, int nw_all, bool virt, int grid, hipStream_t s) {
  if (b.total <= 0) return hipSuccess;
  if (virt) {
    if (nw_all == 13) hipLaunchKernelGGL((k_detect_batch<13, true>), dim3(grid), dim3(256), 0, s, b);
    else hipLaunchKernelGGL((k_detect_batch<0, true>), dim3(grid), dim3(256), 0, s, b);
  } else {
    if (nw_all == 13) hipLaunchKernelGGL((k_detect_batch<13, false>), dim3(grid), dim3(256), 0, s, b);
    else hipLaunchKernelGGL((k_detect_batch<0, false>), dim3(grid), dim3(256), 0, s, b);
  }
  return hipGetLastError();
}

int detect_batch_grid(int nw_all) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  hipError_t e = nw_all == 13
      ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_detect_batch<13, false>, 256, 0)
      : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_detect_batch<0, false>, 256, 0);
  if (e != hipSuccess) return 0;
  return cus * (per > 0 ? per : 1);
}

hipError_t launch_fixup_batch(const BatchDetect& b, const int32_t* d_offs, int total, hipStream_t s) {
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fixup_batch, dim3((total + 255) / 256), dim3(256), 0, s, b, d_offs);
  return hipGetLastError();
}

hipError_t launch_batch_zero(uint32_t* const* d_ncand, int n, uint32_t* counters, hipStream_t s) {
  const int m = n > 2 ? n : 2;
  hipLaunchKernelGGL(k_batch_zero, dim3((m + 255) / 256), dim3(256), 0, s, d_ncand, n, counters);
  return hipGetLastError();
}

hipError_t launch_validate(const float* x, int64_t n, float bound, uint32_t* bad, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_validate, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(256), 0, s, x, n, bound, bad);
  return hipGetLastError();
}

hipError_t launch_zero_u32(uint32_t* p, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_u32, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace sps
