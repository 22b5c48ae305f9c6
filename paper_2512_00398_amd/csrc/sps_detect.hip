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
// block S/N is strictly increasing in S, so run maxima are found on S; best
// positions are compared across blocks by cross-multiplication and only a
// near-tie falls back to the two divisions, which reproduces the comparison of
// the rounded S/N values exactly. The S/N value itself is divided once, when a
// candidate is emitted.
//
// Layout (gfx950, wave64). One 256-thread workgroup streams one segment of a
// row in steps of 1024 samples: coalesced float4 loads, residuals, a
// workgroup scan into an 8192-entry LDS ring of P (max_width of history).
// For width w the step's positions are grouped 64 per (wave, q) so that each
// group shares one centre block k* (window ends E with E - ceil(w/2) = 0 mod
// 64): the group's bound is one scalar. Fast pass: per lane and width two LDS
// reads, a subtract and a compare folded into a ballot. Widths with any
// position beyond the bound take the run pass: the above-mask of each group
// is walked in scalar code, a DPP max-reduction finds each run's best S, and
// associative RunSum summaries stitch runs across groups, waves (one owner
// wave per width), steps and, through the fix-up kernel, segments.
// Candidates are staged in LDS and flushed with one global atomic per step.
#include <climits>

#include "sps_internal.h"
#include "sps_wave.h"

namespace sps {

namespace {

constexpr int kC = 1024;                 // samples (window ends) per step
constexpr int kRing = 8192;              // ring entries, >= kC + 64 + max width
constexpr int kGroups = kC / 64;         // 64-position groups per step and width
constexpr int kCbuf = 512;               // LDS candidate staging records

struct Emitter {
  sps_cand* cbuf;       // LDS staging (null: write to global directly)
  uint32_t* cbuf_n;
  sps_cand* cands;
  uint32_t* ncand;
  uint32_t cap;
  uint32_t dm;
  uint32_t width;
  bool writer;          // the one thread that writes (lane 0 in wave code)
};

__device__ __forceinline__ void emit(const Emitter& E, int32_t sample, int32_t S, double den) {
  if (!E.writer) return;
  sps_cand c;
  c.sample = sample;
  c.dm_idx = E.dm;
  c.width = E.width;
  c.snr = (float)((double)S / den);
  if (E.cbuf) {
    const uint32_t s = atomicAdd(E.cbuf_n, 1u);
    if (s < (uint32_t)kCbuf) {
      E.cbuf[s] = c;
      return;
    }
  }
  const uint32_t slot = atomicAdd(E.ncand, 1u);
  if (slot < E.cap) E.cands[slot] = c;
}

__device__ __forceinline__ RunSum rs_empty() {
  RunSum r;
  r.flags = 0; r.hi = 0; r.ti = 0; r.hS = 0; r.tS = 0; r.pad = 0; r.hd = 1.0; r.td = 1.0;
  return r;
}

// true if S1/d1 at i1 beats S2/d2 at i2 in the rounded-double order (larger
// S/N, earlier sample on ties). S > 0 and d > 0 for every above position.
__device__ __forceinline__ bool beats(int S1, double d1, int i1, int S2, double d2, int i2) {
  if (d1 == d2) return S1 > S2 || (S1 == S2 && i1 < i2);
  const double a = (double)S1 * d2, b = (double)S2 * d1;
  // a, b carry < 2^-53 relative error each: a gap of 1e-15 proves the
  // rounded quotients differ in the same direction
  if (a > b * (1.0 + 1e-15)) return true;
  if (a < b * (1.0 - 1e-15)) return false;
  const double q1 = (double)S1 / d1, q2 = (double)S2 / d2;
  return q1 > q2 || (q1 == q2 && i1 < i2);
}

// Summary of range L followed immediately by range R. Runs that end at the
// junction (and so touch neither end of L+R) are emitted.
__device__ RunSum rs_combine(const RunSum& L, const RunSum& R, const Emitter& E) {
  if (!(L.flags & kNonEmpty)) return R;
  if (!(R.flags & kNonEmpty)) return L;
  RunSum o = rs_empty();
  o.flags = kNonEmpty;
  if (L.flags & kFull) {
    o.flags |= kHead;
    o.hi = L.hi; o.hS = L.hS; o.hd = L.hd;
    if ((R.flags & kHead) && beats(R.hS, R.hd, R.hi, o.hS, o.hd, o.hi)) { o.hi = R.hi; o.hS = R.hS; o.hd = R.hd; }
    if (R.flags & kFull) { o.flags |= kFull; return o; }
    if (R.flags & kTail) { o.flags |= kTail; o.ti = R.ti; o.tS = R.tS; o.td = R.td; }
    return o;
  }
  if (L.flags & kHead) { o.flags |= kHead; o.hi = L.hi; o.hS = L.hS; o.hd = L.hd; }
  if (R.flags & kFull) {
    o.flags |= kTail;
    o.ti = R.hi; o.tS = R.hS; o.td = R.hd;
    if ((L.flags & kTail) && !beats(R.hS, R.hd, R.hi, L.tS, L.td, L.ti)) { o.ti = L.ti; o.tS = L.tS; o.td = L.td; }
    return o;
  }
  if (R.flags & kTail) { o.flags |= kTail; o.ti = R.ti; o.tS = R.tS; o.td = R.td; }
  const bool lt = L.flags & kTail, rh = R.flags & kHead;
  if (lt && rh) {
    if (beats(R.hS, R.hd, R.hi, L.tS, L.td, L.ti)) emit(E, R.hi, R.hS, R.hd);
    else emit(E, L.ti, L.tS, L.td);
  } else if (lt) {
    emit(E, L.ti, L.tS, L.td);
  } else if (rh) {
    emit(E, R.hi, R.hS, R.hd);
  }
  return o;
}

// Runs touching the ends of a whole row are closed there.
__device__ void rs_close(const RunSum& s, const Emitter& E) {
  if (s.flags & kHead) emit(E, s.hi, s.hS, s.hd);
  if (s.flags & kTail) emit(E, s.ti, s.tS, s.td);
}

// Best (largest S, earliest lane) of the lanes in `run`; wave-uniform result.
__device__ __forceinline__ void run_best(uint64_t run, int S, int lane, int& bestS, int& bestLane) {
  const bool in = (run >> lane) & 1ull;
  bestS = wave_max_u(in ? S : INT_MIN);
  bestLane = ctz(ballot(in && S == bestS));
}

// Summary of one 64-position group with a single denominator d. M: above
// lanes, V: valid lanes (contiguous), i0: sample index of lane 0.
__device__ RunSum group_summary(uint64_t M, uint64_t V, int S, double d, int i0, int lane, const Emitter& E) {
  RunSum g = rs_empty();
  if (!V) return g;
  g.flags = kNonEmpty;
  if (!M) return g;
  int bs, bl;
  if (M == V) {
    run_best(M, S, lane, bs, bl);
    g.flags |= kFull | kHead;
    g.hi = i0 + bl; g.hS = bs; g.hd = d;
    return g;
  }
  const int fv = ctz(V), lv = msb(V);
  uint64_t m = M;
  while (m) {
    const int a = ctz(m);
    const uint64_t gap = ~m & (~0ull << a);
    const int b = gap ? ctz(gap) : 64;
    const uint64_t run = (b == 64 ? ~0ull : ((1ull << b) - 1ull)) & (~0ull << a);
    run_best(run, S, lane, bs, bl);
    if (a == fv) { g.flags |= kHead; g.hi = i0 + bl; g.hS = bs; g.hd = d; }
    else if (b - 1 == lv) { g.flags |= kTail; g.ti = i0 + bl; g.tS = bs; g.td = d; }
    else emit(E, i0 + bl, bs, d);
    m &= ~run;
  }
  return g;
}

// Window ends of width w in a step start (64 - ceil(w/2) mod 64) mod 64
// before the step, so that every 64-lane group shares one centre block.
__device__ __forceinline__ int group_shift(int w) {
  const int sub = w - (w >> 1);
  return (64 - (sub & 63)) & 63;
}

__global__ __launch_bounds__(256) void k_detect(DetectArgs A) {
  __shared__ uint32_t ring[kRing];
  __shared__ int32_t tlo[kMaxWidths][kGroups];
  __shared__ int32_t thi[kMaxWidths][kGroups];
  __shared__ double tden[kMaxWidths][kGroups];
  __shared__ RunSum carry[kMaxWidths];
  __shared__ RunSum wsum[kMaxWidths][4];
  __shared__ sps_cand cbuf[kCbuf];
  __shared__ uint32_t wtot[4];
  __shared__ uint32_t step_mask, cbuf_n, flush_n, flush_base;

  const int tid = threadIdx.x, wave = tid >> 6, lane = lane_id();
  const int row = blockIdx.x / A.nseg;
  const int seg = blockIdx.x - row * A.nseg;
  const int N = A.N;
  const int s0 = seg * A.seg_len;
  const int s1 = min(N, s0 + A.seg_len);
  const float* xr = A.x + (int64_t)row * A.ld;
  const int32_t* medr = A.med + (int64_t)row * A.nblocks;
  const int32_t* madr = A.mad + (int64_t)row * A.nblocks;
  const int emax = min(s1 - s0 + A.maxw - 1, N - s0);  // last window end needed
  const int nsteps = (emax + 64) / kC + 1;              // + group shift headroom
  const bool vec = ((reinterpret_cast<uintptr_t>(xr) & 15u) == 0);
  const uint32_t dm = (uint32_t)row + A.row_offset;
  const int e_row = N - s0;  // E <= N - s0      <=> i <= N - w
  const int e_seg = s1 - s0; // E < s1 - s0 + w  <=> i < s1

  if (tid < A.nw) carry[tid] = rs_empty();
  if (tid == 0) { ring[3] = 0u; cbuf_n = 0u; }
  uint32_t carryP = 0;  // P at the step's first sample
  __syncthreads();

  for (int c = 0; c < nsteps; ++c) {
    const int cC = c * kC;
    // residuals of samples s0 + cC + 4*tid + q and their local prefix
    const int t0 = s0 + cC + 4 * tid;
    int r0 = 0, r1 = 0, r2 = 0, r3 = 0;
    if (t0 < N) {
      const int mk = medr[t0 >> 6];
      if (vec && t0 + 3 < N) {
        const float4 v = *reinterpret_cast<const float4*>(xr + t0);
        r0 = __float2int_rz(v.x) - mk; r1 = __float2int_rz(v.y) - mk;
        r2 = __float2int_rz(v.z) - mk; r3 = __float2int_rz(v.w) - mk;
      } else {
        r0 = __float2int_rz(xr[t0]) - mk;
        if (t0 + 1 < N) r1 = __float2int_rz(xr[t0 + 1]) - mk;
        if (t0 + 2 < N) r2 = __float2int_rz(xr[t0 + 2]) - mk;
        if (t0 + 3 < N) r3 = __float2int_rz(xr[t0 + 3]) - mk;
      }
    }
    const uint32_t p0 = (uint32_t)r0, p1 = p0 + (uint32_t)r1, p2 = p1 + (uint32_t)r2, p3 = p2 + (uint32_t)r3;
    const uint32_t incl = (uint32_t)wave_scan_incl((int)p3);
    if (lane == 63) wtot[wave] = incl;
    __syncthreads();  // B1: wave totals; last step's emissions are complete

    uint32_t woff = 0;
    for (int v = 0; v < wave; ++v) woff += wtot[v];
    const uint32_t tot = wtot[0] + wtot[1] + wtot[2] + wtot[3];
    const uint32_t pb = carryP + woff + incl - p3;
    *reinterpret_cast<uint4*>(&ring[(cC + 4 * tid + 4) & (kRing - 1)]) =
        make_uint4(pb + p0, pb + p1, pb + p2, pb + p3);
    carryP += tot;
    // integer bounds and denominators: one per (width, group)
    if (tid < A.nw * kGroups) {
      const int j = tid / kGroups, g = tid - j * kGroups;
      const int w = 1 << j, sub = w - (w >> 1);
      const int k = ((s0 + cC - group_shift(w) - sub) >> 6) + g;
      const int madv = (k >= 0 && k < A.nblocks) ? madr[k] : 0;
      const double den = (kMadToSigma * (double)madv) * A.sqrtw[j];
      int lo = INT_MAX, hi = INT_MAX;
      if (madv > 0) {
        const double tt = A.theta * den;
        if (tt < 2147483648.0) {
          lo = (int)(floor(tt) - 1.0);
          const double hd = ceil(tt) + 1.0;
          hi = hd >= 2147483647.0 ? INT_MAX : (int)hd;
        }
      }
      tlo[j][g] = lo;
      thi[j][g] = hi;
      tden[j][g] = madv > 0 ? den : 1.0;
    }
    if (tid == 0) {
      step_mask = 0u;
      const uint32_t n = min(cbuf_n, (uint32_t)kCbuf);
      flush_n = n;
      flush_base = n ? atomicAdd(A.ncand, n) : 0u;
      cbuf_n = 0u;
    }
    __syncthreads();  // B2: ring, bounds, flush slot

    {  // flush the previous step's staged candidates
      const uint32_t n = flush_n, base = flush_base;
      for (uint32_t i = tid; i < n; i += 256)
        if (base + i < A.cap) A.cands[base + i] = cbuf[i];
    }

    // fast pass: does any position of this step pass a width's bound?
    {
      int cur_shift = -1;
      uint32_t pe[4] = {0u, 0u, 0u, 0u};
      for (int j = 0; j < A.nw; ++j) {
        const int w = 1 << j, sh = group_shift(w);
        const int eg = cC - sh + 256 * wave;
        if (sh != cur_shift) {
          cur_shift = sh;
#pragma unroll
          for (int q = 0; q < 4; ++q) pe[q] = ring[(eg + 64 * q + lane + 3) & (kRing - 1)];
        }
        const int vhi = min(e_seg + w - 1, e_row);
        uint64_t acc = 0ull;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e0 = eg + 64 * q;
          const int S = (int)(pe[q] - ring[(e0 + lane - w + 3) & (kRing - 1)]);
          const int T = tlo[j][4 * wave + q];
          acc |= ballot(S > T) & lane_range(w - e0, vhi - e0);
        }
        if (acc && lane == 0) atomicOr(&step_mask, 1u << j);
      }
    }
    __syncthreads();  // B3: step_mask complete; flush copies done

    // run pass for widths with candidates in this step
    const uint32_t smask = step_mask;
    for (int j = 0; j < A.nw; ++j) {
      if (!((smask >> j) & 1u)) continue;
      const int w = 1 << j, sh = group_shift(w);
      const int eg = cC - sh + 256 * wave;
      const int vhi = min(e_seg + w - 1, e_row);
      const Emitter em{cbuf, &cbuf_n, A.cands, A.ncand, A.cap, dm, (uint32_t)w, lane == 0};
      RunSum acc = rs_empty();
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e0 = eg + 64 * q, g = 4 * wave + q;
        const int e = e0 + lane;
        const int S = (int)(ring[(e + 3) & (kRing - 1)] - ring[(e - w + 3) & (kRing - 1)]);
        const int lo = tlo[j][g], hi = thi[j][g];
        const double d = tden[j][g];
        const bool above = S > lo && ((S >= hi && hi != INT_MAX) || (double)S / d > A.theta);
        const uint64_t V = lane_range(w - e0, vhi - e0);
        const uint64_t M = ballot(above) & V;
        const RunSum gs = group_summary(M, V, S, d, s0 + e0 - w, lane, em);
        acc = rs_combine(acc, gs, em);
      }
      if (lane == 0) wsum[j][wave] = acc;
    }
    __syncthreads();  // B4: wave summaries

    // width j is owned by wave j % 4: fold the step into its running summary
    for (int j = wave; j < A.nw; j += 4) {
      const int w = 1 << j, sh = group_shift(w);
      const Emitter em{cbuf, &cbuf_n, A.cands, A.ncand, A.cap, dm, (uint32_t)w, lane == 0};
      RunSum cj = carry[j];
      bool dirty = false;
      if ((smask >> j) & 1u) {
        for (int v = 0; v < 4; ++v) cj = rs_combine(cj, wsum[j][v], em);
        dirty = true;
      } else {
        // nothing above for width j: a non-empty step closes an open run
        const int elo = max(cC - sh, w), ehi = min(cC - sh + kC - 1, min(e_seg + w - 1, e_row));
        if (elo <= ehi) {
          if (!(cj.flags & kNonEmpty)) {
            cj.flags = kNonEmpty;
            dirty = true;
          } else if (cj.flags & (kTail | kFull)) {
            RunSum below = rs_empty();
            below.flags = kNonEmpty;
            cj = rs_combine(cj, below, em);
            dirty = true;
          }
        }
      }
      if (dirty && lane == 0) carry[j] = cj;
    }
  }

  __syncthreads();
  for (int j = wave; j < A.nw; j += 4) {
    const RunSum cj = carry[j];
    const Emitter em{cbuf, &cbuf_n, A.cands, A.ncand, A.cap, dm, (uint32_t)(1 << j), lane == 0};
    if (A.nseg == 1) rs_close(cj, em);
    else if (lane == 0) A.frag[((int64_t)row * A.nw + j) * A.nseg + seg] = cj;
  }
  __syncthreads();
  if (tid == 0) {
    const uint32_t n = min(cbuf_n, (uint32_t)kCbuf);
    flush_n = n;
    flush_base = n ? atomicAdd(A.ncand, n) : 0u;
  }
  __syncthreads();
  for (uint32_t i = tid; i < flush_n; i += 256)
    if (flush_base + i < A.cap) A.cands[flush_base + i] = cbuf[i];
}

// Stitch the segment summaries of each (row, width) in order.
__global__ __launch_bounds__(256) void k_fixup(DetectArgs A) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= A.rows * A.nw) return;
  const int row = t / A.nw, j = t - row * A.nw;
  const Emitter em{nullptr, nullptr, A.cands, A.ncand, A.cap, (uint32_t)row + A.row_offset, (uint32_t)(1 << j),
                   true};
  const RunSum* f = A.frag + (int64_t)t * A.nseg;
  RunSum acc = rs_empty();
  for (int s = 0; s < A.nseg; ++s) acc = rs_combine(acc, f[s], em);
  rs_close(acc, em);
}

__global__ void k_zero_u32(uint32_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

}  // namespace

hipError_t launch_detect(const DetectArgs& a, hipStream_t s) {
  const int64_t grid = (int64_t)a.rows * a.nseg;
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_detect, dim3((unsigned)grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_fixup(const DetectArgs& a, hipStream_t s) {
  const int n = a.rows * a.nw;
  if (n <= 0 || a.nseg <= 1) return hipSuccess;
  hipLaunchKernelGGL(k_fixup, dim3((n + 255) / 256), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_zero_u32(uint32_t* p, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_u32, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace sps
