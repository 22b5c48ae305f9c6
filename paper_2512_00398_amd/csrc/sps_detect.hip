// sps_detect.hip - matched filtering and peak detection stages (Heimdall++,
// Section II-B), fused: residuals, boxcar sums at every power-of-two width,
// the S/N threshold and run-based peak picking in one pass over the block.
//
// Arithmetic (exact): r_t = x_t - m_{t/64}; prefix P[E] = sum of r over the
// first E samples of the segment (uint32, wrapping; differences are exact
// while |S| < 2^31); S_w(i) = P[E] - P[E - w] with E = i - s0 + w. The S/N
// decision "S / ((K * MAD_{k*}) * sqrt(w)) > theta" is taken in IEEE double,
// exactly as the definition states, but only for S inside a 3-integer band
// around the threshold: integer bounds lo < S < hi computed per (block, width)
// decide every other position without floating point. Within one centre block
// S/N is strictly increasing in S, so a run's arg-max is found on S and only
// the winner is divided.
//
// Layout (gfx950): one 256-thread workgroup streams one segment of one row in
// steps of 1024 window ends. Step: coalesced float4 loads of 1024 samples,
// residual, workgroup scan into an 8192-entry LDS ring of P (the ring keeps
// max_width history), then each lane evaluates 4 window ends
// (E = 256*wave + 64*q + lane) for every width: two LDS reads, one subtract,
// one compare against the block's integer bound. Widths with any candidate
// in the step (one ballot per width) take the run pass: ballots give the
// above-mask of each 64-position group, runs are walked in scalar code, a
// wave max-reduction finds each run's best S. Runs are stitched across
// groups, waves and steps with associative RunSum summaries; runs that touch
// a segment edge are left to the fix-up kernel.
#include <climits>

#include "sps_internal.h"
#include "sps_wave.h"

namespace sps {

namespace {

constexpr int kC = 1024;             // window ends per step (256 threads x 4)
constexpr int kRing = 8192;          // ring entries, >= kC + max width + 1
constexpr int kTbl = kC / kStride + 1;  // centre blocks touched per width per step

struct Emitter {
  sps_cand* cands;
  uint32_t* ncand;
  uint32_t cap;
  uint32_t dm;
  uint32_t width;
  bool writer;  // the one thread that writes (lane 0 in wave code)
};

__device__ __forceinline__ void emit(const Emitter& E, int32_t sample, double snr) {
  if (E.writer) {
    const uint32_t slot = atomicAdd(E.ncand, 1u);
    if (slot < E.cap) {
      sps_cand c;
      c.sample = sample;
      c.dm_idx = E.dm;
      c.width = E.width;
      c.snr = (float)snr;
      E.cands[slot] = c;
    }
  }
}

__device__ __forceinline__ RunSum rs_empty() {
  RunSum r;
  r.flags = 0; r.hi = 0; r.ti = 0; r.pad = 0; r.hs = 0.0; r.ts = 0.0;
  return r;
}

// true if (s1, i1) beats (s2, i2): larger S/N, earlier sample on ties
__device__ __forceinline__ bool beats(double s1, int i1, double s2, int i2) {
  return s1 > s2 || (s1 == s2 && i1 < i2);
}

// Summary of range L followed immediately by range R. Runs that end at the
// junction (and so touch neither end of L+R) are emitted.
__device__ RunSum rs_combine(const RunSum& L, const RunSum& R, const Emitter& E) {
  if (!(L.flags & kNonEmpty)) return R;
  if (!(R.flags & kNonEmpty)) return L;
  RunSum o = rs_empty();
  o.flags = kNonEmpty;
  const bool lf = L.flags & kFull, rf = R.flags & kFull;
  if (lf) {
    o.flags |= kHead;
    o.hs = L.hs; o.hi = L.hi;
    if ((R.flags & kHead) && beats(R.hs, R.hi, o.hs, o.hi)) { o.hs = R.hs; o.hi = R.hi; }
    if (rf) { o.flags |= kFull; return o; }
    if (R.flags & kTail) { o.flags |= kTail; o.ts = R.ts; o.ti = R.ti; }
    return o;
  }
  if (L.flags & kHead) { o.flags |= kHead; o.hs = L.hs; o.hi = L.hi; }
  if (rf) {
    o.flags |= kTail;
    o.ts = R.hs; o.ti = R.hi;
    if ((L.flags & kTail) && !beats(R.hs, R.hi, L.ts, L.ti)) { o.ts = L.ts; o.ti = L.ti; }
    return o;
  }
  if (R.flags & kTail) { o.flags |= kTail; o.ts = R.ts; o.ti = R.ti; }
  const bool lt = L.flags & kTail, rh = R.flags & kHead;
  if (lt && rh) {
    if (beats(R.hs, R.hi, L.ts, L.ti)) emit(E, R.hi, R.hs); else emit(E, L.ti, L.ts);
  } else if (lt) {
    emit(E, L.ti, L.ts);
  } else if (rh) {
    emit(E, R.hi, R.hs);
  }
  return o;
}

// Runs touching the ends of a whole row are closed there.
__device__ void rs_close(const RunSum& s, const Emitter& E) {
  if (s.flags & kHead) emit(E, s.hi, s.hs);
  if (s.flags & kTail) emit(E, s.ti, s.ts);
}

struct Best {
  double s;
  int32_t i;
  bool v;
};

// Best position of `run` (a lane mask) by S/N, earliest on ties. Lanes below
// `off` have centre block A (denominator dA), the others block B.
__device__ __forceinline__ Best run_best(uint64_t run, int S, int off, double dA, double dB, int i0, int lane) {
  const uint64_t maskA = off ? ((1ull << off) - 1ull) : 0ull;
  const uint64_t pa = run & maskA, pb = run & ~maskA;
  Best b;
  b.v = false; b.s = 0.0; b.i = 0;
  if (pa) {
    const bool in = (pa >> lane) & 1ull;
    const int m = wave_max(in ? S : INT_MIN);
    const int j = ctz(ballot(in && S == m));
    b.s = (double)m / dA; b.i = i0 + j; b.v = true;
  }
  if (pb) {
    const bool in = (pb >> lane) & 1ull;
    const int m = wave_max(in ? S : INT_MIN);
    const int j = ctz(ballot(in && S == m));
    const double s = (double)m / dB;
    if (!b.v || s > b.s) { b.s = s; b.i = i0 + j; b.v = true; }
  }
  return b;
}

// Summary of one 64-position group: M above-mask, V valid-mask (contiguous).
__device__ RunSum group_summary(uint64_t M, uint64_t V, int S, int off, double dA, double dB, int i0, int lane,
                                const Emitter& E) {
  RunSum g = rs_empty();
  if (!V) return g;
  g.flags = kNonEmpty;
  if (M == V) {
    const Best b = run_best(M, S, off, dA, dB, i0, lane);
    g.flags |= kFull | kHead;
    g.hs = b.s; g.hi = b.i;
    return g;
  }
  const int fv = ctz(V), lv = msb(V);
  uint64_t m = M;
  while (m) {
    const int a = ctz(m);
    const uint64_t gap = ~m & (~0ull << a);
    const int b = gap ? ctz(gap) : 64;
    const uint64_t run = (b == 64 ? ~0ull : ((1ull << b) - 1ull)) & (~0ull << a);
    const Best bb = run_best(run, S, off, dA, dB, i0, lane);
    if (a == fv) { g.flags |= kHead; g.hs = bb.s; g.hi = bb.i; }
    else if (b - 1 == lv) { g.flags |= kTail; g.ts = bb.s; g.ti = bb.i; }
    else emit(E, bb.i, bb.s);
    m &= ~run;
  }
  return g;
}

__global__ __launch_bounds__(256) void k_detect(DetectArgs A) {
  __shared__ uint32_t ring[kRing];
  __shared__ int32_t tlo[kMaxWidths][kTbl];
  __shared__ int32_t thi[kMaxWidths][kTbl];
  __shared__ double tden[kMaxWidths][kTbl];
  __shared__ uint32_t wtot[4];
  __shared__ uint32_t step_mask;
  __shared__ RunSum carry[kMaxWidths];
  __shared__ RunSum wsum[kMaxWidths][4];

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
  const int nsteps = emax / kC + 1;
  const bool vec = ((reinterpret_cast<uintptr_t>(xr) & 15u) == 0);
  const uint32_t dm = (uint32_t)row + A.row_offset;

  if (tid < A.nw) carry[tid] = rs_empty();
  if (tid == 0) ring[3] = 0u;  // P[0] lives at ring index 0 + 3
  uint32_t carryP = 0;         // P at the first window end of the step
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
    __syncthreads();
    uint32_t woff = 0;
    for (int v = 0; v < wave; ++v) woff += wtot[v];
    const uint32_t tot = wtot[0] + wtot[1] + wtot[2] + wtot[3];
    const uint32_t pb = carryP + woff + incl - p3;
    *reinterpret_cast<uint4*>(&ring[(cC + 4 * tid + 4) & (kRing - 1)]) =
        make_uint4(pb + p0, pb + p1, pb + p2, pb + p3);
    carryP += tot;

    // integer bounds and denominators for the centre blocks of this step
    if (tid < A.nw * kTbl) {
      const int j = tid / kTbl, o = tid - j * kTbl;
      const int w = 1 << j, sub = w - (w >> 1);
      const int k = ((s0 + cC - sub) >> 6) + o;
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
      tlo[j][o] = lo;
      thi[j][o] = hi;
      tden[j][o] = den;
    }
    if (tid == 0) step_mask = 0u;
    __syncthreads();

    // fast pass: does any position of this step pass a width's bound?
    const int eb = cC + 256 * wave + lane;
    uint32_t pe[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) pe[q] = ring[(eb + 64 * q + 3) & (kRing - 1)];
    const int e_row = N - s0;            // E <= N - s0  <=>  i <= N - w
    const int e_seg = s1 - s0;           // E < s1 - s0 + w  <=>  i < s1
    for (int j = 0; j < A.nw; ++j) {
      const int w = 1 << j, sub = w - (w >> 1);
      const int kb = (s0 + cC - sub) >> 6;
      bool any = false;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = eb + 64 * q;
        const int S = (int)(pe[q] - ring[(e - w + 3) & (kRing - 1)]);
        const bool valid = e >= w && e < e_seg + w && e <= e_row;
        const int o = ((s0 + e - sub) >> 6) - kb;
        any |= valid && S > tlo[j][o];
      }
      if (ballot(any) && lane == 0) atomicOr(&step_mask, 1u << j);
    }
    __syncthreads();

    // run pass for widths with candidates in this step
    const uint32_t smask = step_mask;
    for (int j = 0; j < A.nw; ++j) {
      if (!((smask >> j) & 1u)) continue;
      const int w = 1 << j, sub = w - (w >> 1);
      const int kb = (s0 + cC - sub) >> 6;
      const Emitter em{A.cands, A.ncand, A.cap, dm, (uint32_t)w, lane == 0};
      RunSum acc = rs_empty();
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = eb + 64 * q;
        const int S = (int)(pe[q] - ring[(e - w + 3) & (kRing - 1)]);
        const bool valid = e >= w && e < e_seg + w && e <= e_row;
        const int o = ((s0 + e - sub) >> 6) - kb;
        const int lo = tlo[j][o], hi = thi[j][o];
        const bool above = valid && S > lo && ((S >= hi && hi != INT_MAX) || (double)S / tden[j][o] > A.theta);
        const uint64_t M = ballot(above), V = ballot(valid);
        const int e0 = cC + 256 * wave + 64 * q;
        const int oA = ((s0 + e0 - sub) >> 6) - kb;
        const int off = sub & 63;
        const double dA = tden[j][oA];
        const double dB = off ? tden[j][oA + 1] : dA;
        const RunSum g = group_summary(M, V, S, off, dA, dB, s0 + e0 - w, lane, em);
        acc = rs_combine(acc, g, em);
      }
      if (lane == 0) wsum[j][wave] = acc;
    }
    __syncthreads();

    // wave 0 folds this step into the segment's running summaries
    if (wave == 0) {
      for (int j = 0; j < A.nw; ++j) {
        const int w = 1 << j;
        const Emitter em{A.cands, A.ncand, A.cap, dm, (uint32_t)w, lane == 0};
        RunSum cj = carry[j];
        if ((smask >> j) & 1u) {
          for (int v = 0; v < 4; ++v) cj = rs_combine(cj, wsum[j][v], em);
        } else {
          // nothing above for this width: a non-empty step closes an open run
          const int elo = max(cC, w), ehi = min(cC + kC - 1, min(e_seg + w - 1, e_row));
          if (elo <= ehi) {
            RunSum below = rs_empty();
            below.flags = kNonEmpty;
            cj = rs_combine(cj, below, em);
          }
        }
        if (lane == 0) carry[j] = cj;
      }
    }
  }

  if (wave == 0) {
    for (int j = 0; j < A.nw; ++j) {
      const RunSum cj = carry[j];
      const Emitter em{A.cands, A.ncand, A.cap, dm, (uint32_t)(1 << j), lane == 0};
      if (A.nseg == 1) rs_close(cj, em);
      else if (lane == 0) A.frag[((int64_t)row * A.nw + j) * A.nseg + seg] = cj;
    }
  }
}

// Stitch the segment summaries of each (row, width) in order.
__global__ __launch_bounds__(256) void k_fixup(DetectArgs A) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= A.rows * A.nw) return;
  const int row = t / A.nw, j = t - row * A.nw;
  const Emitter em{A.cands, A.ncand, A.cap, (uint32_t)row + A.row_offset, (uint32_t)(1 << j), true};
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
