// sps_detect_body.h - the fused matched-filter and peak-detection body
// (Heimdall++, Section II-B) behind k_detect, shared by the detection kernels
// and the fused batch kernel. See sps_detect.hip for the design.
#pragma once

#include <climits>
#include <type_traits>

#include "sps_internal.h"
#include "sps_runs.h"
#include "sps_wave.h"

namespace sps {

namespace {

constexpr int kC = 1024;                 // samples (window ends) per step
constexpr int kRing = 8192;              // ring entries, >= kC + 64 + max width
constexpr int kGroups = kC / 64;         // 64-position groups per step and width

// Best (largest S, earliest lane) of the lanes in `run`; wave-uniform result.
__device__ __forceinline__ void run_best(uint64_t run, int S, int lane, int& bestS, int& bestLane) {
  const bool in = (run >> lane) & 1ull;
  bestS = wave_max_u(in ? S : INT_MIN);
  bestLane = ctz(ballot(in && S == bestS));
}

// Number of lanes below this one in mask m.
__device__ __forceinline__ int lane_prefix(uint64_t m) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Writes the lanes' pending candidates with one LDS atomic for the whole
// wave: records go to the LDS staging buffer, past its end to global memory.
// E.width is the lane's own width. All lanes of the wave must call it.
template <int NP>
__device__ __forceinline__ void emit_batch(const Pending (&p)[NP], const Emitter& E, int lane) {
  int off[NP];
  int tot = 0;
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const uint64_t m = ballot(p[k].f);
    off[k] = tot + lane_prefix(m);
    tot += popc(m);
  }
  if (tot == 0) return;
  uint32_t base = 0;
  if (lane == 0) base = atomicAdd(E.cbuf_n, (uint32_t)tot);
  base = (uint32_t)readfirst((int)base);
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    if (p[k].f) {
      const uint32_t slot = base + (uint32_t)off[k];
      const sps_cand c = make_cand(E, p[k].i, p[k].q);
      if (slot < (uint32_t)kCbuf) E.cbuf[slot] = c;
      else emit_global(E, c);
    }
  }
}

// A 64-position group's run summary, packed for LDS: x = flags | head best
// lane << 8 | tail best lane << 16, y = head S, z = tail S, w = MAD of the
// group's centre block (the group's S/N denominator is K * MAD * sqrt(w)).
// M: above lanes, V: valid lanes (contiguous). Runs touching neither end of
// the valid lanes are emitted here; `full_best`/`full_lane` is the best of
// all valid lanes (used when every valid lane is above).
__device__ __forceinline__ uint4 group_pack(uint64_t M, uint64_t V, int S, int mad, double den, int i0, int lane,
                                            int full_best, const Emitter& E) {
  if (!V) return make_uint4(0u, 0u, 0u, (uint32_t)mad);
  if (!M) return make_uint4((uint32_t)kNonEmpty, 0u, 0u, (uint32_t)mad);
  if (M == V) {
    const int bl = ctz(ballot(((V >> lane) & 1ull) && S == full_best));
    return make_uint4((uint32_t)(kNonEmpty | kFull | kHead) | ((uint32_t)bl << 8), (uint32_t)full_best, 0u,
                      (uint32_t)mad);
  }
  uint32_t flags = kNonEmpty;
  int hl = 0, tl = 0, hS = 0, tS = 0;
  const int fv = ctz(V), lv = msb(V);
  // runs touching neither end: lane k collects the k-th one (at most 32),
  // divided and written together after the loop
  int pi = 0, pS = 0, np = 0;
  uint64_t m = M;
  while (m) {
    const int a = ctz(m);
    const uint64_t gap = ~m & (~0ull << a);
    const int b = gap ? ctz(gap) : 64;
    const uint64_t run = (b == 64 ? ~0ull : ((1ull << b) - 1ull)) & (~0ull << a);
    int bs, bl;
    run_best(run, S, lane, bs, bl);
    if (a == fv) { flags |= kHead; hl = bl; hS = bs; }
    else if (b - 1 == lv) { flags |= kTail; tl = bl; tS = bs; }
    else {
      const bool mine = lane == np;
      pi = mine ? i0 + bl : pi;
      pS = mine ? bs : pS;
      ++np;
    }
    m &= ~run;
  }
  if (np) {
    Pending p[1];
    p[0].f = lane < np;
    p[0].i = pi;
    p[0].q = (double)pS / den;
    emit_batch(p, E, lane);
  }
  return make_uint4(flags | ((uint32_t)hl << 8) | ((uint32_t)tl << 16), (uint32_t)hS, (uint32_t)tS, (uint32_t)mad);
}


// One level of the segmented max-scan in step_fold: unless a run starts in
// the lanes this one already covers, take the best of the lanes D further
// back (earlier positions win ties).
template <int D>
__device__ __forceinline__ void scan_level(double& q, int& qi, int& s, int& fs) {
  const double pq = row_up<D>(0.0, q);
  const int pi = row_up<D>(0, qi), ps = row_up<D>(1, s), pfs = row_up<D>(0, fs);
  const bool take = !s && !(q > pq);
  q = take ? pq : q;
  qi = take ? pi : qi;
  fs = s ? fs : pfs;
  s |= ps;
}

// Combines the 16 group summaries held by each row of 16 lanes (lane k =
// group k, in window-end order; at most the leading and trailing groups of a
// row are empty) into the row's summary, and returns in pe[0], pe[1] the runs
// that close inside the row without touching its ends. On return lane 0 of
// each row holds the row summary in (fl, hi, hq, ti, tq).
//
// A group contributes up to two pieces of runs: its head piece (the run at
// its start, or the whole group when full) and its tail piece. The tail piece
// of group k-1 (or the whole group when full) joins the head piece of group k
// when both are above at the junction. The best of the run leaving each group
// at its end is a segmented max-scan over the groups (a new segment wherever
// the group is not full or does not join the one before), carrying whether
// that run began at the row start.
__device__ __forceinline__ void step_fold(int& fl, int& hi, double& hq, int& ti, double& tq, int k, Pending (&pe)[3]) {
  const bool ne = fl & kNonEmpty, F = fl & kFull, H = fl & kHead, T = fl & kTail;
  const bool eo = F || T;  // above at the group end
  // (lane exchanges run in every lane: never on the right of && or ||, which
  // would run them only where the left side holds)
  const int eo_prev = row_up<1>(0, (int)eo);
  const int ne_prev = row_up<1>(0, (int)ne), ne_next = row_down<1>(0, (int)ne);
  const bool C = H & (eo_prev != 0);                // joins the run of group k-1
  const bool Cn = row_down<1>(0, (int)C) != 0;      // group k+1 joins this one
  const bool first = ne & (ne_prev == 0);
  const bool last = ne & (ne_next == 0);
  // run leaving each group: best (q at qi) and whether it began at the row start
  double q = F ? hq : tq;
  int qi = F ? hi : ti;
  int s = !(F && C);
  int fs = first && F;
  scan_level<1>(q, qi, s, fs);
  scan_level<2>(q, qi, s, fs);
  scan_level<4>(q, qi, s, fs);
  scan_level<8>(q, qi, s, fs);
  // head piece of a group that is not full: the run closes inside the group
  const double oq = row_up<1>(0.0, q);
  const int oi = row_up<1>(0, qi), ofs = row_up<1>(0, fs);
  const bool r1 = H && !F;
  const bool join = C && !(hq > oq);
  const double r1q = join ? oq : hq;
  const int r1i = join ? oi : hi;
  const bool r1fs = C ? ofs != 0 : first;
  // run leaving the group: closes at its end unless group k+1 joins it
  const bool r2 = eo && !Cn;
  pe[0].f = r1 && !r1fs;
  pe[0].i = r1i;
  pe[0].q = r1q;
  pe[1].f = r2 && !last && !fs;
  pe[1].i = qi;
  pe[1].q = q;
  // the run from the row start ends in exactly one lane (if the first group
  // starts above); the run reaching the row end leaves the last group
  const bool hl = (r1 && r1fs) || (r2 && fs);
  const int hsrc = max(row_max(hl ? (int)lane_id() : -1), 0);
  const int tsrc = max(row_max(last ? (int)lane_id() : -1), 0);
  const double hv_q = (r1 && r1fs) ? r1q : q;
  const int hv_i = (r1 && r1fs) ? r1i : qi;
  const double rhq = lane_read(hv_q, hsrc), rtq = lane_read(q, tsrc);
  const int rhi = lane_read(hv_i, hsrc), rti = lane_read(qi, tsrc);
  const int bits = row_or((ne ? 1 : 0) | ((ne && !F) ? 2 : 0) | ((first && H) ? 4 : 0) | ((last && eo) ? 8 : 0));
  const bool rne = bits & 1, full = rne && !(bits & 2);
  fl = !rne ? 0 : (kNonEmpty | (full ? (kFull | kHead) : (((bits & 4) ? kHead : 0) | ((bits & 8) ? kTail : 0))));
  hi = rhi;
  hq = rhq;
  ti = rti;
  tq = rtq;
}

// Window ends of width w in a step start (64 - ceil(w/2) mod 64) mod 64
// before the step, so that every 64-lane group shares one centre block.
__device__ __forceinline__ int group_shift(int w) {
  const int sub = w - (w >> 1);
  return (64 - (sub & 63)) & 63;
}

// NW > 0: the number of widths is a compile-time constant (fast pass unrolled);
// NW == 0: any number of widths.
//
// Step c has four phases separated by three barriers:
//   A  write P of step c into the ring; bounds for step c's centre blocks
//   B  fast pass over step c (summaries of groups above for sure); residuals
//      and wave scan of step c+1; flush slot for the candidates staged
//      during step c-1
//   C  copy those candidates out; run pass over step c's other flagged
//      groups: one packed summary per (width, 64-position group) into LDS
//   D  each flagged width's 16 group summaries are combined by a segmented
//      scan in one row of 16 lanes and folded into the width's carried run
//      (no barrier before the next A)
// Samples, medians and MADs are fetched one step ahead of their use.
// The prefix-sum ring of a detection workgroup (32 KB of its ~40 KB of LDS).
// One array per kernel, whoever asks: the fused batch kernel keeps its
// statistics histograms in it before the workgroup turns to detection.
__device__ __forceinline__ uint32_t* detect_ring() {
  __shared__ uint32_t ring[kRing];
  return ring;
}

template <int NW, bool VIRT>
__device__ __forceinline__ void detect_body(const DetectArgs& A, const int task) {
  const int nw = NW > 0 ? NW : A.nw;
  uint32_t* const ring = detect_ring();
  __shared__ int32_t tlo[kMaxWidths][kGroups];
  __shared__ int32_t thi[kMaxWidths][kGroups];  // S > thi: above for sure (INT_MAX: never)
  __shared__ int32_t tmad[kMaxWidths][kGroups];
  __shared__ uint4 gsum[kMaxWidths][kGroups];
  __shared__ RunSum carry[kMaxWidths];
  __shared__ double s_sqw[kMaxWidths];
  __shared__ sps_cand cbuf[2][kCbuf];
  __shared__ __align__(16) uint32_t wtot[2][4];
  __shared__ uint32_t step_mask, flush_n, flush_base;
  __shared__ uint32_t cbuf_n[2];

  const int tid = threadIdx.x, lane = lane_id();
  const int wave = readfirst(tid >> 6);
  const int row = task / A.nseg;
  const int seg = task - row * A.nseg;
  const int N = A.N;
  const int s0 = A.seg_base + seg * A.seg_len;
  const int s1 = min(N, s0 + A.seg_len);
  // virtual sample t: t < Hx from the history row, else x row at t - Hx
  const float* xr = A.x + (int64_t)row * A.ld - (VIRT ? A.Hx : 0);
  const float* hr = VIRT ? A.hist + (int64_t)row * A.ldh : nullptr;
  const int32_t* medr = A.med + (int64_t)row * A.nblocks;
  const int32_t* madr = A.mad + (int64_t)row * A.nblocks;
  const int emax = min(s1 - s0 + A.maxw - 1, N - s0);  // last window end needed
  const int nsteps = (emax + 64) / kC + 1;              // + group shift headroom
  const bool vec = ((reinterpret_cast<uintptr_t>(A.x + (int64_t)row * A.ld) & 15u) == 0) &&
                   (!VIRT || ((reinterpret_cast<uintptr_t>(hr) & 15u) == 0));
  const int tmin = A.tmin ? *A.tmin : 0;
  const uint32_t dm = (uint32_t)row + A.row_offset;
  const int e_row0 = readfirst(N - s0);  // E <= N - s0      <=> i <= N - w
  const int e_seg0 = readfirst(s1 - s0); // E < s1 - s0 + w  <=> i < s1
  // E >= e_lo0 and E >= tmin - s0 + w: window ends after e_first, starts at or after tmin
  const int e_lo00 = readfirst(A.e_first - s0), e_lo10 = readfirst(tmin - s0);

  // bound-table thread: (width tj, group tg)
  const bool tthr = tid < nw * kGroups;
  const int tj = tthr ? tid / kGroups : 0, tg = tid - tj * kGroups;
  const double tsq = tthr ? A.sqrtw[tj] : 1.0;
  const int tw = 1 << tj;
  const int tk0 = s0 - group_shift(tw) - (tw - (tw >> 1));  // centre of group 0, step 0
  const int32_t* wmadr = A.wmad ? A.wmad + (int64_t)row * A.nw : nullptr;
  auto fetch_mad = [&](int c) -> int {
    if (!tthr) return 0;
    // one scale per (row, width): positions outside the row are masked out
    if (wmadr) return wmadr[tj];
    const int k = ((tk0 + c * kC) >> 6) + tg;
    return (k >= 0 && k < A.nblocks) ? madr[k] : 0;
  };
  // samples s0 + c*kC + 4*tid + q of step c
  auto fetch = [&](int c, int& mk, float& f0, float& f1, float& f2, float& f3) {
    const int t0 = s0 + c * kC + 4 * tid;
    mk = 0; f0 = f1 = f2 = f3 = 0.f;
    if (t0 < N) {
      mk = medr[t0 >> 6];
      // a step never straddles the history end (both are multiples of 1024)
      const float* src = (VIRT && s0 + c * kC < A.Hx) ? hr : xr;
      if (vec && t0 + 3 < N) {
        const float4 v = *reinterpret_cast<const float4*>(src + t0);
        f0 = v.x; f1 = v.y; f2 = v.z; f3 = v.w;
      } else {
        f0 = src[t0];
        if (t0 + 1 < N) f1 = src[t0 + 1];
        if (t0 + 2 < N) f2 = src[t0 + 2];
        if (t0 + 3 < N) f3 = src[t0 + 3];
      }
    }
  };
  // residuals (zero past the row), local prefix and wave scan of step c
  uint32_t p0, p1, p2, p3, incl;
  auto prefix = [&](int c, int mk, float f0, float f1, float f2, float f3) {
    const int t0 = s0 + c * kC + 4 * tid;
    const int r0 = t0 < N ? (int)f0 - mk : 0;
    const int r1 = t0 + 1 < N ? (int)f1 - mk : 0;
    const int r2 = t0 + 2 < N ? (int)f2 - mk : 0;
    const int r3 = t0 + 3 < N ? (int)f3 - mk : 0;
    p0 = (uint32_t)r0; p1 = p0 + (uint32_t)r1; p2 = p1 + (uint32_t)r2; p3 = p2 + (uint32_t)r3;
    incl = (uint32_t)wave_scan_incl((int)p3);
    if (lane == 63) wtot[c & 1][wave] = incl;
  };

  int nmk, cur_mad = fetch_mad(0), next_mad = 0;
  float nf0, nf1, nf2, nf3;
  fetch(0, nmk, nf0, nf1, nf2, nf3);
  prefix(0, nmk, nf0, nf1, nf2, nf3);
  if (nsteps > 1) fetch(1, nmk, nf0, nf1, nf2, nf3);
  if (tid < nw) {
    carry[tid] = rs_empty();
    s_sqw[tid] = A.sqrtw[tid];
  }
  if (tid == 0) { cbuf_n[0] = 0u; cbuf_n[1] = 0u; }
  uint32_t carryP = 0;  // P at the step's first sample
  __syncthreads();

  for (int c = 0; c < nsteps; ++c) {
    const int cC = c * kC;
    const int buf = c & 1;
    // The valid-range limits, opaque per step: otherwise the compiler hoists
    // every per-width limit derived from them out of the loop, and the
    // scalar registers they take are spilled and reloaded in every step.
    int e_row = e_row0, e_seg = e_seg0, e_lo0 = e_lo00, e_lo1 = e_lo10;
    asm volatile("" : "+s"(e_row), "+s"(e_seg), "+s"(e_lo0), "+s"(e_lo1));
    // ---- A: ring and bounds of step c
    {
      const uint4 wt = *reinterpret_cast<const uint4*>(&wtot[buf][0]);
      const uint32_t woff = (wave > 0 ? wt.x : 0u) + (wave > 1 ? wt.y : 0u) + (wave > 2 ? wt.z : 0u);
      const uint32_t tot = wt.x + wt.y + wt.z + wt.w;
      // P[E] = sum of r over the segment's first E samples; thread tid owns
      // E = cC + 4*tid + q, so every 64 consecutive E of a wave row are one group
      const uint32_t pb = carryP + woff + incl - p3;
      *reinterpret_cast<uint4*>(&ring[(cC + 4 * tid) & (kRing - 1)]) = make_uint4(pb, pb + p0, pb + p1, pb + p2);
      carryP += tot;
    }
    if (tthr) {
      const Bound bd = make_bound(cur_mad, tsq, A.theta);
      tlo[tj][tg] = bd.lo;
      thi[tj][tg] = bd.hi == INT_MAX ? INT_MAX : bd.hi - 1;
      tmad[tj][tg] = cur_mad;
    }
    if (c + 1 < nsteps) next_mad = fetch_mad(c + 1);
    if (tid == 0) step_mask = 0u;
    __syncthreads();  // BA

    // ---- B: flush slot for step c-1's candidates; fast pass; prefix of step c+1
    uint32_t fl_n = 0, fl_base = 0;
    if (tid == 0) {
      fl_n = min(cbuf_n[buf ^ 1], (uint32_t)kCbuf);
      cbuf_n[buf ^ 1] = 0u;
      if (fl_n) fl_base = atomicAdd(A.ncand, fl_n);
    }
    uint32_t fullmask;  // widths whose 4 groups of this wave are full runs (summaries written)
    // interior step: every position of every width is valid, no masks needed
    const bool clean = cC - 64 >= max(A.maxw, max(e_lo0, e_lo1 + A.maxw)) &&
                       cC + kC - 1 <= min(e_seg, e_row - A.maxw);
    {
      uint32_t flagged = 0u;
      fullmask = 0u;
      auto fast = [&](auto CLEAN) {
        // widths below 8: lane l reads window end l of each of the wave's 4 groups
        int cur_shift = -1;
        uint32_t pe[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          if (j >= nw) break;
          const int w = 1 << j, sh = group_shift(w);
          const int eg = cC - sh + 256 * wave;
          if (sh != cur_shift) {
            cur_shift = sh;
#pragma unroll
            for (int q = 0; q < 4; ++q) pe[q] = ring[(eg + 64 * q + lane) & (kRing - 1)];
          }
          const int4 T4 = *reinterpret_cast<const int4*>(&tlo[j][4 * wave]);
          uint64_t acc = 0ull;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int e0 = eg + 64 * q;
            const int S = (int)(pe[q] - ring[(e0 - w + lane) & (kRing - 1)]);
            const int T = q == 0 ? T4.x : q == 1 ? T4.y : q == 2 ? T4.z : T4.w;
            const uint64_t hit = ballot(S > T);
            if (CLEAN) {
              acc |= hit;
            } else {
              const int vhi = min(e_seg + w - 1, e_row);
              const int vlo = max(w, max(e_lo0, e_lo1 + w));
              acc |= hit & lane_range(vlo - e0, vhi - e0);
            }
          }
          flagged |= acc ? (1u << j) : 0u;
        }
        // widths 8 and up: the group shift is a multiple of 4, so lane l reads
        // window ends 4l .. 4l+3 of the wave's 256 with one 16-byte LDS read
        // (group l / 16)
        int cur_sh4 = -1;
        uint4 pe4 = make_uint4(0u, 0u, 0u, 0u);
        const int gq = lane >> 4;
#pragma unroll
        for (int j = 3; j < (NW > 0 ? NW : kMaxWidths); ++j) {
          if (NW == 0 && j >= nw) break;
          const int w = 1 << j, sh = group_shift(w);
          const int eg = cC - sh + 256 * wave;
          const int e4 = eg + 4 * lane;
          if (sh != cur_sh4) {
            cur_sh4 = sh;
            pe4 = *reinterpret_cast<const uint4*>(&ring[e4 & (kRing - 1)]);
          }
          const uint4 pw4 = *reinterpret_cast<const uint4*>(&ring[(e4 - w) & (kRing - 1)]);
          const int T = tlo[j][4 * wave + gq];
          int d0 = (int)(pe4.x - pw4.x), d1 = (int)(pe4.y - pw4.y);
          int d2 = (int)(pe4.z - pw4.z), d3 = (int)(pe4.w - pw4.w);
          if (!CLEAN) {
            const int vhi = min(e_seg + w - 1, e_row);
            const int vlo = max(w, max(e_lo0, e_lo1 + w));
            d0 = (e4 >= vlo && e4 <= vhi) ? d0 : INT_MIN;
            d1 = (e4 + 1 >= vlo && e4 + 1 <= vhi) ? d1 : INT_MIN;
            d2 = (e4 + 2 >= vlo && e4 + 2 <= vhi) ? d2 : INT_MIN;
            d3 = (e4 + 3 >= vlo && e4 + 3 <= vhi) ? d3 : INT_MIN;
          }
          // one comparison of the largest of the four (no short-circuit: a
          // logical or lets the compiler split the load and branch)
          const int dm = max(max(d0, d1), max(d2, d3));
          const uint64_t hit = ballot(dm > T);
          flagged |= hit ? (1u << j) : 0u;
          if (CLEAN && hit == ~0ull) {
            // Every lane has a candidate: if every one of the wave's 256
            // positions is above for sure, its 4 groups are single full runs
            // and their summaries are written here (the run pass skips them).
            const int F = thi[j][4 * wave + gq];
            if (ballot(min(min(d0, d1), min(d2, d3)) > F) == ~0ull) {
              int rm = dm;  // group maximum, in every lane of the row
              rm = max_step<0xb1>(rm);
              rm = max_step<0x4e>(rm);
              rm = max_step<0x141>(rm);
              rm = max_step<0x140>(rm);
              // first position of the maximum within the group (0..63)
              const int kk = d0 == rm ? 0 : (d1 == rm ? 1 : (d2 == rm ? 2 : 3));
              int pos = dm == rm ? 4 * (lane & 15) + kk : 64;
              pos = min_step<0xb1>(pos);
              pos = min_step<0x4e>(pos);
              pos = min_step<0x141>(pos);
              pos = min_step<0x140>(pos);
              if ((lane & 15) == 0) {
                const int g = 4 * wave + gq;
                gsum[j][g] = make_uint4((uint32_t)(kNonEmpty | kFull | kHead) | ((uint32_t)pos << 8), (uint32_t)rm,
                                        0u, (uint32_t)tmad[j][g]);
              }
              fullmask |= 1u << j;
            }
          }
        }
      };
      if (clean) fast(std::true_type{});
      else fast(std::false_type{});
      if (flagged && lane == 0) atomicOr(&step_mask, flagged);
    }
    if (c + 1 < nsteps) {
      prefix(c + 1, nmk, nf0, nf1, nf2, nf3);
      if (c + 2 < nsteps) fetch(c + 2, nmk, nf0, nf1, nf2, nf3);
    }
    if (tid == 0) { flush_n = fl_n; flush_base = fl_base; }
    __syncthreads();  // BB

    // ---- C: copy out step c-1's candidates; run pass
    {
      const uint32_t n = flush_n, base = flush_base;
      for (uint32_t i = tid; i < n; i += 256)
        if (base + i < A.cap) A.cands[base + i] = cbuf[buf ^ 1][i];
    }
    const uint32_t smask = step_mask;
    const uint32_t rmask = smask & ~fullmask;
    for (int j = 0; j < nw; ++j) {
      if (!((rmask >> j) & 1u)) continue;
      const int w = 1 << j, sh = group_shift(w);
      const int eg = cC - sh + 256 * wave;
      const int vhi = min(e_seg + w - 1, e_row);
      const int vlo = max(w, max(e_lo0, e_lo1 + w));
      const double sqw = A.sqrtw[j];
      const Emitter em{cbuf[buf], &cbuf_n[buf], A.cands, A.ncand, A.cap, dm, (uint32_t)w, lane == 0,
                       A.sample_offset};
      const int4 LO = *reinterpret_cast<const int4*>(&tlo[j][4 * wave]);
      const int4 HI = *reinterpret_cast<const int4*>(&thi[j][4 * wave]);  // S > HI: above for sure
      const int4 MD = *reinterpret_cast<const int4*>(&tmad[j][4 * wave]);
      int S[4], best[4];
      bool in[4];
      uint64_t M[4], V[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = eg + 64 * q + lane;
        S[q] = (int)(ring[e & (kRing - 1)] - ring[(e - w) & (kRing - 1)]);
        const int lo = q == 0 ? LO.x : q == 1 ? LO.y : q == 2 ? LO.z : LO.w;
        const int hi = q == 0 ? HI.x : q == 1 ? HI.y : q == 2 ? HI.z : HI.w;
        const int mad = q == 0 ? MD.x : q == 1 ? MD.y : q == 2 ? MD.z : MD.w;
        bool ab = S[q] > hi;
        if (S[q] > lo && !ab) ab = (double)S[q] / ((kMadToSigma * (double)mad) * sqw) > A.theta;
        in[q] = ab;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        M[q] = ballot(in[q]);
        best[q] = in[q] ? S[q] : INT_MIN;
      }
      // (the per-lane flags are consumed above: masking them under the
      // branch below would make the compiler keep them as bytes in a VGPR)
      if (clean) {
#pragma unroll
        for (int q = 0; q < 4; ++q) V[q] = ~0ull;
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          V[q] = lane_range(vlo - eg - 64 * q, vhi - eg - 64 * q);
          M[q] &= V[q];
          best[q] = ((V[q] >> lane) & 1ull) ? best[q] : INT_MIN;
        }
      }
      wave_max4_u(best[0], best[1], best[2], best[3]);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int mad = q == 0 ? MD.x : q == 1 ? MD.y : q == 2 ? MD.z : MD.w;
        const uint4 pk = group_pack(M[q], V[q], S[q], mad, (kMadToSigma * (double)mad) * sqw,
                                    s0 + eg + 64 * q - w, lane, best[q], em);
        if (lane == 0) gsum[j][4 * wave + q] = pk;
      }
    }
    cur_mad = next_mad;
    __syncthreads();  // BC

    // ---- D: the 16 group summaries of each flagged width are combined in
    // one row of 16 lanes (four widths per wave; the wave that takes the
    // first four rotates with the step), then folded into the width's carried
    // run. Unflagged widths only close a run.
    {
      const int nflag = __popc(smask);
      const int r = lane >> 4, k = lane & 15;
      const int slot = 4 * ((wave + c) & 3) + r;
      if (4 * ((wave + c) & 3) < nflag) {
        const bool act = slot < nflag;
        // j = index of the slot-th set bit: the largest j with slot set bits below it
        int jb = 0;
#pragma unroll
        for (int st = 8; st > 0; st >>= 1)
          if (__popc(smask & ((1u << (jb + st)) - 1u)) <= slot) jb += st;
        const int j = act ? jb : 0;
        const int w = 1 << j, sh = group_shift(w);
        const uint4 pk = gsum[j][k];
        int fl = 0, hi = 0, ti = 0;
        double hq = 0.0, tq = 0.0;
        if (act) {
          const double den = (kMadToSigma * (double)(int)pk.w) * s_sqw[j];
          const int i0 = s0 + cC - sh + 64 * k - w;
          fl = (int)(pk.x & 15u);
          hi = i0 + (int)((pk.x >> 8) & 63u);
          ti = i0 + (int)((pk.x >> 16) & 63u);
          hq = (double)(int)pk.y / den;
          tq = (double)(int)pk.z / den;
        }
        const Emitter em{cbuf[buf], &cbuf_n[buf], A.cands, A.ncand, A.cap, dm, (uint32_t)w, true,
                         A.sample_offset};
        Pending pe[3];
        step_fold(fl, hi, hq, ti, tq, k, pe);
        // the row's step summary, folded into the width's carried run by lane 0 of the row
        const bool owner = act && k == 0;
        RunSum cj = rs_empty();
        if (owner) cj = carry[j];
        RunSum st;
        st.flags = fl;
        st.hi = hi;
        st.ti = ti;
        st.pad = 0;
        st.hq = hq;
        st.tq = tq;
        cj = rs_combine_p(cj, st, pe[2]);
        pe[2].f = pe[2].f && owner;
        if (owner) carry[j] = cj;
        emit_batch(pe, em, lane);
      }
    }
    for (int j = wave; j < nw; j += 4) {
      if ((smask >> j) & 1u) continue;
      const int w = 1 << j, sh = group_shift(w);
      const Emitter em{cbuf[buf], &cbuf_n[buf], A.cands, A.ncand, A.cap, dm, (uint32_t)w, lane == 0,
                       A.sample_offset};
      RunSum cj = carry[j];
      // nothing above for width j: a non-empty step closes an open run
      const int elo = max(cC - sh, max(w, max(e_lo0, e_lo1 + w)));
      const int ehi = min(cC - sh + kC - 1, min(e_seg + w - 1, e_row));
      if (elo <= ehi) {
        bool dirty = false;
        if (!(cj.flags & kNonEmpty)) {
          cj.flags = kNonEmpty;
          dirty = true;
        } else if (cj.flags & (kTail | kFull)) {
          RunSum below = rs_empty();
          below.flags = kNonEmpty;
          cj = rs_combine(cj, below, em);
          dirty = true;
        }
        if (dirty && lane == 0) carry[j] = cj;
      }
    }
  }

  __syncthreads();
  const int lb = (nsteps - 1) & 1;  // staging buffer of the last step
  for (int j = wave; j < nw; j += 4) {
    const RunSum cj = carry[j];
    const Emitter em{cbuf[lb], &cbuf_n[lb], A.cands, A.ncand, A.cap, dm, (uint32_t)(1 << j), lane == 0,
                     A.sample_offset};
    if (A.nseg == 1 && !A.keep_edges) rs_close(cj, em);
    else if (lane == 0) A.frag[((int64_t)row * nw + j) * A.nseg + seg] = cj;
  }
  __syncthreads();
  if (tid == 0) {
    const uint32_t n = min(cbuf_n[lb], (uint32_t)kCbuf);
    flush_n = n;
    flush_base = n ? atomicAdd(A.ncand, n) : 0u;
  }
  __syncthreads();
  for (uint32_t i = tid; i < flush_n; i += 256)
    if (flush_base + i < A.cap) A.cands[flush_base + i] = cbuf[lb][i];
}

}  // namespace

}  // namespace sps
