// sps_chain.h - the baseline and normalisation chain (Heimdall++, Section
// II-B): the device code behind k_block_stats, shared by the statistics
// kernels and the fused batch kernel. See sps_stats.hip for the design.
#pragma once

#include "sps_internal.h"
#include "sps_wave.h"

namespace sps {

namespace {

// Virtual row: samples t < Hx come from the stream history h, the rest from
// the input g (g[t - Hx]). VIRT = false: no history, t indexes g directly.
template <bool VIRT>
struct RowRef {
  const float* g;
  const float* h;
  int Hx;
  __device__ __forceinline__ float at(int t) const {
    if (VIRT) return *(t < Hx ? h + t : g + (t - Hx));  // one load from the selected address
    return g[t];
  }
  __device__ __forceinline__ int iat(int t) const { return (int)at(t); }
};

__device__ __forceinline__ uint32_t absdiff(int v, int m) {
  return v >= m ? (uint32_t)v - (uint32_t)m : (uint32_t)m - (uint32_t)v;
}

__device__ __forceinline__ void hist_add(uint32_t* H, uint32_t idx, uint32_t one) {
  // one = 1 (insert) or 0xFFFFFFFF (remove); the count lives in the idx&1 half
  atomicAdd(&H[idx >> 1], one << ((idx & 1u) << 4));
}

__device__ __forceinline__ int hist_get(const uint32_t* H, int idx) {
  return (int)((H[idx >> 1] >> ((idx & 1) << 4)) & 0xFFFFu);
}

template <int NB, bool VIRT>
struct Chain {
  uint32_t* H;        // this wave's NB/2 histogram words
  RowRef<VIRT> row;
  int L;
  int lane;
  int base;           // value of histogram bin 0
  int n;              // window size
  int m, cm;          // median, #{x < m}
  int d, cL, cU;      // MAD, #{x < m - d}, #{x < m + d + 1}
  bool raw;           // histogram not maintained (data too spread)
};

// Element of 0-based rank `rank` of the keys of samples [lo, hi):
// MODE 0 keys are x ^ 0x80000000 (order of int32 x), MODE 1 keys are |x - m|.
// Four passes over the window, 8 key bits each; H[0..255] serves as the
// digit histogram (callers rebuild or abandon the value histogram afterwards).
template <int MODE, bool VIRT>
__device__ uint32_t radix_select(uint32_t* H, const RowRef<VIRT>& row, int lo, int hi, int rank, int m, int lane) {
  uint32_t prefix = 0, pmask = 0;
  for (int shift = 24; shift >= 0; shift -= 8) {
    for (int i = lane; i < 256; i += 64) H[i] = 0;
    wave_lds_fence();
    for (int t0 = lo; t0 < hi; t0 += 64) {
      const int t = t0 + lane;
      if (t < hi) {
        const int v = row.iat(t);
        const uint32_t key = MODE == 0 ? ((uint32_t)v ^ 0x80000000u) : absdiff(v, m);
        if ((key & pmask) == prefix) atomicAdd(&H[(key >> shift) & 255u], 1u);
      }
    }
    wave_lds_fence();
    const int c0 = (int)H[4 * lane], c1 = (int)H[4 * lane + 1], c2 = (int)H[4 * lane + 2];
    const int c3 = (int)H[4 * lane + 3];
    const int s = c0 + c1 + c2 + c3;
    const int inc = wave_scan_incl(s);
    const int j = ctz(ballot(inc > rank));  // total count > rank, so some lane qualifies
    int r = rank - (readlane(inc, j) - readlane(s, j));
    const int d0 = readlane(c0, j), d1 = readlane(c1, j), d2 = readlane(c2, j);
    int dig = 4 * j;
    if (r >= d0) {
      r -= d0; ++dig;
      if (r >= d1) {
        r -= d1; ++dig;
        if (r >= d2) { r -= d2; ++dig; }
      }
    }
    rank = r;
    prefix |= (uint32_t)dig << shift;
    pmask |= 0xFFu << shift;
    wave_lds_fence();
  }
  return prefix;
}

// Recount the window [lo, hi) into a histogram whose bin 0 is `base`;
// returns #{x < base}.
template <int NB, bool VIRT>
__device__ int rebuild(Chain<NB, VIRT>& c, int lo, int hi, int base) {
  c.base = base;
  for (int i = c.lane; i < NB / 2; i += 64) c.H[i] = 0;
  wave_lds_fence();
  int below = 0;
  for (int t0 = lo; t0 < hi; t0 += 64) {
    const int t = t0 + c.lane;
    const bool ok = t < hi;
    const int v = ok ? c.row.iat(t) : 0;
    const uint32_t idx = (uint32_t)v - (uint32_t)base;
    if (ok && idx < (uint32_t)NB) hist_add(c.H, idx, 1u);
    below += popc(ballot(ok && v < base));
  }
  wave_lds_fence();
  c.raw = false;
  return below;
}

// Median and MAD from the whole histogram, given #{x < base}. Fails (returns
// false) when a needed quantile lies outside the histogram's range.
template <int NB, bool VIRT>
__device__ bool full_query(Chain<NB, VIRT>& c, int below) {
  const int rho = (c.n - 1) >> 1;
  if (below > rho) return false;
  int acc = below, m2 = 0, cm2 = 0;
  bool found = false;
  for (int i0 = 0; i0 < NB; i0 += 64) {
    const int h = hist_get(c.H, i0 + c.lane);
    const int inc = wave_scan_incl(h);
    const uint64_t mk = ballot(acc + inc > rho);
    if (mk) {
      const int j = ctz(mk);
      m2 = c.base + i0 + j;
      cm2 = acc + readlane(inc, j) - readlane(h, j);
      found = true;
      break;
    }
    acc += readlane(inc, 63);
  }
  if (!found) return false;
  // MAD: fold the histogram at m2; g(0) = h(m2), g(e) = h(m2 + e) + h(m2 - e).
  const int i2 = m2 - c.base;
  int acc_lo = 0, acc_hi = 0;
  for (int e0 = 0;; e0 += 64) {
    const int e = e0 + c.lane;
    const bool in_hi = i2 + e < NB, in_lo = i2 - e >= 0;
    const int ghi = in_hi ? hist_get(c.H, i2 + e) : 0;
    const int glo = (e > 0 && in_lo) ? hist_get(c.H, i2 - e) : 0;
    const int ihi = wave_scan_incl(ghi), ilo = wave_scan_incl(glo);
    const bool ok = in_hi && in_lo;
    const uint64_t okm = ballot(ok);
    const uint64_t mk = ballot(ok && acc_lo + acc_hi + ihi + ilo > rho);
    if (mk) {  // okm is a prefix of the lanes, so every e <= j was in range
      const int j = ctz(mk);
      c.m = m2;
      c.cm = cm2;
      c.d = e0 + j;
      c.cL = cm2 - (acc_lo + readlane(ilo, j));
      c.cU = cm2 + acc_hi + readlane(ihi, j);
      return true;
    }
    if (okm != ~0ull) return false;
    acc_lo += readlane(ilo, 63);
    acc_hi += readlane(ihi, 63);
  }
}

// Local query: new median within 31 values of the old one and new MAD within
// 31 of the old one (the usual case). Returns false when it cannot decide.
template <int NB, bool VIRT>
__device__ __forceinline__ bool fast_query(Chain<NB, VIRT>& c) {
  const int rho = (c.n - 1) >> 1;
  const int im = c.m - c.base, iL = c.m - c.d - c.base, iU = c.m + c.d + 1 - c.base;
  if (im - 32 < 0 || im + 32 > NB || iL - 32 < 0 || iU + 32 > NB) return false;
  const int lane = c.lane;
  const int h = hist_get(c.H, im - 32 + lane);
  const int hL = hist_get(c.H, iL - 32 + lane);
  const int hU = hist_get(c.H, iU - 32 + lane);
  const int inc = wave_scan_incl(h), incL = wave_scan_incl(hL), incU = wave_scan_incl(hU);
  const int lt = c.cm - readlane(inc, 31) + inc - h;  // #{x < m - 32 + lane}
  const uint64_t mk = ballot(lt + h > rho);
  if (!mk) return false;
  const int j = ctz(mk);
  const int ltj = readlane(lt, j);
  if (ltj > rho) return false;  // median below the window
  const int delta = j - 32;      // new median - old median
  const int ltL = c.cL - readlane(incL, 31) + incL - hL;  // #{x < (m - d) - 32 + lane}
  const int ltU = c.cU - readlane(incU, 31) + incU - hU;  // #{x < (m + d + 1) - 32 + lane}
  // lane tests d' = d + lane - 32 around the new median m + delta:
  // #{|x - m'| <= d'} = #{x < m' + d' + 1} - #{x < m' - d'}
  const int a = delta + 64 - lane, b = delta + lane;
  const int dp = c.d + lane - 32;
  const bool ok = a >= 0 && a < 64 && b >= 0 && b < 64 && dp >= 0;
  const int va = __shfl(ltL, a & 63, 64), vb = __shfl(ltU, b & 63, 64);
  const uint64_t okm = ballot(ok), fm = ballot(ok && vb - va > rho);
  if (!fm) return false;
  const int jj = ctz(fm);
  if (jj == ctz(okm) && readlane(dp, jj) > 0) return false;  // MAD may be smaller still
  c.m = c.m + delta;
  c.cm = ltj;
  c.d = readlane(dp, jj);
  c.cL = readlane(va, jj);
  c.cU = readlane(vb, jj);
  return true;
}

// Narrow local query (the common case): 16 bins around each of the three
// pivots, one DPP row (16 lanes) per pivot, one row-local prefix sum for all
// three. Row 0 finds the new median within [m - 8, m + 7]; row 3 lanes test
// MAD candidates d + t around it from rows 1 (lower pivot) and 2 (upper
// pivot). Returns false when the answer may lie outside these windows.
template <int NB, bool VIRT>
__device__ __forceinline__ bool narrow_query(Chain<NB, VIRT>& c) {
  const int rho = (c.n - 1) >> 1;
  const int im = c.m - c.base, iL = c.m - c.d - c.base, iU = c.m + c.d + 1 - c.base;
  if (iL - 8 < 0 || iU + 8 > NB) return false;  // im lies between them
  const int lane = c.lane, r = lane >> 4, k = lane & 15;
  // per-row selects written as a chain of two-way selects (a nested
  // conditional on scalar operands compiles to branches)
  int ib = iU;
  ib = r == 1 ? iL : ib;
  ib = r == 0 ? im : ib;
  const int h = hist_get(c.H, ib - 8 + k);
  const int inc = row_scan_incl(h);
  const int i0 = readlane(inc, 7), i1 = readlane(inc, 23), i2 = readlane(inc, 39);
  int cb = c.cU - i2;
  cb = r == 1 ? c.cL - i1 : cb;
  cb = r == 0 ? c.cm - i0 : cb;
  const int lt = cb + inc - h;  // #{x < pivot - 8 + k} in rows 0..2
  const uint64_t mk = ballot(lt + h > rho) & 0xFFFFull;
  if (!mk) return false;       // median above the window
  const int j = ctz(mk);
  const int ltj = readlane(lt, j);
  if (ltj > rho) return false;  // median below the window
  const int delta = j - 8;
  // row 3: lane tests d' = d + t, t = k - 8, around m' = m + delta:
  // #{|x - m'| <= d'} = #{x < pU + delta + t} - #{x < pL + delta - t}
  const int t = k - 8;
  const int kl = 8 + delta - t, ku = 8 + delta + t;
  const bool ok = r == 3 && kl >= 0 && kl < 16 && ku >= 0 && ku < 16 && c.d + t >= 0;
  const int va = __shfl(lt, 16 + (kl & 15), 64), vb = __shfl(lt, 32 + (ku & 15), 64);
  const uint64_t okm = ballot(ok), fm = ballot(ok && vb - va > rho);
  if (!fm) return false;        // MAD above the tested range
  const int jj = ctz(fm);
  const int dp = c.d + readlane(t, jj);
  if (jj == ctz(okm) && dp > 0) return false;  // MAD may be smaller still
  c.m = c.m + delta;
  c.cm = ltj;
  c.d = dp;
  c.cL = readlane(va, jj);
  c.cU = readlane(vb, jj);
  return true;
}

// Exact answer for window [lo, hi) from the samples themselves, then a
// histogram centred on the median when the data allow one.
template <int NB, bool VIRT>
__device__ void exact_block(Chain<NB, VIRT>& c, int lo, int hi) {
  const int rho = (c.n - 1) >> 1;
  const int m = (int)(radix_select<0, VIRT>(c.H, c.row, lo, hi, rho, 0, c.lane) ^ 0x80000000u);
  const uint32_t d = radix_select<1, VIRT>(c.H, c.row, lo, hi, rho, m, c.lane);
  c.m = m;
  c.d = (int)d;
  if (d < (uint32_t)(NB / 2 - 128)) {
    const int below = rebuild(c, lo, hi, m - NB / 2);
    const bool ok = full_query(c, below);  // succeeds: both quantiles are in range
    c.raw = !ok;
  } else {
    c.raw = true;
  }
}

// Median of up to 256 samples spread evenly over [lo, hi) (four per lane):
// a bitwise binary search on the order-preserving keys, counted with ballots.
template <bool VIRT>
__device__ int sample_median(const RowRef<VIRT>& row, int lo, int hi, int lane) {
  const int n = hi - lo;
  const int ns = n < 256 ? n : 256;
  uint32_t k[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = lane + 64 * q;
    k[q] = i < ns ? ((uint32_t)row.iat(lo + (int)(((int64_t)i * n) / ns)) ^ 0x80000000u) : 0xFFFFFFFFu;
  }
  const int rank = (ns - 1) >> 1;
  uint32_t p = 0;  // largest key with #{k < p} <= rank
  for (int b = 31; b >= 0; --b) {
    const uint32_t cand = p | (1u << b);
    int cnt = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) cnt += popc(ballot(k[q] < cand));
    if (cnt <= rank) p = cand;
  }
  return (int)(p ^ 0x80000000u);
}

// span_hi >= hi: the samples that centre the histogram are spread over
// [lo, span_hi) (the windows this chain will see, when the first is clipped).
template <int NB, bool VIRT>
__device__ void chain_init(Chain<NB, VIRT>& c, int lo, int hi, int span_hi) {
  // Centre the first histogram on the median of samples spread over the
  // whole window (a contiguous run of samples can sit far from it when the
  // data drift); for a window clipped at the row start, over the samples the
  // growing windows will take in, so that it need not be recentred (and the
  // window recounted) as they grow.
  const int g = sample_median(c.row, lo, span_hi, c.lane);
  const int below = rebuild(c, lo, hi, g - NB / 2);
  if (!full_query(c, below)) exact_block(c, lo, hi);
}

// Rare path: answer from the whole histogram, recentre it when the quantiles
// near its edges, or fall back to the exact select. Kept out of line so the
// unrolled block loop stays small.
template <int NB, bool VIRT>
__device__ void slow_block(Chain<NB, VIRT>& c, int lo, int hi) {
  // #{x < base} from the exact count below the old median
  const int im = c.m - c.base;
  int s = 0;
  for (int i0 = 0; i0 < im; i0 += 64) {
    const int i = i0 + c.lane;
    s += i < im ? hist_get(c.H, i) : 0;
  }
  const int below = c.cm - wave_sum_u(s);
  if (full_query(c, below)) {
    // keep the local queries' windows inside the histogram: recentre near an edge
    if (c.m - c.d - 96 < c.base || c.m + c.d + 97 > c.base + NB) {
      if (c.d < NB / 2 - 128) {
        const int b2 = rebuild(c, lo, hi, c.m - NB / 2);
        c.raw = !full_query(c, b2);
      }
    }
    return;
  }
  exact_block(c, lo, hi);
}

template <int NB, bool VIRT>
__device__ __forceinline__ void chain_step(Chain<NB, VIRT>& c, int lo, int hi, bool a_ok, int av, bool b_ok, int bv) {
  // lane masks of the entering (a) and leaving (b) samples; the counts below
  // AND raw comparison ballots with them (a comparison's ballot is its own
  // lane mask, a combined condition would be materialised and compared again)
  const uint64_t aM = ballot(a_ok), bM = ballot(b_ok);
  c.n += popc(aM) - popc(bM);
  if (c.raw) {
    exact_block(c, lo, hi);
    return;
  }
  const uint32_t ua = (uint32_t)av - (uint32_t)c.base, ub = (uint32_t)bv - (uint32_t)c.base;
  if (a_ok && ua < (uint32_t)NB) hist_add(c.H, ua, 1u);
  if (b_ok && ub < (uint32_t)NB) hist_add(c.H, ub, 0xFFFFFFFFu);
  const int pL = c.m - c.d, pU = c.m + c.d + 1;
  c.cm += popc(ballot(av < c.m) & aM) - popc(ballot(bv < c.m) & bM);
  c.cL += popc(ballot(av < pL) & aM) - popc(ballot(bv < pL) & bM);
  c.cU += popc(ballot(av < pU) & aM) - popc(ballot(bv < pU) & bM);
  wave_lds_fence();
  if (!narrow_query(c) && !fast_query(c)) slow_block(c, lo, hi);
}

// WPG chains (waves) per workgroup; LDS = WPG * NB * 2 bytes. Blocks
// [kb_first, nblocks) of every row are computed; windows never reach below
// the device value *tmin (the first sample of a stream). LEAD: the window
// reaches a.lead samples past its block (false: trailing, offset compiled out).
template <int NB, bool VIRT, bool LEAD>
__device__ __forceinline__ void stats_chain(const StatsArgs& a, const int chain, uint32_t* H, const int lane) {
  const int row = chain / a.nseg;
  const int seg = chain - row * a.nseg;
  // segment 0 has head_blocks blocks, the others seg_blocks each
  const int kb0 = a.kb_first + (seg == 0 ? 0 : a.head_blocks + (seg - 1) * a.seg_blocks);
  const int kb1 = min(a.nblocks, seg == 0 ? a.kb_first + a.head_blocks : kb0 + a.seg_blocks);
  const int N = a.N, L = a.L, lead = LEAD ? a.lead : 0;
  const int t0 = a.tmin ? *a.tmin : 0;
  Chain<NB, VIRT> c;
  c.H = H;
  c.row.g = a.x + (int64_t)row * a.ld;
  c.row.h = VIRT ? a.hist + (int64_t)row * a.ldh : nullptr;
  c.row.Hx = VIRT ? a.Hx : 0;
  c.L = L;
  c.lane = lane;
  int32_t* med = a.med + (int64_t)row * a.nblocks;
  int32_t* mad = a.mad + (int64_t)row * a.nblocks;

  // Block k's window is [max(t0, E_k - L), min(N, E_k)) with E_k = min(64k + 64, N) + lead:
  // from block k-1 to k the samples [min(N, E_{k-1}), min(N, E_k)) enter it and
  // [max(t0, E_{k-1} - L), max(t0, E_k - L)) leave it, at most 64 each.
  {
    const int E = min(kb0 * kStride + kStride, N) + lead;
    const int e = min(N, E), lo = max(t0, E - L);
    c.n = e - lo;
    chain_init(c, lo, e, min(N, max(e, lo + L)));
    if (lane == 0) { med[kb0] = c.m; mad[kb0] = c.d; }
  }

  // Samples entering / leaving the window at block kk, prefetched 4 blocks
  // ahead. Every lane loads (from a clamped in-row position) and unused lanes
  // are zeroed afterwards: loads skipped under a branch would leave the
  // compiler unsure how many are in flight, and it would then wait for all of
  // them, the prefetch included, before each block.
  auto fetch = [&](int kk, float& va, float& vb) {
    const int Ep = min(kk * kStride, N) + lead, E = min(kk * kStride + kStride, N) + lead;
    const int ep = min(N, Ep), e = min(N, E), lp = max(t0, Ep - L), l2 = max(t0, E - L);
    const float ra = c.row.at(min(ep + lane, N - 1)), rb = c.row.at(min(lp + lane, N - 1));
    va = (lane < e - ep) ? ra : 0.f;
    vb = (lane < l2 - lp) ? rb : 0.f;
  };
  float pa[4], pb[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) fetch(kb0 + 1 + j, pa[j], pb[j]);

  for (int k = kb0 + 1; k < kb1; k += 4) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int kk = k + j;
      const float va = pa[j], vb = pb[j];
      fetch(kk + 4, pa[j], pb[j]);
      if (kk < kb1) {
        const int Ep = min(kk * kStride, N) + lead, E = min(kk * kStride + kStride, N) + lead;
        const int ep = min(N, Ep), e = min(N, E), lp = max(t0, Ep - L), l2 = max(t0, E - L);
        chain_step(c, l2, e, lane < e - ep, (int)va, lane < l2 - lp, (int)vb);
        // every lane stores the same (wave-uniform) values: no branch around the stores
        med[kk] = c.m;
        mad[kk] = c.d;
      }
    }
  }
}

}  // namespace

}  // namespace sps
