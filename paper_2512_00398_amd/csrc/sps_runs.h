// sps_runs.h - peak-detection run summaries shared by the fused and the
// per-stage kernels (Heimdall++ Section II-B, "Peak Detection": one candidate
// per run of positions above the S/N threshold, at its maximum).
#pragma once

#include <climits>

#include "sps_internal.h"

namespace sps {
namespace {

constexpr int kCbuf = 48;  // LDS candidate staging records per buffer

// The S/N test of one (centre block, width): den = (K * MAD) * sqrt(w);
// "S / den > theta" holds for S >= hi (when hi < INT_MAX), fails for
// S <= lo, and is decided by the double division in between. MAD = 0 (or a
// bound beyond the int32 range) gives lo = hi = INT_MAX: never above.
struct Bound {
  int32_t lo, hi;
  double den;
};

__device__ __forceinline__ Bound make_bound(int mad, double sqrtw, double theta) {
  Bound b;
  b.lo = INT_MAX;
  b.hi = INT_MAX;
  b.den = 1.0;
  if (mad > 0) {
    const double den = (kMadToSigma * (double)mad) * sqrtw;
    b.den = den;
    const double tt = theta * den;
    if (tt < 2147483648.0) {
      b.lo = (int)(floor(tt) - 1.0);
      const double hd = ceil(tt) + 1.0;
      b.hi = hd >= 2147483647.0 ? INT_MAX : (int)hd;
    }
  }
  return b;
}

__device__ __forceinline__ bool above(int S, const Bound& b, double theta) {
  return S > b.lo && ((S >= b.hi && b.hi != INT_MAX) || (double)S / b.den > theta);
}

struct Emitter {
  sps_cand* cbuf;       // LDS staging (null: write to global directly)
  uint32_t* cbuf_n;
  sps_cand* cands;
  uint32_t* ncand;
  uint32_t cap;
  uint32_t dm;
  uint32_t width;
  bool writer;          // the one thread that writes (lane 0 in wave code)
  int32_t soff;         // emitted sample = position - soff
};

__device__ __forceinline__ void emit(const Emitter& E, int32_t sample, int32_t S, double den) {
  if (!E.writer) return;
  sps_cand c;
  c.sample = sample - E.soff;
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

}  // namespace
}  // namespace sps
