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

__device__ __forceinline__ sps_cand make_cand(const Emitter& E, int32_t sample, double q) {
  sps_cand c;
  c.sample = sample - E.soff;
  c.dm_idx = E.dm;
  c.width = E.width;
  c.snr = (float)q;
  return c;
}

// Global write of one record past the LDS staging (or without staging). The
// non-temporal store keeps the compiler from merging it with the LDS store
// into one slower flat store.
__device__ __forceinline__ void emit_global(const Emitter& E, const sps_cand& c) {
  const uint32_t slot = atomicAdd(E.ncand, 1u);
  if (slot < E.cap) {
    typedef int v4i __attribute__((ext_vector_type(4)));
    const v4i v = {c.sample, (int)c.dm_idx, (int)c.width, __float_as_int(c.snr)};
    __builtin_nontemporal_store(v, reinterpret_cast<v4i*>(E.cands + slot));
  }
}

__device__ __forceinline__ void emit(const Emitter& E, int32_t sample, double q) {
  if (!E.writer) return;
  const sps_cand c = make_cand(E, sample, q);
  if (E.cbuf) {
    const uint32_t s = atomicAdd(E.cbuf_n, 1u);
    if (s < (uint32_t)kCbuf) {
      E.cbuf[s] = c;
      return;
    }
  }
  emit_global(E, c);
}

__device__ __forceinline__ RunSum rs_empty() {
  RunSum r;
  r.flags = 0; r.hi = 0; r.ti = 0; r.pad = 0; r.hq = 0.0; r.tq = 0.0;
  return r;
}

// true if the best (q1 at i1) beats (q2 at i2): larger S/N, earlier on ties.
__device__ __forceinline__ bool beats(double q1, int i1, double q2, int i2) {
  return (q1 > q2) | ((q1 == q2) & (i1 < i2));  // no short-circuit: no branches
}

// A candidate held back for a batched write: valid, sample, S/N.
struct Pending {
  bool f;
  int i;
  double q;
};

// Summary of range L followed immediately by range R. The run that ends at
// the junction (touching neither end of L+R) is returned in `out`. Written with
// selects on scalars (never on whole summaries, which would make the
// compiler select addresses and keep the summaries in scratch memory), so
// lanes holding different summaries combine without branching.
__device__ __forceinline__ RunSum rs_combine_p(const RunSum L, const RunSum R, Pending& out) {
  const int Lfl = L.flags, Rfl = R.flags;
  const int Lhi = L.hi, Lti = L.ti, Rhi = R.hi, Rti = R.ti;
  const double Lhq = L.hq, Ltq = L.tq, Rhq = R.hq, Rtq = R.tq;
  const bool Lne = Lfl & kNonEmpty, Rne = Rfl & kNonEmpty;
  const bool Lf = Lfl & kFull, Lh = Lfl & kHead, Lt = Lfl & kTail;
  const bool Rf = Rfl & kFull, Rh = Rfl & kHead, Rt = Rfl & kTail;
  // head: L's head run, extended through R's head run when L is full
  const bool hR = Lf && Rh && beats(Rhq, Rhi, Lhq, Lhi);
  int hi = hR ? Rhi : Lhi;
  double hq = hR ? Rhq : Lhq;
  // tail: through R when R is full (joined with L's tail), else R's tail
  const bool joinR = !Lf && Rf;
  const bool keepL = joinR && Lt && !beats(Rhq, Rhi, Ltq, Lti);
  int ti = keepL ? Lti : (joinR ? Rhi : Rti);
  double tq = keepL ? Ltq : (joinR ? Rhq : Rtq);
  int fl = kNonEmpty | ((Lf || Lh) ? kHead : 0) | ((Lf && Rf) ? kFull : 0) | ((joinR || (!Rf && Rt)) ? kTail : 0);
  // the run ending at the junction
  const bool junction = Lne && Rne && !Lf && !Rf && (Lt || Rh);
  const bool pickR = Rh && (!Lt || beats(Rhq, Rhi, Ltq, Lti));
  out.f = junction;
  out.i = pickR ? Rhi : Lti;
  out.q = pickR ? Rhq : Ltq;
  // an empty side leaves the other unchanged
  fl = !Lne ? Rfl : (!Rne ? Lfl : fl);
  hi = !Lne ? Rhi : (!Rne ? Lhi : hi);
  ti = !Lne ? Rti : (!Rne ? Lti : ti);
  hq = !Lne ? Rhq : (!Rne ? Lhq : hq);
  tq = !Lne ? Rtq : (!Rne ? Ltq : tq);
  RunSum o;
  o.flags = fl;
  o.hi = hi;
  o.ti = ti;
  o.pad = 0;
  o.hq = hq;
  o.tq = tq;
  return o;
}

// The same, emitting the junction run at once.
__device__ __forceinline__ RunSum rs_combine(const RunSum L, const RunSum R, const Emitter& E) {
  Pending p;
  const RunSum o = rs_combine_p(L, R, p);
  if (p.f) emit(E, p.i, p.q);
  return o;
}

// Runs touching the ends of a whole row are closed there.
__device__ void rs_close(const RunSum& s, const Emitter& E) {
  if (s.flags & kHead) emit(E, s.hi, s.hq);
  if (s.flags & kTail) emit(E, s.ti, s.tq);
}

}  // namespace
}  // namespace sps
