// sps_widthnorm.hip - per-width re-normalisation (Heimdall++ Section II-B,
// the normalisation stage read as one robust noise scale for every
// boxcar-filtered series): for every row and width w = 2^j, over the
// filtered series T_w = {S_w(i) : 0 <= i <= N - w}, S_w(i) = sum of r over
// [i, i + w), r_t = x_t - m_{floor(t/64)}, the lower median c_w (rank
// floor((n - 1) / 2) of n = N - w + 1 values) and MAD_w, the lower median of
// |S_w(i) - c_w|. Exact.
//
// Design (gfx950): one 1024-thread workgroup per row. The row is streamed in
// steps of 4096 samples; the prefix sums P of the residual of two steps live
// in an LDS ring, so every boxcar sum of every width is one difference
// P[E] - P[E - w] (uint32, wrapping; exact for |S| < 2^31). Each pass over
// the row evaluates all widths at once: pass 0 takes their minima and maxima;
// then exact selections, each by levels of 11-bit digits of the key's
// distance from the current lower bound (one 2048-bin LDS histogram per
// width): a level histograms the keys inside the current range, one wave per
// width finds the bin holding the wanted rank, and the range shrinks to that
// bin. A range of R values takes ceil(log2(R) / 11) levels (at most three),
// so the median takes one to three passes and the MAD as many again. Median
// keys are S with the sign bit flipped (unsigned order = signed order); MAD
// keys are |S - c_w| as uint32.
#include <climits>

#include "sps_internal.h"
#include "sps_wave.h"

namespace sps {

namespace {

constexpr int kWT = 1024;           // threads per workgroup
constexpr int kWaves = kWT / 64;
constexpr int kWStep = 4 * kWT;     // samples per step (4 per thread)
constexpr int kWRing = 2 * kWStep;  // prefix sums of two steps
constexpr int kWBits = 11;
constexpr int kWBins = 1 << kWBits; // histogram bins per width and level

__device__ __forceinline__ uint32_t absdiff_u(int a, int b) {
  return a >= b ? (uint32_t)a - (uint32_t)b : (uint32_t)b - (uint32_t)a;
}

__device__ __forceinline__ int bits_of(uint32_t r) { return r == 0u ? 0 : 32 - __clz((int)r); }

struct WidthShared {
  uint32_t ring[kWRing];
  uint32_t hist[kMaxWidths][kWBins];
  uint32_t wtot[kWaves];
  int32_t mn[kMaxWidths], mx[kMaxWidths];
  // selection state per width: lower bound of the key range, bucket shift of
  // the level (-1: finished or no positions), rank sought, result key
  uint32_t lo[kMaxWidths];
  int32_t sh[kMaxWidths];
  uint32_t rank[kMaxWidths];
  uint32_t res[kMaxWidths];
  int32_t cen[kMaxWidths];  // the median c_w
};

// Streams the row once; for every step and width calls f(j, S, valid) with
// the boxcar sums S[q] of the thread's four window ends E = E0 + q (position
// E - w), valid iff w <= E <= N.
template <int NW, class F>
__device__ __forceinline__ void stream_row(const WidthStatsArgs& A, const int row, WidthShared& sm, const int nw,
                                           F&& f) {
  const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
  const float* xr = A.x + (int64_t)row * A.ld;
  const int32_t* mr = A.med + (int64_t)row * A.nblocks;
  const int N = A.N;
  const int nsteps = N / kWStep + 1;  // window ends 0 .. N
  const bool vec = (reinterpret_cast<uintptr_t>(xr) & 15u) == 0;
  uint32_t carry = 0;
  for (int c = 0; c < nsteps; ++c) {
    const int t0 = c * kWStep + 4 * tid;
    int r0 = 0, r1 = 0, r2 = 0, r3 = 0;
    if (t0 < N) {
      const int m = mr[t0 >> 6];  // the four samples share one 64-sample block
      float f0, f1 = 0.f, f2 = 0.f, f3 = 0.f;
      if (vec && t0 + 3 < N) {
        const float4 v = *reinterpret_cast<const float4*>(xr + t0);
        f0 = v.x; f1 = v.y; f2 = v.z; f3 = v.w;
      } else {
        f0 = xr[t0];
        if (t0 + 1 < N) f1 = xr[t0 + 1];
        if (t0 + 2 < N) f2 = xr[t0 + 2];
        if (t0 + 3 < N) f3 = xr[t0 + 3];
      }
      r0 = (int)f0 - m;
      r1 = t0 + 1 < N ? (int)f1 - m : 0;
      r2 = t0 + 2 < N ? (int)f2 - m : 0;
      r3 = t0 + 3 < N ? (int)f3 - m : 0;
    }
    const uint32_t p0 = (uint32_t)r0, p1 = p0 + (uint32_t)r1, p2 = p1 + (uint32_t)r2, p3 = p2 + (uint32_t)r3;
    const uint32_t incl = (uint32_t)wave_scan_incl((int)p3);
    if (lane == 63) sm.wtot[wave] = incl;
    __syncthreads();
    uint32_t woff = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) {
      const uint32_t v = sm.wtot[k];
      woff += k < wave ? v : 0u;
      tot += v;
    }
    // P[E0 + q] = sum of r over the row's first E0 + q samples
    const uint32_t pb = carry + woff + incl - p3;
    const uint4 pe = make_uint4(pb, pb + p0, pb + p1, pb + p2);
    const int E0 = c * kWStep + 4 * tid;
    *reinterpret_cast<uint4*>(&sm.ring[E0 & (kWRing - 1)]) = pe;
    carry += tot;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      if (j >= nw) break;
      const int w = 1 << j;
      uint4 ps;
      if (w >= 4) {
        // E0 - w is a multiple of 4; when it is negative every end is invalid
        ps = *reinterpret_cast<const uint4*>(&sm.ring[(E0 - w) & (kWRing - 1)]);
      } else {
        ps.x = sm.ring[(E0 - w) & (kWRing - 1)];
        ps.y = sm.ring[(E0 + 1 - w) & (kWRing - 1)];
        ps.z = sm.ring[(E0 + 2 - w) & (kWRing - 1)];
        ps.w = sm.ring[(E0 + 3 - w) & (kWRing - 1)];
      }
      const int S[4] = {(int)(pe.x - ps.x), (int)(pe.y - ps.y), (int)(pe.z - ps.z), (int)(pe.w - ps.w)};
      const bool v[4] = {E0 >= w && E0 <= N, E0 + 1 >= w && E0 + 1 <= N, E0 + 2 >= w && E0 + 2 <= N,
                         E0 + 3 >= w && E0 + 3 <= N};
      f(j, S, v);
    }
    __syncthreads();  // the next step rewrites wtot and the older ring half
  }
}

// Adds the thread's keys in range to width j's histogram (equal neighbouring
// buckets merged into one atomic).
__device__ __forceinline__ void hist_keys(uint32_t* h, const uint32_t (&key)[4], const bool (&v)[4], uint32_t lo,
                                          int sh) {
  uint32_t prev = 0xFFFFFFFFu, cnt = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t d = key[q] - lo;
    const bool in = v[q] && key[q] >= lo && (d >> sh) < (uint32_t)kWBins;
    const uint32_t b = d >> sh;
    if (in) {
      if (b == prev) {
        ++cnt;
      } else {
        if (cnt) atomicAdd(&h[prev], cnt);
        prev = b;
        cnt = 1;
      }
    }
  }
  if (cnt) atomicAdd(&h[prev], cnt);
}

// One wave per active width: the bin of the histogram holding the wanted
// rank; the range shrinks to it (or the key is found), the histogram is
// cleared for the next level.
__device__ __forceinline__ void resolve_level(WidthShared& sm, const int nw) {
  const int wave = threadIdx.x >> 6, lane = lane_id();
  for (int j = wave; j < nw; j += kWaves) {
    const int sh = sm.sh[j];
    uint32_t* h = sm.hist[j];
    if (sh >= 0) {
      uint32_t b32[32];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const uint4 v = *reinterpret_cast<const uint4*>(&h[32 * lane + 4 * k]);
        b32[4 * k] = v.x; b32[4 * k + 1] = v.y; b32[4 * k + 2] = v.z; b32[4 * k + 3] = v.w;
      }
      uint32_t s = 0;
#pragma unroll
      for (int k = 0; k < 32; ++k) s += b32[k];
      const uint32_t incl = (uint32_t)wave_scan_incl((int)s);  // at most 2^31 keys per row
      const uint32_t rank = sm.rank[j];
      const uint64_t mk = ballot(incl > rank);  // the range holds more than rank keys
      const int L = mk ? ctz(mk) : 63;
      uint32_t r = rank - ((uint32_t)readlane((int)incl, L) - (uint32_t)readlane((int)s, L));
      // within lane L's 32 bins (evaluated in every lane, used from lane L)
      int bin = 31;
      bool found = false;
#pragma unroll
      for (int k = 0; k < 32; ++k) {
        const bool here = !found && r < b32[k];
        bin = here ? k : bin;
        found = found || here;
        r = (found || here) ? r : r - b32[k];
      }
      const int B = 32 * L + readlane(bin, L);
      const uint32_t rr = (uint32_t)readlane((int)r, L);
      if (lane == 0) {
        const uint32_t lo = sm.lo[j] + ((uint32_t)B << sh);
        if (sh == 0) {
          sm.res[j] = lo;
          sm.sh[j] = -1;
        } else {
          sm.lo[j] = lo;
          sm.rank[j] = rr;
          sm.sh[j] = sh > kWBits ? sh - kWBits : 0;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) *reinterpret_cast<uint4*>(&h[32 * lane + 4 * k]) = make_uint4(0u, 0u, 0u, 0u);
  }
}

template <int NW>
__global__ __launch_bounds__(kWT) void k_width_stats(WidthStatsArgs A) {
  __shared__ WidthShared sm;
  constexpr int NWU = NW > 0 ? NW : kMaxWidths;  // widths unrolled in the streaming loop
  const int row = blockIdx.x;
  const int tid = threadIdx.x;
  const int nw = NW > 0 ? NW : A.nw;
  const int N = A.N;
  for (int i = tid; i < kMaxWidths * kWBins; i += kWT) (&sm.hist[0][0])[i] = 0u;
  if (tid < kMaxWidths) {
    sm.mn[tid] = INT_MAX;
    sm.mx[tid] = INT_MIN;
  }
  __syncthreads();

  // pass 0: range of every filtered series
  {
    int mn[kMaxWidths], mx[kMaxWidths];
#pragma unroll
    for (int j = 0; j < kMaxWidths; ++j) {
      mn[j] = INT_MAX;
      mx[j] = INT_MIN;
    }
    stream_row<NWU>(A, row, sm, nw, [&](int j, const int (&S)[4], const bool (&v)[4]) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        mn[j] = v[q] ? min(mn[j], S[q]) : mn[j];
        mx[j] = v[q] ? max(mx[j], S[q]) : mx[j];
      }
    });
#pragma unroll
    for (int j = 0; j < kMaxWidths; ++j) {
      if (j >= nw) break;
      const int a = wave_min_u(mn[j]), b = wave_max_u(mx[j]);
      if (lane_id() == 0) {
        atomicMin(&sm.mn[j], a);
        atomicMax(&sm.mx[j], b);
      }
    }
  }
  __syncthreads();

  // median of each series: keys S ^ 0x80000000 in [key(min), key(max)]
  if (tid < nw) {
    const int j = tid, w = 1 << j;
    const int n = N - w + 1;
    if (n <= 0) {
      sm.sh[j] = -1;
      sm.res[j] = 0x80000000u;  // c_w = 0
    } else {
      const uint32_t lo = (uint32_t)sm.mn[j] ^ 0x80000000u, hi = (uint32_t)sm.mx[j] ^ 0x80000000u;
      sm.lo[j] = lo;
      sm.rank[j] = (uint32_t)((n - 1) >> 1);
      sm.sh[j] = max(0, bits_of(hi - lo) - kWBits);
    }
  }
  __syncthreads();
  for (int level = 0; level < 3; ++level) {
    bool any = false;
    for (int j = 0; j < nw; ++j) any = any || sm.sh[j] >= 0;
    if (!any) break;
    uint32_t lo[kMaxWidths];
    int sh[kMaxWidths];
#pragma unroll
    for (int j = 0; j < kMaxWidths; ++j) {
      lo[j] = j < nw ? sm.lo[j] : 0u;
      sh[j] = j < nw ? sm.sh[j] : -1;
    }
    stream_row<NWU>(A, row, sm, nw, [&](int j, const int (&S)[4], const bool (&v)[4]) {
      if (sh[j] < 0) return;
      const uint32_t key[4] = {(uint32_t)S[0] ^ 0x80000000u, (uint32_t)S[1] ^ 0x80000000u,
                               (uint32_t)S[2] ^ 0x80000000u, (uint32_t)S[3] ^ 0x80000000u};
      hist_keys(sm.hist[j], key, v, lo[j], sh[j]);
    });
    resolve_level(sm, nw);
    __syncthreads();
  }

  // MAD of each series: keys |S - c| in [0, max(max - c, c - min)]
  if (tid < nw) {
    const int j = tid, w = 1 << j;
    const int n = N - w + 1;
    const int c = (int)(sm.res[j] ^ 0x80000000u);
    sm.cen[j] = c;
    sm.lo[j] = 0u;
    sm.res[j] = 0u;  // MAD 0 for widths longer than the row
    if (n <= 0) {
      sm.sh[j] = -1;
    } else {
      const uint32_t r = max(absdiff_u(sm.mx[j], c), absdiff_u(c, sm.mn[j]));
      sm.rank[j] = (uint32_t)((n - 1) >> 1);
      sm.sh[j] = max(0, bits_of(r) - kWBits);
    }
  }
  __syncthreads();
  int cj[kMaxWidths];
#pragma unroll
  for (int j = 0; j < kMaxWidths; ++j) cj[j] = j < nw ? sm.cen[j] : 0;
  for (int level = 0; level < 3; ++level) {
    bool any = false;
    for (int j = 0; j < nw; ++j) any = any || sm.sh[j] >= 0;
    if (!any) break;
    uint32_t lo[kMaxWidths];
    int sh[kMaxWidths];
#pragma unroll
    for (int j = 0; j < kMaxWidths; ++j) {
      lo[j] = j < nw ? sm.lo[j] : 0u;
      sh[j] = j < nw ? sm.sh[j] : -1;
    }
    stream_row<NWU>(A, row, sm, nw, [&](int j, const int (&S)[4], const bool (&v)[4]) {
      if (sh[j] < 0) return;
      const uint32_t key[4] = {absdiff_u(S[0], cj[j]), absdiff_u(S[1], cj[j]), absdiff_u(S[2], cj[j]),
                               absdiff_u(S[3], cj[j])};
      hist_keys(sm.hist[j], key, v, lo[j], sh[j]);
    });
    resolve_level(sm, nw);
    __syncthreads();
  }
  if (tid < nw) {
    const int64_t o = (int64_t)row * nw + tid;
    A.center[o] = sm.cen[tid];
    // a MAD beyond INT32_MAX (half the series more than 2^31 from its median)
    // is reported as INT32_MAX
    A.mad[o] = (int32_t)min(sm.res[tid], (uint32_t)INT_MAX);
  }
}

}  // namespace

hipError_t launch_width_stats(const WidthStatsArgs& a, hipStream_t s) {
  if (a.rows <= 0) return hipSuccess;
  if (a.nw == kMaxWidths) hipLaunchKernelGGL((k_width_stats<kMaxWidths>), dim3(a.rows), dim3(kWT), 0, s, a);
  else hipLaunchKernelGGL((k_width_stats<0>), dim3(a.rows), dim3(kWT), 0, s, a);
  return hipGetLastError();
}

}  // namespace sps
