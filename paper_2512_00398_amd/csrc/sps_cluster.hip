// sps_cluster.hip - candidate merging and clustering (Heimdall++, Section
// II-B "Candidate Merging and Clustering", Section III's analysis of that
// stage and the last step of Algorithm 1).
//
// Candidates a and b are linked when their samples differ by at most
// time_tol, their DM indices by at most dm_tol and their log2 widths by at
// most width_tol; clusters are the connected components of the links, each
// reported by its member of largest S/N (equal S/N: smallest dm, width,
// sample) with its member count and extents.
//
// The paper's point about this stage is that all-pairs comparison is
// quadratic and scattered. Here the candidates are first bucketed by (time,
// DM) cell with a counting sort (cells at least time_tol + 1 samples and
// dm_tol + 1 trials wide, so linked candidates are in the same or adjacent
// cells) and gathered into bucket order; each candidate is then compared only
// with the candidates of its own cell and of the four neighbouring cells that
// follow it, read contiguously. Components are found by lock-free union-find on the bucketed
// positions (a root is always the smallest position of its tree; hooking a
// root under a smaller one is a compare-and-swap); per-root atomics then
// collect the best member, the count and the extents.
#include <climits>

#include "sps_internal.h"
#include "sps_wave.h"

namespace sps {

namespace {

__device__ __forceinline__ int ld_relaxed(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_relaxed(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x's tree, halving the path on the way (parent[v] <= v always).
__device__ int find_root(int* parent, int x) {
  int cur = ld_relaxed(&parent[x]);
  if (cur == x) return x;
  int prev = x;
  int next;
  while (cur > (next = ld_relaxed(&parent[cur]))) {
    st_relaxed(&parent[prev], next);
    prev = cur;
    cur = next;
  }
  return cur;
}

// Joins the trees of a and b: the larger root is hooked under the smaller.
__device__ void unite(int* parent, int a, int b) {
  int ra = find_root(parent, a), rb = find_root(parent, b);
  while (ra != rb) {
    const int hi = ra > rb ? ra : rb, lo = ra > rb ? rb : ra;
    const int old = atomicCAS(&parent[hi], hi, lo);
    if (old == hi) return;
    // hi was hooked elsewhere meanwhile: retry from the current roots
    ra = find_root(parent, hi == ra ? old : ra);
    rb = find_root(parent, hi == rb ? old : rb);
  }
}

__device__ __forceinline__ int log2w(uint32_t w) { return 31 - __clz((int)w); }

// Number of lanes below this one in mask m.
__device__ __forceinline__ int lanes_below(uint64_t m) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Positions per workgroup of the kernels that claim shared counters once per
// workgroup (the range and the output slots: same-address atomics from every
// wave would serialise).
constexpr int kChunks = 16;
constexpr int kSpan = 256 * kChunks;

__global__ __launch_bounds__(256) void k_cluster_init(const sps_cand* c, uint32_t n, ClusterScratch s) {
  __shared__ int red[4][4];
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  int smin = INT_MAX, smax = INT_MIN, dmin = INT_MAX, dmax = INT_MIN;
  for (int k = 0; k < kChunks; ++k) {
    const uint32_t i = blockIdx.x * kSpan + k * 256 + threadIdx.x;
    if (i < n) {
      const sps_cand a = c[i];
      smin = min(smin, a.sample);
      smax = max(smax, a.sample);
      dmin = min(dmin, (int)a.dm_idx);
      dmax = max(dmax, (int)a.dm_idx);
      s.parent[i] = (int)i;
      s.members[i] = 0u;
      s.snrbits[i] = 0u;
      s.slo[i] = INT_MAX;
      s.shi[i] = INT_MIN;
      s.dlo[i] = UINT_MAX;
      s.dhi[i] = 0u;
      s.tie[i] = ~0ull;
    }
  }
  // sample and DM ranges: one atomic per workgroup and value
  smin = wave_min_u(smin);
  smax = wave_max_u(smax);
  dmin = wave_min_u(dmin);
  dmax = wave_max_u(dmax);
  if (lane == 0) {
    red[0][wave] = smin;
    red[1][wave] = smax;
    red[2][wave] = dmin;
    red[3][wave] = dmax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicMin(&s.geo[0], min(min(red[0][0], red[0][1]), min(red[0][2], red[0][3])));
    atomicMax(&s.geo[1], max(max(red[1][0], red[1][1]), max(red[1][2], red[1][3])));
    atomicMin(&s.geo[4], min(min(red[2][0], red[2][1]), min(red[2][2], red[2][3])));
    atomicMax(&s.geo[5], max(max(red[3][0], red[3][1]), max(red[3][2], red[3][3])));
  }
}

__global__ void k_cluster_fill(ClusterScratch s) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kClusterCells + 2) s.count[i] = 0u;
  if (i == 0) {
    s.geo[0] = INT_MAX;
    s.geo[1] = INT_MIN;
    s.geo[4] = INT_MAX;
    s.geo[5] = INT_MIN;
  }
}

// Cell sizes: at least dm_tol + 1 trials and time_tol + 1 samples, and large
// enough that all cells fit in kClusterCells. geo: [0, 1] sample range, [2]
// time cell width, [3] DM cells per time row, [4, 5] DM range, [6] DM cell
// width, [7] time rows (rows x DM cells <= kClusterCells).
__global__ void k_cluster_geometry(int time_tol, int dm_tol, ClusterScratch s) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const int64_t tlo = s.geo[0], thi = s.geo[1], dlo = s.geo[4], dhi = s.geo[5];
  const int64_t trange = thi >= tlo ? thi - tlo + 1 : 1, drange = dhi >= dlo ? dhi - dlo + 1 : 1;
  // at most a quarter of the cells across DM, so that at least four time rows
  // fit (a time cell width capped at INT_MAX still covers the int32 range)
  int64_t cd = (int64_t)dm_tol + 1;
  const int64_t dneed = (drange + kClusterCells / 4 - 1) / (kClusterCells / 4);
  if (cd < dneed) cd = dneed;
  const int64_t nd = (drange + cd - 1) / cd;
  const int64_t nt_max = kClusterCells / nd;
  int64_t cw = (int64_t)time_tol + 1;
  const int64_t tneed = (trange + nt_max - 1) / nt_max;
  if (cw < tneed) cw = tneed;
  s.geo[2] = (int)(cw > INT_MAX ? INT_MAX : cw);
  s.geo[3] = (int)nd;
  s.geo[6] = (int)cd;
  s.geo[7] = (int)((trange + cw - 1) / cw);
}

// Cell of a candidate and its (time, DM) cell coordinates.
__device__ __forceinline__ uint32_t cell_of(const ClusterScratch& s, int sample, uint32_t dm, int& ct, int& cd) {
  ct = (int)(((int64_t)sample - s.geo[0]) / s.geo[2]);
  cd = (int)(((int64_t)dm - s.geo[4]) / s.geo[6]);
  return (uint32_t)ct * (uint32_t)s.geo[3] + (uint32_t)cd;
}

__device__ __forceinline__ uint32_t cell_of(const ClusterScratch& s, const sps_cand& a) {
  int ct, cd;
  return cell_of(s, a.sample, a.dm_idx, ct, cd);
}

__global__ void k_cluster_count(const sps_cand* c, uint32_t n, ClusterScratch s) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) atomicAdd(&s.count[cell_of(s, c[i])], 1u);
}

// Exclusive prefix sums of count[0 .. kClusterCells + 2), in place, in three
// passes: 1024 entries per workgroup, then the workgroup totals, then the
// offsets added back.
constexpr int kScanTile = 1024;
constexpr int kScanTiles = (kClusterCells + 2 + kScanTile - 1) / kScanTile;

__global__ __launch_bounds__(256) void k_scan_tiles(ClusterScratch s) {
  __shared__ uint32_t wsum[4];
  const int t = threadIdx.x, lane = lane_id(), wave = t >> 6;
  const int base = blockIdx.x * kScanTile + 4 * t;
  uint32_t v[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) v[q] = base + q < kClusterCells + 2 ? s.count[base + q] : 0u;
  const uint32_t own = v[0] + v[1] + v[2] + v[3];
  const uint32_t incl = (uint32_t)wave_scan_incl((int)own);
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  uint32_t off = 0;
  for (int w = 0; w < wave; ++w) off += wsum[w];
  uint32_t run = off + incl - own;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (base + q < kClusterCells + 2) s.count[base + q] = run;
    run += v[q];
  }
  if (t == 255) s.bsum[blockIdx.x] = off + incl;
}

__global__ __launch_bounds__(1024) void k_scan_totals(ClusterScratch s) {
  __shared__ uint32_t wsum[16];
  __shared__ uint32_t carry;
  const int t = threadIdx.x, lane = lane_id(), wave = t >> 6;
  if (t == 0) carry = 0u;
  __syncthreads();
  for (int b0 = 0; b0 < kScanTiles; b0 += 1024) {
    const uint32_t own = b0 + t < kScanTiles ? s.bsum[b0 + t] : 0u;
    const uint32_t incl = (uint32_t)wave_scan_incl((int)own);
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint32_t off = carry;
    for (int w = 0; w < wave; ++w) off += wsum[w];
    if (b0 + t < kScanTiles) s.bsum[b0 + t] = off + incl - own;
    __syncthreads();
    if (t == 1023) carry = off + incl;
    __syncthreads();
  }
}

__global__ void k_scan_add(ClusterScratch s) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kClusterCells + 2) {
    const uint32_t v = s.count[i] + s.bsum[i / kScanTile];
    s.count[i] = v;
    s.cursor[i] = v;
  }
}

// Records in bucket order.
__global__ void k_cluster_scatter(const sps_cand* c, uint32_t n, ClusterScratch s) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const sps_cand a = c[i];
    s.sorted[atomicAdd(&s.cursor[cell_of(s, a)], 1u)] = a;
  }
}

__device__ __forceinline__ bool linked(const sps_cand& a, int la, const sps_cand& b, int tt, int dt, int wt) {
  const int64_t ds = (int64_t)b.sample - a.sample;
  const int64_t dd = (int64_t)b.dm_idx - a.dm_idx;
  const int dw = log2w(b.width) - la;
  return (ds <= tt && ds >= -tt) && (dd <= dt && dd >= -dt) && (dw <= wt && dw >= -wt);
}

// Position p against the later positions of its own cell and every position
// of the cells (t, d+1), (t+1, d-1), (t+1, d), (t+1, d+1): each pair of
// neighbouring cells is visited from one side only.
__global__ void k_cluster_link(uint32_t n, int tt, int dt, int wt, ClusterScratch s) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const sps_cand a = s.sorted[p];
  int ct, cd;
  const uint32_t cell = cell_of(s, a.sample, a.dm_idx, ct, cd);
  const int nd = s.geo[3], nt = s.geo[7];
  const int la = log2w(a.width);
  auto join = [&](uint32_t q) {
    if (ld_relaxed(&s.parent[p]) == ld_relaxed(&s.parent[q])) return;  // same tree, nothing to look up
    unite(s.parent, (int)p, (int)q);
  };
  // cells are numbered row by row (time), DM cells within a row: a run of
  // neighbouring DM cells is one contiguous range of positions
  for (uint32_t q = p + 1, e = s.count[cell + 1]; q < e; ++q)
    if (linked(a, la, s.sorted[q], tt, dt, wt)) join(q);
  if (cd + 1 < nd)
    for (uint32_t q = s.count[cell + 1], e = s.count[cell + 2]; q < e; ++q)
      if (linked(a, la, s.sorted[q], tt, dt, wt)) join(q);
  if (ct + 1 < nt) {
    const uint32_t r = (uint32_t)(ct + 1) * (uint32_t)nd;
    const uint32_t c0 = r + (uint32_t)(cd > 0 ? cd - 1 : 0), c1 = r + (uint32_t)(cd + 1 < nd ? cd + 1 : nd - 1);
    for (uint32_t q = s.count[c0], e = s.count[c1 + 1]; q < e; ++q)
      if (linked(a, la, s.sorted[q], tt, dt, wt)) join(q);
  }
}

// Per-root member count, largest S/N and extents. A cluster's members are
// mostly neighbours in bucket order, so lanes that share the root of the
// first pending lane are combined in the wave first (at most two such groups
// of four or more lanes); the remaining lanes add their own values.
__global__ void k_cluster_collect(uint32_t n, ClusterScratch s) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = lane_id();
  const bool valid = p < n;
  int r = -1;
  sps_cand a;
  a.sample = 0;
  a.dm_idx = 0u;
  a.width = 1u;
  a.snr = 0.f;
  if (valid) {
    r = find_root(s.parent, (int)p);  // trees no longer change; roots stay roots
    a = s.sorted[p];
  }
  const int q = (int)__float_as_uint(a.snr);  // S/N > 0: its bits order as the values
  bool done = !valid;
  for (int it = 0; it < 2; ++it) {
    const uint64_t pend = ballot(!done);
    if (!pend) break;
    const int leader = ctz(pend);
    const int rl = readlane(r, leader);
    const bool mine = !done && r == rl;
    const uint64_t grp = ballot(mine);
    if (popc(grp) < 4) break;
    const int gq = wave_max_u(mine ? q : 0);
    const int gslo = wave_min_u(mine ? a.sample : INT_MAX), gshi = wave_max_u(mine ? a.sample : INT_MIN);
    const int gdlo = wave_min_u(mine ? (int)a.dm_idx : INT_MAX), gdhi = wave_max_u(mine ? (int)a.dm_idx : -1);
    if (lane == leader) {
      atomicAdd(&s.members[rl], (uint32_t)popc(grp));
      atomicMax(&s.snrbits[rl], (uint32_t)gq);
      atomicMin(&s.slo[rl], gslo);
      atomicMax(&s.shi[rl], gshi);
      atomicMin(&s.dlo[rl], (uint32_t)gdlo);
      atomicMax(&s.dhi[rl], (uint32_t)gdhi);
    }
    done = done || mine;
  }
  if (!done) {
    atomicAdd(&s.members[r], 1u);
    atomicMax(&s.snrbits[r], (uint32_t)q);
    atomicMin(&s.slo[r], a.sample);
    atomicMax(&s.shi[r], a.sample);
    atomicMin(&s.dlo[r], a.dm_idx);
    atomicMax(&s.dhi[r], a.dm_idx);
  }
}

// (dm, log2 width, sample) in one key that orders as the tie-break does.
__device__ __forceinline__ unsigned long long tie_key(const sps_cand& a) {
  return ((unsigned long long)a.dm_idx << 37) | ((unsigned long long)log2w(a.width) << 32) |
         (unsigned long long)((uint32_t)a.sample ^ 0x80000000u);
}

__global__ void k_cluster_best(uint32_t n, ClusterScratch s) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int root = find_root(s.parent, (int)p);
  const sps_cand a = s.sorted[p];
  if (__float_as_uint(a.snr) == s.snrbits[root]) atomicMin(&s.tie[root], tie_key(a));
}

// One record per root; the workgroup claims its output slots with one atomic.
__global__ __launch_bounds__(256) void k_cluster_emit(uint32_t n, ClusterScratch s, sps_cluster_rec* out,
                                                      uint32_t* nout) {
  __shared__ uint32_t wcount[4];
  __shared__ uint32_t base;
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  uint32_t mine = 0u;
  for (int k = 0; k < kChunks; ++k) {
    const uint32_t p = blockIdx.x * kSpan + k * 256 + threadIdx.x;
    mine += (uint32_t)popc(ballot(p < n && ld_relaxed(&s.parent[p]) == (int)p));
  }
  if (lane == 0) wcount[wave] = mine;
  __syncthreads();
  if (threadIdx.x == 0) base = atomicAdd(nout, wcount[0] + wcount[1] + wcount[2] + wcount[3]);
  __syncthreads();
  uint32_t at = base;
  for (int v = 0; v < wave; ++v) at += wcount[v];
  for (int k = 0; k < kChunks; ++k) {
    const uint32_t p = blockIdx.x * kSpan + k * 256 + threadIdx.x;
    const bool root = p < n && ld_relaxed(&s.parent[p]) == (int)p;
    const uint64_t m = ballot(root);
    if (root) {
      const unsigned long long key = s.tie[p];
      sps_cluster_rec r;
      r.dm_idx = (uint32_t)(key >> 37);
      r.width = 1u << (uint32_t)((key >> 32) & 31u);
      r.sample = (int32_t)((uint32_t)key ^ 0x80000000u);
      r.snr = __uint_as_float(s.snrbits[p]);
      r.members = s.members[p];
      r.sample_lo = s.slo[p];
      r.sample_hi = s.shi[p];
      r.dm_lo = s.dlo[p];
      r.dm_hi = s.dhi[p];
      r.reserved = 0u;
      out[at + (uint32_t)lanes_below(m)] = r;
    }
    at += (uint32_t)popc(m);
  }
}

}  // namespace

hipError_t launch_cluster(const sps_cand* c, uint32_t n, int tt, int dt, int wt, const ClusterScratch& s,
                          sps_cluster_rec* out, uint32_t* nout, hipStream_t st) {
  const dim3 b(256);
  const dim3 gc((kClusterCells + 2 + 255) / 256);
  hipLaunchKernelGGL(k_cluster_fill, gc, b, 0, st, s);
  if (launch_zero_u32(nout, 1, st) != hipSuccess) return hipGetLastError();
  if (n > 0) {
    const dim3 gn((n + 255) / 256);
    const dim3 gw((n + kSpan - 1) / kSpan);
    hipLaunchKernelGGL(k_cluster_init, gw, b, 0, st, c, n, s);
    hipLaunchKernelGGL(k_cluster_geometry, dim3(1), dim3(64), 0, st, tt, dt, s);
    hipLaunchKernelGGL(k_cluster_count, gn, b, 0, st, c, n, s);
    hipLaunchKernelGGL(k_scan_tiles, dim3(kScanTiles), b, 0, st, s);
    hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(1024), 0, st, s);
    hipLaunchKernelGGL(k_scan_add, gc, b, 0, st, s);
    hipLaunchKernelGGL(k_cluster_scatter, gn, b, 0, st, c, n, s);
    hipLaunchKernelGGL(k_cluster_link, gn, b, 0, st, n, tt, dt, wt, s);
    hipLaunchKernelGGL(k_cluster_collect, gn, b, 0, st, n, s);
    hipLaunchKernelGGL(k_cluster_best, gn, b, 0, st, n, s);
    hipLaunchKernelGGL(k_cluster_emit, gw, b, 0, st, n, s, out, nout);
  }
  return hipGetLastError();
}

}  // namespace sps
