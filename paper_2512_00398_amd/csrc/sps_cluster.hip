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
// quadratic and scattered. Here the candidates are first bucketed by time
// cell (cells at least time_tol + 1 samples wide, so linked candidates are in
// the same or adjacent cells) with a counting sort, and each candidate is
// compared only with the candidates of its own and the next cell, read
// contiguously. Components are found by lock-free union-find on the bucketed
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
    if (ra < rb) {
      const int t = ra;
      ra = rb;
      rb = t;
    }
    const int old = atomicCAS(&parent[ra], ra, rb);
    if (old == ra) return;
    ra = find_root(parent, old);
    rb = find_root(parent, rb);
  }
}

__device__ __forceinline__ int log2w(uint32_t w) { return 31 - __clz((int)w); }

__global__ void k_cluster_init(const sps_cand* c, uint32_t n, ClusterScratch s) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    atomicMin(&s.geo[0], c[i].sample);
    atomicMax(&s.geo[1], c[i].sample);
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

__global__ void k_cluster_fill(ClusterScratch s) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kClusterCells + 2) s.count[i] = 0u;
  if (i == 0) {
    s.geo[0] = INT_MAX;
    s.geo[1] = INT_MIN;
  }
}

// Cell width: at least time_tol + 1, and wide enough that the sample range
// fits in kClusterCells cells.
__global__ void k_cluster_geometry(int time_tol, ClusterScratch s) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const int64_t lo = s.geo[0], hi = s.geo[1];
  const int64_t range = hi >= lo ? hi - lo + 1 : 1;
  int64_t cw = (int64_t)time_tol + 1;
  const int64_t need = (range + kClusterCells - 1) / kClusterCells;
  if (cw < need) cw = need;
  s.geo[2] = (int)(cw > INT_MAX ? INT_MAX : cw);
  s.geo[3] = (int)((range + cw - 1) / cw);
}

__device__ __forceinline__ uint32_t cell_of(const ClusterScratch& s, int sample) {
  return (uint32_t)(((int64_t)sample - s.geo[0]) / s.geo[2]);
}

__global__ void k_cluster_count(const sps_cand* c, uint32_t n, ClusterScratch s) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) atomicAdd(&s.count[cell_of(s, c[i].sample)], 1u);
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

__global__ void k_cluster_scatter(const sps_cand* c, uint32_t n, ClusterScratch s) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) s.order[atomicAdd(&s.cursor[cell_of(s, c[i].sample)], 1u)] = i;
}

// Position p (bucketed order) against the later positions of its own cell
// and every position of the next cell.
__global__ void k_cluster_link(const sps_cand* c, uint32_t n, int tt, int dt, int wt, ClusterScratch s) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const sps_cand a = c[s.order[p]];
  const uint32_t cell = cell_of(s, a.sample);
  const uint32_t end = s.count[cell + 2];  // start of the cell after the next
  const int la = log2w(a.width);
  for (uint32_t q = p + 1; q < end; ++q) {
    const sps_cand b = c[s.order[q]];
    const int64_t ds = (int64_t)b.sample - a.sample;
    const int64_t dd = (int64_t)b.dm_idx - a.dm_idx;
    const int dw = log2w(b.width) - la;
    if ((ds <= tt && ds >= -tt) && (dd <= dt && dd >= -dt) && (dw <= wt && dw >= -wt)) unite(s.parent, (int)p, (int)q);
  }
}

__global__ void k_cluster_collect(const sps_cand* c, uint32_t n, ClusterScratch s) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int r = find_root(s.parent, (int)p);  // trees no longer change; roots stay roots
  const sps_cand a = c[s.order[p]];
  atomicAdd(&s.members[r], 1u);
  atomicMax(&s.snrbits[r], __float_as_uint(a.snr));  // S/N > 0: its bits order as the values
  atomicMin(&s.slo[r], a.sample);
  atomicMax(&s.shi[r], a.sample);
  atomicMin(&s.dlo[r], a.dm_idx);
  atomicMax(&s.dhi[r], a.dm_idx);
}

// (dm, log2 width, sample) in one key that orders as the tie-break does.
__device__ __forceinline__ unsigned long long tie_key(const sps_cand& a) {
  return ((unsigned long long)a.dm_idx << 37) | ((unsigned long long)log2w(a.width) << 32) |
         (unsigned long long)((uint32_t)a.sample ^ 0x80000000u);
}

__global__ void k_cluster_best(const sps_cand* c, uint32_t n, ClusterScratch s) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int root = find_root(s.parent, (int)p);
  const sps_cand a = c[s.order[p]];
  if (__float_as_uint(a.snr) == s.snrbits[root]) atomicMin(&s.tie[root], tie_key(a));
}

__global__ void k_cluster_emit(uint32_t n, ClusterScratch s, sps_cluster_rec* out, uint32_t* nout) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n || ld_relaxed(&s.parent[p]) != (int)p) return;
  const unsigned long long k = s.tie[p];
  sps_cluster_rec r;
  r.dm_idx = (uint32_t)(k >> 37);
  r.width = 1u << (uint32_t)((k >> 32) & 31u);
  r.sample = (int32_t)((uint32_t)k ^ 0x80000000u);
  r.snr = __uint_as_float(s.snrbits[p]);
  r.members = s.members[p];
  r.sample_lo = s.slo[p];
  r.sample_hi = s.shi[p];
  r.dm_lo = s.dlo[p];
  r.dm_hi = s.dhi[p];
  r.reserved = 0u;
  out[atomicAdd(nout, 1u)] = r;
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
    hipLaunchKernelGGL(k_cluster_init, gn, b, 0, st, c, n, s);
    hipLaunchKernelGGL(k_cluster_geometry, dim3(1), dim3(64), 0, st, tt, s);
    hipLaunchKernelGGL(k_cluster_count, gn, b, 0, st, c, n, s);
    hipLaunchKernelGGL(k_scan_tiles, dim3(kScanTiles), b, 0, st, s);
    hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(1024), 0, st, s);
    hipLaunchKernelGGL(k_scan_add, gc, b, 0, st, s);
    hipLaunchKernelGGL(k_cluster_scatter, gn, b, 0, st, c, n, s);
    hipLaunchKernelGGL(k_cluster_link, gn, b, 0, st, c, n, tt, dt, wt, s);
    hipLaunchKernelGGL(k_cluster_collect, gn, b, 0, st, c, n, s);
    hipLaunchKernelGGL(k_cluster_best, gn, b, 0, st, c, n, s);
    hipLaunchKernelGGL(k_cluster_emit, gn, b, 0, st, n, s, out, nout);
  }
  return hipGetLastError();
}

}  // namespace sps
