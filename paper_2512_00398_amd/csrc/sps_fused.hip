// sps_fused.hip - the whole search of a batch of blocks in one persistent
// launch (Heimdall++ Section II-B's per-trial stages; the paper runs files
// one after another, Section V): baseline and normalisation chains first,
// then the fused filter and peak detection of row segments, each waiting
// only for the chains of its own row.
//
// Every wave first takes statistics chains from the chain queue on its own,
// its histogram in its quarter of the workgroup's detection ring (4 x 2048
// words = the ring's 8192). A chain publishes its medians and MADs with an
// agent-scope release (the XCDs' L2 caches are not coherent for plain
// stores) before it counts itself done for its row. When the chain queue is
// empty the workgroup takes detection tasks; a task's first thread waits,
// with an acquire, until its row's count reaches the row's chains. No wait
// can block forever: a workgroup reaches the detection phase only once every
// chain has been taken by a running wave, and chains never wait.
#include "sps_chain.h"
#include "sps_detect_body.h"

namespace sps {

namespace {

constexpr int kFusedBins = 4096;

template <int NW, bool LEAD>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_search_batch(BatchStats S,
                                                                                             BatchDetect D) {
  __shared__ int s_task;
  static_assert(4 * (kFusedBins / 2) <= kRing, "four chain histograms fit the ring");
  const int wave = readfirst((int)(threadIdx.x >> 6));
  const int lane = lane_id();
  uint32_t* hist = detect_ring() + wave * (kFusedBins / 2);
  // The chain loop has no lane-dependent branch: both atomics are issued by
  // the whole wave with an increment of 1 from lane 0 and 0 from the others.
  // A lane-0 branch at each end of the loop lets the compiler thread one into
  // the other, which splits lane 0 from the rest of the wave across the back
  // edge; the other lanes then read the task from a lane that never took one.
  const uint32_t one = lane == 0 ? 1u : 0u;
  while (true) {
    const int task = readfirst((int)atomicAdd(S.counter, one));  // lane 0's value: the task taken
    if (task >= S.total) break;
    int it = 0;
    while (it + 1 < S.nitems && S.offs[it + 1] <= task) ++it;
    const StatsArgs& a = S.items[it];
    const int chain = task - S.offs[it];
    stats_chain<kFusedBins, false, LEAD>(a, chain, hist, lane);
    // every lane's stores of this chain, then the row's count
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __builtin_amdgcn_wave_barrier();
    __hip_atomic_fetch_add(a.done + chain / a.nseg, one, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();  // the ring holds prefix sums from here on
  // Detection: thread 0 takes the task and waits for its row's chains in one
  // branch; the workgroup reads the task from LDS after the barrier.
  while (true) {
    if (threadIdx.x == 0) {
      const int task = (int)atomicAdd(D.counter, 1u);
      if (task < D.total) {
        int it = 0;
        while (it + 1 < D.nitems && D.offs[it + 1] <= task) ++it;
        const DetectArgs& A = D.items[it];
        const uint32_t* cnt = A.done + (task - D.offs[it]) / A.nseg;
        while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < A.done_target)
          __builtin_amdgcn_s_sleep(4);
        // the thread that saw the count acquires the chains' releases; the
        // barrier passes that on to the workgroup
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
      s_task = task;
    }
    __syncthreads();
    const int task = readfirst(s_task);
    __syncthreads();
    if (task >= D.total) break;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // every wave's own view, after the barrier
    int it = 0;
    while (it + 1 < D.nitems && D.offs[it + 1] <= task) ++it;
    detect_body<NW, false>(D.items[it], task - D.offs[it]);
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_search_batch(const BatchStats& bs, const BatchDetect& bd, int nw_all, bool lead, int grid,
                               hipStream_t s) {
  if (bs.total <= 0 && bd.total <= 0) return hipSuccess;
  const dim3 g(grid), t(256);
  if (nw_all == 13) {
    if (lead) hipLaunchKernelGGL((k_search_batch<13, true>), g, t, 0, s, bs, bd);
    else hipLaunchKernelGGL((k_search_batch<13, false>), g, t, 0, s, bs, bd);
  } else {
    if (lead) hipLaunchKernelGGL((k_search_batch<0, true>), g, t, 0, s, bs, bd);
    else hipLaunchKernelGGL((k_search_batch<0, false>), g, t, 0, s, bs, bd);
  }
  return hipGetLastError();
}

int search_batch_grid(int nw_all) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  const hipError_t e = nw_all == 13
      ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_search_batch<13, false>, 256, 0)
      : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_search_batch<0, false>, 256, 0);
  if (e != hipSuccess) return 0;
  return cus * (per > 0 ? per : 1);
}

}  // namespace sps
