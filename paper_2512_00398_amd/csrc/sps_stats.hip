// sps_stats.hip - baseline removal and normalisation stages (Heimdall++,
// Section II-B): per 64-sample block k of every row, the lower median m_k and
// the lower median absolute deviation MAD_k of the trailing window
// W_k = x[max(0, e_k - L) : e_k], e_k = min(64k + 64, N), or of the window
// centred on the block, which reaches `lead` = (L - 64) / 2 samples further:
// W_k = x[max(0, e_k + lead - L) : min(N, e_k + lead)]. Results are exact.
//
// Design (gfx950, wave64). One wave owns one "chain": a contiguous run of
// blocks of one row, walked in order. The wave keeps a counting histogram of
// its window in LDS: NB consecutive integer values starting at `base`, two
// 16-bit counts per 32-bit word (window sizes are < 2^16, and packed
// add/subtract is exact modulo 2^32 once every count is back in [0, 2^16)).
// Moving from block k-1 to k inserts the <= 64 new samples and removes the
// <= 64 samples that left the window (one LDS atomic per sample). Beside the
// histogram the wave tracks exact counts #{x < p} at three pivots: the
// current median m, the lower edge m - MAD and the upper edge m + MAD + 1;
// ballots update them for every inserted/removed sample, in or out of the
// histogram's range. The common query reads 64 bins around each pivot, one
// bin per lane, and finds the new median and MAD with three wave prefix sums
// and two lane shuffles. When a quantity moves further than the 64-bin
// windows, a full scan of the histogram answers; when it leaves the histogram
// range the window is recounted around the exact median (radix select over
// the window in global memory), and data too spread for any placement of the
// histogram is answered block by block by radix select.
#include "sps_chain.h"

namespace sps {

namespace {

template <int NB, int WPG, bool VIRT, bool LEAD>
__global__ __launch_bounds__(64 * WPG) void k_block_stats(StatsArgs a) {
  __shared__ uint32_t hist[WPG][NB / 2];
  // wave index made uniform: the chain's bookkeeping then runs on the scalar
  // unit beside the vector work of the other waves
  const int wave = readfirst(threadIdx.x >> 6);
  const int chain = blockIdx.x * WPG + wave;
  if (chain >= a.nchains) return;  // whole wave leaves; no block barriers are used
  stats_chain<NB, VIRT, LEAD>(a, chain, hist[wave], lane_id());
}

// Persistent form over a batch: every wave takes chains from the queue on its
// own (no block barriers) until the counter passes the total. VIRT: the items
// are gulps of streams (rows read through their histories).
template <int NB, int WPG, bool VIRT, bool LEAD>
__global__ __launch_bounds__(64 * WPG) void k_block_stats_batch(BatchStats B) {
  __shared__ uint32_t hist[WPG][NB / 2];
  const int wave = threadIdx.x >> 6;
  const int lane = lane_id();
  while (true) {
    uint32_t t = 0;
    if (lane == 0) t = atomicAdd(B.counter, 1u);
    const int task = __builtin_amdgcn_readfirstlane((int)t);
    if (task >= B.total) break;
    int it = 0;
    while (it + 1 < B.nitems && B.offs[it + 1] <= task) ++it;
    stats_chain<NB, VIRT, LEAD>(B.items[it], task - B.offs[it], hist[wave], lane);
  }
}

}  // namespace

hipError_t launch_block_stats(const StatsArgs& a, int hist_bins, hipStream_t s) {
  if (a.nchains <= 0) return hipSuccess;
  const bool virt = a.Hx > 0;
  if (virt && a.lead != 0) return hipErrorInvalidValue;  // streams use the trailing window only
  const bool lead = a.lead != 0;
  if (hist_bins == 16384) {
    const dim3 g((a.nchains + 1) / 2), b(128);
    if (virt) hipLaunchKernelGGL((k_block_stats<16384, 2, true, false>), g, b, 0, s, a);
    else if (lead) hipLaunchKernelGGL((k_block_stats<16384, 2, false, true>), g, b, 0, s, a);
    else hipLaunchKernelGGL((k_block_stats<16384, 2, false, false>), g, b, 0, s, a);
  } else {
    const dim3 g((a.nchains + 3) / 4), b(256);
    if (virt) hipLaunchKernelGGL((k_block_stats<4096, 4, true, false>), g, b, 0, s, a);
    else if (lead) hipLaunchKernelGGL((k_block_stats<4096, 4, false, true>), g, b, 0, s, a);
    else hipLaunchKernelGGL((k_block_stats<4096, 4, false, false>), g, b, 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_block_stats_batch(const BatchStats& b, int hist_bins, bool lead, bool virt, int grid, hipStream_t s) {
  if (b.total <= 0) return hipSuccess;
  if (virt && lead) return hipErrorInvalidValue;  // streams use the trailing window only
  if (hist_bins == 16384) {
    const dim3 g(grid), t(128);
    if (virt) hipLaunchKernelGGL((k_block_stats_batch<16384, 2, true, false>), g, t, 0, s, b);
    else if (lead) hipLaunchKernelGGL((k_block_stats_batch<16384, 2, false, true>), g, t, 0, s, b);
    else hipLaunchKernelGGL((k_block_stats_batch<16384, 2, false, false>), g, t, 0, s, b);
  } else {
    const dim3 g(grid), t(256);
    if (virt) hipLaunchKernelGGL((k_block_stats_batch<4096, 4, true, false>), g, t, 0, s, b);
    else if (lead) hipLaunchKernelGGL((k_block_stats_batch<4096, 4, false, true>), g, t, 0, s, b);
    else hipLaunchKernelGGL((k_block_stats_batch<4096, 4, false, false>), g, t, 0, s, b);
  }
  return hipGetLastError();
}

int block_stats_batch_grid(int hist_bins) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  // resident workgroups are limited by LDS, the same for both window placements
  hipError_t e = hist_bins == 16384
      ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_block_stats_batch<16384, 2, false, false>, 128, 0)
      : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_block_stats_batch<4096, 4, false, false>, 256, 0);
  if (e != hipSuccess) return 0;
  return cus * (per > 0 ? per : 1);
}

}  // namespace sps
