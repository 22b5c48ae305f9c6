// sps_internal.h - shared declarations of libsps (HIP, gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sps.h"

namespace sps {

constexpr int kStride = SPS_BLOCK_STRIDE;  // S: samples per baseline block
constexpr int kMaxWidths = 13;             // widths 1 .. 4096
// 1 / Phi^{-1}(3/4): scales a Gaussian's MAD to its sigma.
constexpr double kMadToSigma = 1.482602218505602;

// Summary of the peak-detection runs of one contiguous range of positions of
// one (row, width). A run is a maximal set of consecutive "above" positions.
// head: best of the run that starts at the range's first position (if that
// position is above); tail: best of the run that ends at the range's last
// position (if above and the range is not entirely above); full: every
// position above (then head holds the best of the whole range). Runs touching
// neither end were already emitted when the summary was formed. A best
// position is kept as (sample, S, den): its S/N is S / den in IEEE double.
struct RunSum {
  int32_t flags;  // bit0 nonempty, bit1 full, bit2 head valid, bit3 tail valid
  int32_t hi;     // sample index of the head run's best position
  int32_t ti;     // sample index of the tail run's best position
  int32_t hS;     // boxcar sum at hi
  int32_t tS;     // boxcar sum at ti
  int32_t pad;
  double hd;      // S/N denominator (K * MAD) * sqrt(w) at hi
  double td;      // ... at ti
};
static_assert(sizeof(RunSum) == 40, "RunSum layout");

enum : int32_t { kNonEmpty = 1, kFull = 2, kHead = 4, kTail = 8 };

// Launch descriptors (passed by value as kernel arguments).
struct StatsArgs {
  const float* x;
  int64_t ld;          // row stride in samples
  int32_t N, L;
  int32_t nblocks;     // ceil(N / 64)
  int32_t seg_blocks;  // blocks per chain segment
  int32_t nseg;        // segments per row
  int32_t nchains;     // rows * nseg
  int32_t* med;        // [rows][nblocks]
  int32_t* mad;
};

struct DetectArgs {
  const float* x;
  int64_t ld;
  int32_t N;
  int32_t nblocks;
  int32_t nw;          // number of widths (w = 1 << j)
  int32_t maxw;
  const int32_t* med;  // [rows][nblocks]
  const int32_t* mad;
  double theta;        // (double)(float) threshold
  double sqrtw[kMaxWidths];
  int32_t seg_len;     // positions per segment (multiple of the step size)
  int32_t nseg;        // segments per row
  int32_t rows;
  uint32_t row_offset; // added to dm_idx of emitted candidates
  sps_cand* cands;
  uint32_t* ncand;
  uint32_t cap;
  RunSum* frag;        // [rows][nw][nseg] summaries of multi-segment rows
};

// Host-side launchers (defined in the .hip files).
hipError_t launch_block_stats(const StatsArgs& a, int hist_bins, hipStream_t s);
hipError_t launch_detect(const DetectArgs& a, hipStream_t s);
hipError_t launch_fixup(const DetectArgs& a, hipStream_t s);
hipError_t launch_zero_u32(uint32_t* p, int n, hipStream_t s);

}  // namespace sps
