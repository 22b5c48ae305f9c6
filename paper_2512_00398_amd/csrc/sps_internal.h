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
// position is kept as (sample, S/N) with the S/N the IEEE double S / den, so
// bests compare exactly as the definition orders them.
struct RunSum {
  int32_t flags;  // bit0 nonempty, bit1 full, bit2 head valid, bit3 tail valid
  int32_t hi;     // sample index of the head run's best position
  int32_t ti;     // sample index of the tail run's best position
  int32_t pad;
  double hq;      // S/N at hi
  double tq;      // S/N at ti
};
static_assert(sizeof(RunSum) == 32, "RunSum layout");

enum : int32_t { kNonEmpty = 1, kFull = 2, kHead = 4, kTail = 8 };

// Launch descriptors (passed by value as kernel arguments).
//
// The kernels see each row as "virtual" samples [0, N): the first Hx come
// from `hist` (the device-resident history of a stream; Hx = 0 outside
// streaming) and the rest from `x`. Hx is a multiple of 1024.
struct StatsArgs {
  const float* x;
  int64_t ld;          // row stride of x in samples
  const float* hist;
  int64_t ldh;
  int32_t Hx;
  int32_t N, L;        // virtual row length, baseline window
  int32_t lead;        // samples the window reaches past its block's end (0: trailing)
  int32_t nblocks;     // ceil(N / 64): row stride of med / mad
  int32_t kb_first;    // first block computed (blocks below it are carried in)
  int32_t seg_blocks;  // blocks per chain segment (segments 1, 2, ...)
  int32_t head_blocks; // blocks of segment 0 (<= seg_blocks)
  int32_t nseg;        // segments per row
  int32_t nchains;     // rows * nseg
  const int32_t* tmin; // device: no window reaches below *tmin (null: 0)
  int32_t* med;        // [rows][nblocks]
  int32_t* mad;
  uint32_t* done;      // fused batch: per row, chains finished (null elsewhere)
};

// One scale per row: MAD of the row's residual (against med) about its
// lower median, written to every block of mad.
struct RowMadArgs {
  const float* x;
  int64_t ld;          // row stride of x in samples
  int32_t N;           // row length
  int32_t nblocks;     // blocks of the row (ceil(N / 64)), all written
  int32_t ldm;         // row stride of med / mad in blocks (>= nblocks)
  int32_t rows;
  const int32_t* med;  // [rows][ldm]: the row's first block first
  int32_t* mad;        // [rows][ldm], first nblocks of each row overwritten
};

// Per-width re-normalisation: for every row and width w = 2^j the lower
// median c_w of the boxcar-filtered series S_w(i), 0 <= i <= N - w, and the
// lower MAD about it (residuals against med).
struct WidthStatsArgs {
  const float* x;
  int64_t ld;          // row stride of x in samples
  int32_t N;           // row length
  int32_t nblocks;     // row stride of med
  int32_t rows;
  int32_t nw;          // widths 1 .. 2^(nw-1)
  const int32_t* med;  // [rows][nblocks]
  int32_t* center;     // [rows][nw] c_w
  int32_t* mad;        // [rows][nw] MAD_w
};

// Incoherent dedispersion: words of LDS staging per channel span (8 KiB;
// four spans per workgroup).
constexpr int kDedispSpanWords = 2048;

// Staged span of one channel for one trial group, at time tile 0 (tile t
// starts 256 t words later): first 4-byte word and word count.
struct DedispSpan {
  int64_t w0;
  int32_t nw;
  int32_t pad;
};

struct DedispArgs {
  const uint32_t* fil32;  // filterbank bytes [nchan][ld], 4-byte aligned
  int64_t ld;             // row stride in bytes (= nsamp_in)
  int64_t nfull;          // whole 4-byte words in the filterbank
  int64_t total_bytes;    // nchan * ld
  int32_t nchan, ndm, ndm_pad, nsamp_out;
  int32_t dd;             // trials per workgroup (16, 8, 4, 2 or 1)
  int32_t ngroups;        // ndm_pad / dd
  int32_t ntiles;         // ngroups * time tiles
  int32_t per_xcd;        // tiles per XCD (grid = 8 * per_xcd)
  const DedispSpan* span; // [nchan][ngroups]
  // per channel f and trial d: byte offset of the trial's first sample in its
  // group's staged span (trials past ndm repeat the last)
  const int32_t* base;    // [nchan][ndm_pad]
  float* out;             // [ndm][nsamp_out]
};

// Zero-DM filter: in and out [nchan][nsamp] uint8 (may be the same array).
struct ZeroDmArgs {
  const uint8_t* in;
  uint8_t* out;
  int64_t nsamp;
  int32_t nchan;
  int32_t offset;
};

// Narrowband channel mask: in/out [nchan][nsamp] uint8 (may be the same
// array); stats [nchan][3] bytes: median, MAD, flag.
struct ChanMaskArgs {
  const uint8_t* in;
  uint8_t* out;
  uint8_t* stats;
  int64_t nsamp;
  int32_t nchan;
  int32_t k;
};

struct DetectArgs {
  const float* x;
  int64_t ld;
  const float* hist;
  int64_t ldh;
  int32_t Hx;
  int32_t N;           // virtual row length
  int32_t nblocks;
  int32_t nw;          // number of widths (w = 1 << j)
  int32_t maxw;
  const int32_t* med;  // [rows][nblocks]
  const int32_t* mad;
  const int32_t* wmad; // [rows][nw] one scale per (row, width) in place of mad (null: per-block mad)
  double theta;        // (double)(float) threshold
  double sqrtw[kMaxWidths];
  int32_t seg_base;    // first position of segment 0 (multiple of 1024)
  int32_t seg_len;     // positions per segment (multiple of 1024)
  int32_t nseg;        // segments per row
  int32_t rows;
  int32_t e_first;     // evaluate only windows ending at or after e_first
  const int32_t* tmin; // device: evaluate only positions >= *tmin (null: 0)
  int32_t sample_offset;  // emitted sample = position - sample_offset
  int32_t keep_edges;  // 1: always leave row-edge runs to a fix-up kernel
  uint32_t row_offset; // added to dm_idx of emitted candidates
  sps_cand* cands;
  uint32_t* ncand;
  uint32_t cap;
  RunSum* frag;        // [rows][nw][nseg] summaries of segment edges
  const uint32_t* done;  // fused batch: per row, chains finished (null elsewhere)
  uint32_t done_target;  // chains per row
};

// Streaming: fold one push's segment summaries into the carried per-(row,
// width) summaries, and roll the history forward.
struct StreamArgs {
  int32_t rows, nw, nseg;
  int32_t Hx;          // history samples (multiple of 1024)
  int32_t Hb;          // history blocks = Hx / 64
  int32_t ngulp;       // samples of the gulp just pushed
  int32_t nbv;         // virtual blocks per row = Hb + ceil(ngulp / 64)
  const RunSum* frag;  // [rows][nw][nseg], positions in virtual coordinates
  RunSum* carry;       // [rows][nw], positions relative to the current gulp
  const float* gulp;   // [rows][ngulp]
  const float* hist_in;  // [rows][Hx]
  float* hist_out;
  const int32_t* med_in;  // [rows][nbv] of this push
  const int32_t* mad_in;
  int32_t* med_out;       // [rows][nbv] of the next push (history part written)
  int32_t* mad_out;
  int32_t* tmin;          // device scalar
  uint32_t row_offset;
  sps_cand* cands;
  uint32_t* ncand;
  uint32_t cap;
};

// Plain per-stage path: every intermediate lives in device memory.
struct PlainArgs {
  const float* x;      // [rows][N]
  int32_t N, nblocks, rows;
  const int32_t* med;  // [rows][nblocks]
  const int32_t* mad;
  int32_t* r;          // [rows][N] residuals
  uint32_t* P;         // [rows][N + 1] prefix sums
  int32_t* S;          // [rows][N] boxcar sums of the current width
  uint8_t* flag;       // [rows][N] threshold decisions of the current width
  RunSum* frag;        // [rows][nstrip] strip summaries of the current width
  int32_t strip, nstrip;
  int32_t w;
  double sqrtw, theta;
  sps_cand* cands;
  uint32_t* ncand;
  uint32_t cap;
};

// Batch of independent searches: workgroups of one persistent launch take
// tasks from a queue. Task t belongs to item i with offs[i] <= t < offs[i+1];
// items are ordered by the cost of one task, largest first.
struct BatchStats {
  const StatsArgs* items;  // device array [nitems]
  const int32_t* offs;     // device array [nitems + 1]: first chain of each item
  int32_t nitems, total;
  uint32_t* counter;       // device queue head, zero before the launch
};

struct BatchDetect {
  const DetectArgs* items;
  const int32_t* offs;     // first (row, segment) task of each item
  int32_t nitems, total;
  uint32_t* counter;
};

// Candidate clustering scratch (device arrays; n = candidates of a run).
constexpr int kClusterCells = 1 << 22;  // time cells of the bucketing
struct ClusterScratch {
  sps_cand* sorted;   // [cap] candidates in bucket order
  int32_t* parent;    // [cap] union-find over positions (parent <= position)
  uint32_t* members;  // [cap] per root: member count
  uint32_t* snrbits;  //        largest S/N (float bits)
  int32_t* slo;       //        sample extent
  int32_t* shi;
  uint32_t* dlo;      //        DM extent
  uint32_t* dhi;
  unsigned long long* tie;  // [cap] per root: smallest (dm, width, sample) key at the largest S/N
  uint32_t* count;    // [kClusterCells + 2] cell counts, then cell starts
  uint32_t* cursor;   // [kClusterCells + 2] scatter cursors
  uint32_t* bsum;     // [kClusterCells / 1024 + 1] scan tile totals
  int32_t* geo;       // [8] cell geometry (sample and DM ranges, cell sizes)
};

// Host-side launchers (defined in the .hip files).
hipError_t launch_block_stats(const StatsArgs& a, int hist_bins, hipStream_t s);
hipError_t launch_detect(const DetectArgs& a, hipStream_t s);
hipError_t launch_fixup(const DetectArgs& a, hipStream_t s);
hipError_t launch_zero_u32(uint32_t* p, int n, hipStream_t s);
hipError_t launch_row_mad(const RowMadArgs& a, hipStream_t s);
hipError_t launch_width_stats(const WidthStatsArgs& a, hipStream_t s);
hipError_t launch_dedisp(const DedispArgs& a, hipStream_t s);
hipError_t launch_zero_dm(const ZeroDmArgs& a, hipStream_t s);
hipError_t launch_chan_mask(const ChanMaskArgs& a, hipStream_t s);
hipError_t launch_validate(const float* x, int64_t n, float bound, uint32_t* bad, hipStream_t s);
hipError_t launch_stream_fold(const StreamArgs& a, hipStream_t s);
hipError_t launch_stream_advance(const StreamArgs& a, hipStream_t s);
hipError_t launch_stream_close(const StreamArgs& a, hipStream_t s);
hipError_t launch_block_stats_batch(const BatchStats& b, int hist_bins, bool lead, bool virt, int grid, hipStream_t s);
int block_stats_batch_grid(int hist_bins);  // resident workgroups on the current device (0: error)
hipError_t launch_detect_batch(const BatchDetect& b, int nw_all, bool virt, int grid, hipStream_t s);
int detect_batch_grid(int nw_all);
hipError_t launch_fixup_batch(const BatchDetect& b, const int32_t* d_offs, int total, hipStream_t s);
hipError_t launch_batch_zero(uint32_t* const* d_ncand, int n, uint32_t* counters, hipStream_t s);
// Fused batch: statistics chains, then detection tasks that wait on their
// rows' chains, in one persistent launch (4096-bin histograms).
hipError_t launch_search_batch(const BatchStats& bs, const BatchDetect& bd, int nw_all, bool lead, int grid,
                               hipStream_t s);
int search_batch_grid(int nw_all);
hipError_t launch_plain_prepare(const PlainArgs& a, hipStream_t s);
hipError_t launch_plain_width(const PlainArgs& a, hipStream_t s);
hipError_t launch_cluster(const sps_cand* c, uint32_t n, int time_tol, int dm_tol, int width_tol,
                          const ClusterScratch& s, sps_cluster_rec* out, uint32_t* nout, hipStream_t st);

}  // namespace sps
