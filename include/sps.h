/*
 * sps.h - C interface of libsps, the MI355X (gfx950) single-pulse search.
 *
 * The library runs, on one GPU, the per-DM-trial part of a single-pulse
 * search over a block of dedispersed time series: baseline removal,
 * normalisation, matched filtering with a bank of boxcars, and peak
 * detection above an S/N threshold, producing candidates (time, DM trial,
 * filter width, peak S/N). These are the four stages of the DM-trial loop in
 * Heimdall++ (Section II-B, "Pipeline Stages in Heimdall"; Algorithm 1, the
 * parallel candidate search). The paper names the stages without formulas;
 * the exact arithmetic implemented here is:
 *
 *   x_t       integer value of sample t of a row (inputs are integer-valued)
 *   block k   samples [kS, min(kS+S, N)), S = 64; e_k = min(kS+S, N)
 *   W_k       trailing window x[max(0, e_k - L) : e_k]
 *   m_k       lower median of W_k (element of rank floor((n-1)/2))
 *   MAD_k     lower median of |W_k - m_k|
 *   r_t       x_t - m_{floor(t/S)}
 *   S_w(i)    sum of r over [i, i+w), w = 1, 2, 4, ..., max_width, 0 <= i <= N-w
 *   snr       S_w(i) / ((K * MAD_{k*}) * sqrt(w)) in IEEE double, K = 1/Phi^-1(3/4),
 *             k* = floor((i + floor(w/2)) / S); positions with MAD_{k*} = 0 are never above
 *   above     snr > (double)snr_thresh
 *   candidate one per maximal run of above positions of a (row, width), at the
 *             run's first arg-max: {sample = i, dm_idx = row, width = w, snr = (float)snr}
 *
 * Conventions for every entry point:
 *   - Device pointers ("d_" prefix) are HIP device memory owned by the caller
 *     (e.g. torch tensors); they must stay valid until the stream work ends.
 *   - Calls that take a hipStream_t are asynchronous and stream-ordered; they
 *     never synchronise the device. Argument errors are reported synchronously
 *     by the return code and nothing is enqueued.
 *   - Return codes: SPS_OK (0) or a negative SPS_ERR_* value; sps_last_error()
 *     returns the last code of the calling thread, sps_error_string() a text.
 *   - A plan may be used by one stream at a time (it owns scratch memory).
 *   - Input domain: FP32 samples with integer values, |x| < 2^24, and every
 *     boxcar sum |S_w(i)| < 2^31. Outside this domain results are unspecified
 *     (no out-of-bounds access ever results).
 */
#ifndef SPS_H
#define SPS_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Error codes. */
#define SPS_OK 0
#define SPS_ERR_INVALID_ARG (-1) /* bad argument: nothing was enqueued */
#define SPS_ERR_OOM (-2)         /* device memory allocation failed */
#define SPS_ERR_HIP (-3)         /* a HIP runtime call failed (e.g. launch) */
#define SPS_ERR_OVERFLOW (-4)    /* candidate count exceeded the capacity (reported by callers) */
#define SPS_ERR_DOMAIN (-5)      /* input outside the supported domain */
#define SPS_ERR_SCRATCH (-6)     /* block too large for sps_search_noalloc's fixed scratch */

/* One candidate, 16 bytes. sample: first sample of the boxcar window, counted
 * from the first sample of the call's input (negative in streaming mode when
 * the run began in the carried history); dm_idx: row (plus the batch item's
 * row offset); width: boxcar width; snr: peak S/N rounded to FP32. */
typedef struct {
    int32_t sample;
    uint32_t dm_idx;
    uint32_t width;
    float snr;
} sps_cand;

typedef struct sps_plan sps_plan;

/* Limits of the library. */
#define SPS_BLOCK_STRIDE 64          /* S: samples per baseline block */
#define SPS_MAX_WIDTH_LIMIT 4096     /* largest boxcar width */
#define SPS_MAX_BASELINE_LEN 65535   /* largest baseline window L */

/*
 * Create a plan for blocks of ndm rows x nsamp samples (row-major FP32,
 * row stride nsamp): boxcar widths 1, 2, 4, ..., max_width; baseline window
 * of baseline_len samples; threshold snr_thresh (in units of the robust sigma).
 * Requirements: ndm >= 1; 1 <= nsamp < 2^31; max_width a power of two in
 * [1, SPS_MAX_WIDTH_LIMIT]; 1 <= baseline_len <= SPS_MAX_BASELINE_LEN;
 * snr_thresh finite and > 0. Allocates the plan's device scratch
 * (about 8 bytes per 64 samples plus small tables) on the current device.
 * Returns NULL on error (sps_last_error() tells which).
 * Stages: Section II-B (all four per-trial stages); Algorithm 1.
 */
sps_plan* sps_plan_create(int32_t ndm, int64_t nsamp, int32_t max_width, int32_t baseline_len,
                          float snr_thresh);

/* Free a plan and its device scratch. NULL-safe. Waits first for the plan's
 * last call (the end of its device work) so that no enqueued work still uses
 * the scratch; work of other plans and streams is not waited for. */
void sps_plan_destroy(sps_plan* plan);

/*
 * Search d_series (device, FP32 [ndm][nsamp]) on `stream`.
 * Candidates go to d_cands (device, capacity given by SPS_ATTR_MAX_CANDS,
 * default 2^24 records); *d_ncand (device uint32) is zeroed in-stream and
 * holds the TRUE number of candidates after the work completes. If it exceeds
 * the capacity, only `capacity` records were written (which ones is
 * unspecified) and the caller should retry with a larger buffer. Candidate
 * order is unspecified: compare sorted by (dm_idx, width, sample).
 * Stages: Section II-B; Algorithm 1, the per-trial kernels of the parallel
 * candidate search, here fused and launched over all rows at once.
 */
int sps_search(sps_plan* plan, const float* d_series, hipStream_t stream, sps_cand* d_cands,
               uint32_t* d_ncand);

/*
 * Allocation-free search, for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops and harnesses that forbid
 * hipMalloc. The same search as a plan with default attributes created with
 * these five parameters would run (SPS_ATTR_MAX_CANDS = max_cands), with the
 * same results, but no plan is needed and the call never allocates or frees
 * memory: its scratch (block medians and MADs, 8 bytes per 64-sample block per
 * row rounded up to 256 bytes per array, then run summaries of detection
 * segments) lives in a fixed device array of SPS_NOALLOC_SCRATCH_BYTES that
 * every GPU holds, once loaded, until the process ends. Blocks whose medians
 * and MADs do not fit (ndm * ceil(nsamp/64) > 2^23, e.g. more than 512 rows
 * of 2^20 samples) are refused with SPS_ERR_SCRATCH and nothing is
 * enqueued; when only the run summaries would not fit, each row is detected
 * in one segment. All calls on one GPU share that GPU's array and the array
 * keeps the last call's contents, so calls that overlap on one GPU (on
 * different streams or host threads) race: order them on one stream. The
 * first call on each device looks up the array's address (host-synchronous
 * set-up); later calls are asynchronous on `stream` like sps_search.
 * d_series, d_cands (capacity max_cands records, in [0, 2^32 - 1]) and
 * d_ncand as for sps_search. Returns SPS_OK, SPS_ERR_INVALID_ARG (bad shape,
 * parameters or pointers), SPS_ERR_SCRATCH or SPS_ERR_HIP.
 */
#define SPS_NOALLOC_SCRATCH_BYTES (64u << 20)
int sps_search_noalloc(int32_t ndm, int64_t nsamp, int32_t max_width, int32_t baseline_len, float snr_thresh,
                       const float* d_series, hipStream_t stream, sps_cand* d_cands, uint32_t* d_ncand,
                       int64_t max_cands);

/*
 * Input domain (every search entry point): each sample integer-valued with
 * |x| <= sps_domain_bound(max_width) = min(2^24 - 1, (2^31 - 1) / (2 *
 * max_width)), so that the conversion to integers is exact and every boxcar
 * sum of residuals fits in int32. Outside it results are unspecified. With
 * SPS_ATTR_VALIDATE = 1 every search (and stream push) first checks its input
 * on the device, waits for the answer, and returns SPS_ERR_DOMAIN without
 * searching if a sample falls outside (a debug mode: host-synchronous).
 */
int64_t sps_domain_bound(int32_t max_width);

/*
 * Baseline-removal and normalisation stages only: write m_k and MAD_k of
 * every block of every row to d_median and d_mad (device int32
 * [ndm][ceil(nsamp/64)], row stride ceil(nsamp/64)). Section II-B,
 * "Baseline Removal and Normalization".
 */
int sps_block_stats(sps_plan* plan, const float* d_series, hipStream_t stream, int32_t* d_median,
                    int32_t* d_mad);

/*
 * Per-width statistics (the SPS_ATTR_NORM = 2 scales) alone: for every row d
 * and width w = 2^j, d_center[d * nw + j] = c_w and d_mad[d * nw + j] = MAD_w
 * (device int32 [ndm][nw], nw = number of widths; 0 and 0 for widths longer
 * than the row), whatever the plan's SPS_ATTR_NORM. Also overwrites the
 * plan's block statistics. Section II-B, "Normalization".
 */
int sps_width_stats(sps_plan* plan, const float* d_series, hipStream_t stream, int32_t* d_center, int32_t* d_mad);

/*
 * The same search as sps_search, executed as plain per-stage kernels with
 * every intermediate (medians, residuals, prefix sums, boxcar outputs,
 * per-position S/N decisions) materialised in device memory, one launch per
 * stage and width, as the staged DM-trial loop of Section II-B runs. Results
 * equal sps_search's exactly. Allocates its larger scratch (about
 * 12 bytes per sample) on first use and keeps it with the plan.
 */
int sps_search_plain(sps_plan* plan, const float* d_series, hipStream_t stream, sps_cand* d_cands,
                     uint32_t* d_ncand);

/* Plan attributes (sps_plan_set / sps_plan_get). */
#define SPS_ATTR_MAX_CANDS 1      /* capacity of d_cands in records (default 1<<24) */
#define SPS_ATTR_STATS_SEG 2      /* blocks per baseline chain segment (tuning; 0 = auto) */
#define SPS_ATTR_DETECT_SEG 3     /* samples per detection segment, multiple of 1024 (0 = auto) */
#define SPS_ATTR_HIST_BINS 4      /* fine histogram span in values: 4096 or 16384 (tuning) */
#define SPS_ATTR_TIMING 5         /* 1: record HIP events around every kernel of a search */
#define SPS_ATTR_VALIDATE 6       /* 1: check the input domain before each search (host-synchronous) */
#define SPS_ATTR_WINDOW 7         /* baseline window placement, part of the arithmetic: 0 (default) trailing,
                                     W_k = x[max(0, e_k - L) : e_k]; 1 centred on its block, the window
                                     reaching lead = max(0, (L - 64) / 2) samples past the block's end,
                                     W_k = x[max(0, e_k + lead - L) : min(N, e_k + lead)]
                                     (Section II-B's moving baseline; the paper does not place the window).
                                     Plans and batches; a stream refuses a plan with 1 (its blocks would
                                     wait for lead samples of the next gulp). */
#define SPS_ATTR_NORM 8           /* noise scale, part of the arithmetic: 0 (default) the block's MAD_k;
                                     1 one scale per DM row, MAD_row = lower median of |r_t - c| over the
                                     whole row, r_t = x_t - m_{t/64} and c the lower median of r (Section
                                     II-B's normalisation read as one scale per trial and chunk). Every
                                     block of the row then reports and uses MAD_row. Plans and batches;
                                     in a stream the chunk is the gulp: every block of a gulp takes the
                                     MAD_row of that gulp's residuals (residuals as on the concatenation,
                                     trailing windows reaching into earlier gulps). */
                                  /* 2 one scale per (DM row, width): for the boxcar-filtered series
                                     T_w = {S_w(i) : 0 <= i <= nsamp - w}, c_w = lower median of T_w
                                     and MAD_w = lower median of |S_w(i) - c_w|; then
                                     snr = S_w(i) / (K * MAD_w) (no sqrt(w): MAD_w measures the filtered
                                     series itself), a width with MAD_w = 0 has no above positions
                                     (Section II-B's normalisation read as a scale per filtered series).
                                     Block medians m_k unchanged. Plans and batches only: streams and
                                     sps_search_plain refuse it. MAD_w above 2^31 - 1 (half the series
                                     more than 2^31 from its median) is taken as 2^31 - 1. */
#define SPS_ATTR_FUSED 9          /* batches only (tuning): 1 (default) statistics chains and detection in one
                                     persistent launch, each detection task waiting for its row's chains;
                                     0 one persistent launch per stage. Only SPS_ATTR_NORM = 0 with
                                     SPS_ATTR_HIST_BINS = 4096 runs fused; other settings run per stage. */
#define SPS_ATTR_NBLOCKS 16       /* read-only: ceil(nsamp / 64) */
#define SPS_ATTR_NWIDTHS 17       /* read-only: number of boxcar widths */
#define SPS_ATTR_BLOCK_STRIDE 18  /* read-only: S = SPS_BLOCK_STRIDE, part of the arithmetic (never tuned) */

/* Tuning attributes never change results, only speed. Returns SPS_OK or
 * SPS_ERR_INVALID_ARG (unknown attribute, value out of range, read-only). */
int sps_plan_set(sps_plan* plan, int attr, int64_t value);
int sps_plan_get(const sps_plan* plan, int attr, int64_t* value);

/*
 * Kernel timing (tracing). With SPS_ATTR_TIMING = 1 every search records HIP
 * events on its stream around each kernel. sps_timing_read waits for the
 * recorded events, writes the summed milliseconds per stage since the last
 * read to ms_out[SPS_NSTAGES] and the number of searches to *nsearch, and
 * resets the sums. Stages: 0 baseline/normalisation kernel, 1 fused
 * filter/detect kernel, 2 fix-up and counter reset, 3 plain per-stage path
 * (whole search). Host-synchronous.
 */
#define SPS_NSTAGES 4
int sps_timing_read(sps_plan* plan, double* ms_out, int64_t* nsearch);

/*
 * Streaming: one long observation searched gulp by gulp, exactly as if the
 * gulps were one block (chunks overlap "to preserve signal continuity",
 * Section III-B; double-buffered chunk reads, Sections IV-C and V-C). The
 * carried state stays on the device: per row the last max(baseline_len,
 * max_width) samples (rounded up to 1024) with their block medians/MADs, and
 * per (row, width) a summary of the run still open at the end of the last
 * gulp (20 KiB + 520 B per row at baseline 16384).
 *
 * sps_stream_create: `plan` gives the gulp shape (ndm x nsamp, nsamp a
 *   multiple of 64) and parameters; it must outlive the stream, and the
 *   stream must not run concurrently with another use of the plan. A plan
 *   with SPS_ATTR_WINDOW = 1 or SPS_ATTR_NORM = 2 is refused
 *   (SPS_ERR_INVALID_ARG), here and at every push if the plan's attributes
 *   were changed since; SPS_ATTR_NORM = 1 gives one row scale per gulp.
 * sps_stream_push: search one gulp (device FP32 [ndm][nsamp]); candidates are
 *   those whose runs ended during this gulp, with `sample` relative to the
 *   gulp's first sample (negative: the boxcar started in an earlier gulp).
 *   *gulp_offset (host, may be NULL) receives the global index of the gulp's
 *   first sample. d_ncand/d_cands as in sps_search. Asynchronous.
 * sps_stream_flush: end of observation: emits the runs still open, `sample`
 *   relative to the sample after the last gulp (*end_offset = samples
 *   pushed). The stream can then be reused only after restore.
 * sps_stream_state_size / save / restore: checkpoint the carried state to
 *   host memory and back (host-synchronous on `stream`); a restored stream
 *   continues exactly as the saved one would have.
 */
typedef struct sps_stream sps_stream;
int sps_stream_create(sps_plan* plan, sps_stream** out);
int sps_stream_push(sps_stream* s, const float* d_gulp, hipStream_t stream, sps_cand* d_cands, uint32_t* d_ncand,
                    int64_t* gulp_offset);
/* sps_stream_push_graph: the same gulp step replayed from a captured HIP
 * graph (one per history parity, captured on first use of a (d_gulp,
 * d_cands, d_ncand) triple; the 8 most recently used triples are kept, so a
 * fixed set of double- or triple-buffered input locations is captured once).
 * Same results as sps_stream_push. */
int sps_stream_push_graph(sps_stream* s, const float* d_gulp, hipStream_t stream, sps_cand* d_cands,
                          uint32_t* d_ncand, int64_t* gulp_offset);
int sps_stream_flush(sps_stream* s, hipStream_t stream, sps_cand* d_cands, uint32_t* d_ncand, int64_t* end_offset);
int sps_stream_state_size(const sps_stream* s, uint64_t* bytes);
int sps_stream_save(sps_stream* s, hipStream_t stream, void* host_buf, uint64_t bytes);
int sps_stream_restore(sps_stream* s, hipStream_t stream, const void* host_buf, uint64_t bytes);
void sps_stream_destroy(sps_stream* s);

/*
 * Batch: many independent blocks ("files": the paper processes file after
 * file, Section V; every block is searched exactly as sps_search would search
 * it alone) in one persistent launch of the statistics chains and the
 * detection tasks (SPS_ATTR_FUSED = 1), or one persistent launch per stage.
 * Workgroups take work from device queues shared by all blocks, whose tasks
 * are ordered largest first, so blocks of very different shapes load-balance
 * with no per-block launch tail; a small fix-up launch stitches runs across
 * detection segments.
 *
 * sps_batch_item: one block. d_series device FP32 [ndm][nsamp] (caller-owned,
 *   read-only); parameters obey the sps_plan_create rules; d_cands (capacity
 *   max_cands records; may be NULL when max_cands is 0) and d_ncand are that
 *   block's own outputs, exactly as for sps_search.
 * sps_batch_create: an empty batch context (workspace grows on demand).
 * sps_batch_search: enqueue the search of n items on `stream`. Asynchronous,
 *   except that a call which needs more workspace than any earlier call (the
 *   first one, for instance) first waits for the context's earlier work.
 *   Item descriptors are copied during the call; the caller's array can be
 *   reused on return. One stream at a time per context (calls on different
 *   streams are ordered after the context's previous call). Returns SPS_OK or
 *   SPS_ERR_INVALID_ARG (any item invalid: nothing enqueued), SPS_ERR_OOM,
 *   SPS_ERR_HIP.
 * sps_batch_set: tuning attributes SPS_ATTR_STATS_SEG, SPS_ATTR_DETECT_SEG,
 *   SPS_ATTR_HIST_BINS and SPS_ATTR_FUSED, and the arithmetic variants
 *   SPS_ATTR_WINDOW and SPS_ATTR_NORM (same meaning as for plans; apply to
 *   every item).
 * sps_batch_destroy: waits for the context's work and frees it (NULL-safe).
 */
typedef struct {
  const float* d_series;
  int32_t ndm;
  int32_t max_width;
  int64_t nsamp;
  int32_t baseline_len;
  float snr_thresh;
  sps_cand* d_cands;
  uint32_t* d_ncand;
  int64_t max_cands;
} sps_batch_item;

typedef struct sps_batch sps_batch;
int sps_batch_create(sps_batch** out);
/*
 * sps_batch_push: continuous batching of streams (the serving loop's gulps
 *   of many beams, Section IV-C's overlapped chunk processing): one gulp of
 *   each of n distinct streams (streams[i], device FP32 d_gulps[i] of its
 *   plan's shape) searched by one persistent launch per stage over all of
 *   them, then each stream's carry folded and rolled forward. Results,
 *   carried state and *gulp_offsets (host int64[n], may be NULL) are exactly
 *   those of calling sps_stream_push(streams[i], d_gulps[i], stream,
 *   d_cands[i], d_ncand[i], &gulp_offsets[i]) for each i; streams may have
 *   different shapes and parameters. d_cands / d_ncand are host arrays of n
 *   device pointers (capacity: the stream's plan SPS_ATTR_MAX_CANDS). A
 *   stream may appear once per call (its next gulp needs this one's carry);
 *   it must not be used concurrently elsewhere. Each stream keeps its own
 *   plan's scale (one row scale per gulp with SPS_ATTR_NORM = 1); a stream
 *   whose plan has since been set to a centred window or the per-width
 *   scale is refused. Uses the context's SPS_ATTR_HIST_BINS; plan timing is
 *   not recorded. Asynchronous, except
 *   that a call needing larger tables than any earlier one first waits for
 *   the context's earlier work. SPS_OK, SPS_ERR_INVALID_ARG (nothing
 *   enqueued), SPS_ERR_DOMAIN (plan validation), SPS_ERR_OOM, SPS_ERR_HIP.
 */
int sps_batch_push(sps_batch* b, sps_stream* const* streams, const float* const* d_gulps, int32_t n,
                   hipStream_t stream, sps_cand* const* d_cands, uint32_t* const* d_ncand, int64_t* gulp_offsets);
int sps_batch_set(sps_batch* b, int attr, int64_t value);
int sps_batch_search(sps_batch* b, const sps_batch_item* items, int32_t n, hipStream_t stream);
void sps_batch_destroy(sps_batch* b);

/*
 * Device memory a plan of this shape holds with default tuning (and, with
 * streaming = 1, a stream on it as well), in bytes; nothing is allocated and
 * no device is needed. Inputs and candidate buffers are the caller's and not
 * counted. For admission control against a memory budget. Returns SPS_OK or
 * SPS_ERR_INVALID_ARG (the shape would be rejected by sps_plan_create or
 * sps_stream_create).
 */
int sps_footprint(int32_t ndm, int64_t nsamp, int32_t max_width, int32_t baseline_len, int streaming,
                  uint64_t* bytes);

/*
 * Candidate merging and clustering (Heimdall++, Section II-B "Candidate
 * Merging and Clustering", Section III and the last step of Algorithm 1:
 * detections close in time, DM and filter width are grouped and each group is
 * reported by its strongest member). The paper gives no rule or tolerances;
 * the reading implemented is friends-of-friends: candidates a and b are
 * linked when |sample_a - sample_b| <= time_tol, |dm_a - dm_b| <= dm_tol and
 * |log2 width_a - log2 width_b| <= width_tol; clusters are the connected
 * components of the links; each is reported by its member of largest S/N
 * (equal S/N: smallest dm, then width, then sample), with the member count
 * and the cluster's sample and DM extents.
 *
 * sps_cluster_create: device scratch for up to max_cands candidates per run
 *   (about 40 bytes per candidate plus 48 MiB of time-cell tables). NULL on
 *   error (SPS_ERR_INVALID_ARG for max_cands = 0, SPS_ERR_OOM, SPS_ERR_HIP).
 * sps_cluster_run: clusters the n candidates at d_cands (device, caller-owned,
 *   as written by sps_search; n <= max_cands, given by the host) on `stream`.
 *   Writes one record per cluster to d_out (device, capacity n records; order
 *   unspecified) and their count to *d_nout (device). Asynchronous and
 *   stream-ordered; tolerances must be >= 0, samples within int32, dm_idx
 *   < 2^27 and widths powers of two up to 2^31. A context serves one stream
 *   at a time.
 * sps_cluster_destroy: waits for the context's last run and frees it (NULL-safe).
 */
typedef struct {
  int32_t sample;     /* best member: boxcar start */
  uint32_t dm_idx;
  uint32_t width;
  float snr;
  uint32_t members;   /* candidates in the cluster */
  int32_t sample_lo;  /* smallest and largest sample of its members */
  int32_t sample_hi;
  uint32_t dm_lo;     /* smallest and largest dm_idx of its members */
  uint32_t dm_hi;
  uint32_t reserved;
} sps_cluster_rec;    /* 40 bytes */

typedef struct sps_clusterer sps_clusterer;

sps_clusterer* sps_cluster_create(uint32_t max_cands);
int sps_cluster_run(sps_clusterer* k, const sps_cand* d_cands, uint32_t n, int32_t time_tol, int32_t dm_tol,
                    int32_t width_tol, hipStream_t stream, sps_cluster_rec* d_out, uint32_t* d_nout);
void sps_cluster_destroy(sps_clusterer* k);

/* ---- Incoherent dedispersion (Heimdall++ Section II-B, "Incoherent
 * Dedispersion", the dispersion measure of Eq. 1, and the dedispersion step
 * of Algorithm 1): the producer of the block sps_search consumes, on the
 * device, from an 8-bit filterbank.
 *
 * sps_dedisp_delays (host only, no device work): the cold-plasma delay of
 *   every channel at every trial DM, in samples,
 *     delays[d*nchan + f] = floor(k_DM * dms[d] * (freqs_mhz[f]^-2 - f_ref_mhz^-2) / tsamp_s + 0.5),
 *   k_DM = 4.148808e3 MHz^2 pc^-1 cm^3 s, evaluated in double precision in
 *   that order (dms converted from float). Channel frequencies in MHz, each
 *   in (0, f_ref_mhz]; DMs >= 0 (pc cm^-3); tsamp_s > 0. `delays` is a host
 *   array of ndm * nchan int32 owned by the caller. SPS_ERR_INVALID_ARG for
 *   bad sizes or values or a delay beyond INT32_MAX; SPS_OK otherwise.
 * sps_dedisp_create: copies a host delay table [ndm][nchan] (int32, every
 *   entry >= 0; any table, not only the one above) to the device. nchan in
 *   [1, 65536]; nsamp_in in [1, INT32_MAX - 8192]; the largest delay must be
 *   below nsamp_in. The output row length is nsamp_out = nsamp_in - largest
 *   delay. NULL on error (sps_last_error: SPS_ERR_INVALID_ARG, SPS_ERR_OOM,
 *   SPS_ERR_HIP). Synchronous.
 * sps_dedisp_nsamp_out: nsamp_out (-1 and SPS_ERR_INVALID_ARG for NULL).
 * sps_dedisp_run: d_fil is a device uint8 filterbank, channel-major
 *   [nchan][nsamp_in] (row stride nsamp_in bytes), 4-byte aligned, read
 *   only; d_out is a device FP32 [ndm][nsamp_out] array (row stride
 *   nsamp_out), overwritten with
 *     out[d][t] = sum_f fil[f][t + delays[d][f]],  0 <= t < nsamp_out,
 *   exact integers (below 2^24 for nchan <= 65793, the domain sps_search
 *   accepts). Asynchronous on `stream`; SPS_ERR_INVALID_ARG (NULL or
 *   misaligned pointers), SPS_ERR_HIP (launch failure).
 * sps_dedisp_destroy: waits for the object's last run and frees it (NULL-safe).
 */
typedef struct sps_dedisp sps_dedisp;

/* ---- Broadband (zero-DM) RFI excision (Heimdall++ Section II-B, "RFI
 * Mitigation", the stage before dedispersion in Algorithm 1).
 * sps_zero_dm: d_in and d_out are device uint8 filterbanks, channel-major
 *   [nchan][nsamp] (row stride nsamp bytes); d_out may equal d_in (in place)
 *   but must not otherwise overlap it. For every time sample t,
 *     z_t = floor((2 * sum_f in[f][t] + nchan) / (2 * nchan))
 *   (the channel mean rounded half up) and
 *     out[f][t] = min(255, max(0, in[f][t] - z_t + offset)).
 *   nchan in [1, 65536], nsamp in [1, INT32_MAX - 8192], offset in [0, 255]. Asynchronous on
 *   `stream`; SPS_ERR_INVALID_ARG (bad sizes, NULL or overlapping buffers),
 *   SPS_ERR_HIP (launch failure). */
int sps_zero_dm(const uint8_t* d_in, int32_t nchan, int64_t nsamp, int32_t offset, hipStream_t stream,
                uint8_t* d_out);

/* ---- Narrowband RFI excision (Heimdall++ Section II-B, "RFI Mitigation").
 * sps_chan_mask: d_in and d_out as for sps_zero_dm (d_out may equal d_in).
 *   For each channel f over the chunk, mu_f = lower median of in[f][:] and
 *   sigma_f = lower median of |in[f][t] - mu_f| (rank (nsamp-1)/2); across
 *   channels M = lower median of sigma_f and S = lower median of
 *   |sigma_f - M| (rank (nchan-1)/2). Channel f is flagged iff
 *   sigma_f > M + k * S, and a flagged channel is written as mu_f at every
 *   sample; the others are copied. d_stats is a device byte array
 *   [nchan][3] receiving (mu_f, sigma_f, flag); it must not overlap the
 *   filterbanks. nchan in [1, 65536], nsamp in [1, INT32_MAX - 8192],
 *   k >= 0. Asynchronous on `stream`; SPS_ERR_INVALID_ARG (bad sizes, NULL
 *   or overlapping buffers), SPS_ERR_HIP (launch failure). */
int sps_chan_mask(const uint8_t* d_in, int32_t nchan, int64_t nsamp, int32_t k, hipStream_t stream, uint8_t* d_out,
                  uint8_t* d_stats);

int sps_dedisp_delays(int32_t nchan, const double* freqs_mhz, double f_ref_mhz, double tsamp_s, int32_t ndm,
                      const float* dms, int32_t* delays);
sps_dedisp* sps_dedisp_create(int32_t nchan, int64_t nsamp_in, int32_t ndm, const int32_t* delays);
int64_t sps_dedisp_nsamp_out(const sps_dedisp* k);
int sps_dedisp_run(sps_dedisp* k, const uint8_t* d_fil, hipStream_t stream, float* d_out);
void sps_dedisp_destroy(sps_dedisp* k);

/* Last error code of the calling thread, and a static text for a code. */
int sps_last_error(void);
const char* sps_error_string(int code);

#ifdef __cplusplus
}
#endif

#endif /* SPS_H */
