// sps_api.hip - the C interface of libsps: plans, argument checks, launches.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "sps_internal.h"

struct sps_plan {
  int32_t ndm;
  int32_t nsamp;
  int32_t max_width;
  int32_t baseline_len;
  float thresh;
  int32_t nw;
  int32_t nblocks;
  double sqrtw[sps::kMaxWidths];
  int64_t max_cands;
  // tuning (never changes results)
  int32_t stats_seg;   // blocks per baseline chain, 0 = auto
  int32_t detect_seg;  // samples per detection segment, 0 = auto
  int32_t hist_bins;   // 4096 or 16384
  int32_t window;      // SPS_ATTR_WINDOW: 0 trailing, 1 centred (changes results)
  int32_t norm;        // SPS_ATTR_NORM: 0 per-block MAD, 1 one MAD per row, 2 one MAD per (row, width)
  int device;
  // scratch owned by the plan
  int32_t* d_med;
  int32_t* d_mad;
  sps::RunSum* d_frag;
  int64_t frag_cap;    // RunSum records allocated
  int32_t* d_wstat;    // [2][ndm][nw] per-width medians c_w and MADs (SPS_ATTR_NORM = 2)
  // plain per-stage path scratch (allocated on first use)
  void* d_plain;
  size_t plain_bytes;
  // debug: check the input domain before each search
  int validate;
  uint32_t* d_flag;    // 1 word: the domain check's answer
  // tracing: events recorded around kernels when timing is on
  int timing;
  std::vector<hipEvent_t>* ev_free;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>>* ev_pending;
  double stage_ms[SPS_NSTAGES];
  int64_t nsearch;
  // end of the last call's device work (destroy and scratch regrowth wait for it)
  hipEvent_t done;
  bool pending;
};

namespace {

thread_local int g_last_error = SPS_OK;

int fail(int code) {
  g_last_error = code;
  return code;
}

int ok() {
  g_last_error = SPS_OK;
  return SPS_OK;
}

constexpr int kDetectStep = 1024;

// Blocks per baseline chain for `nb` blocks per row (tuning only).
int stats_seg_for(const sps_plan* p, int64_t nb) {
  if (p->stats_seg > 0) return (int)std::min<int64_t>(p->stats_seg, std::max<int64_t>(nb, 1));
  // ~4k chains: about one per resident wave (256 CUs x 20 waves); longer
  // chains spend less on warm-up recounts and keep fewer windows in flight,
  // which the re-read of samples leaving the window favours (measured).
  // Keep each chain >= 4 windows long.
  const int64_t want_chains = 4096;
  int64_t per_row = (want_chains + p->ndm - 1) / p->ndm;
  if (per_row < 1) per_row = 1;
  int64_t seg = (nb + per_row - 1) / per_row;
  const int64_t min_seg = std::max<int64_t>(64, (4LL * p->baseline_len + 63) / 64);
  if (seg < min_seg) seg = min_seg;
  if (seg > nb) seg = nb;
  if (seg < 1) seg = 1;
  return (int)seg;
}

int auto_stats_seg(const sps_plan* p) { return stats_seg_for(p, p->nblocks); }

// Rows whose first windows are clipped at the row start (they grow from 64
// samples to the full window): there the median and MAD move far from block
// to block and the chain takes the slow queries, so the row's first chain is
// made shorter by four window lengths in blocks (at most half a segment) and
// the others longer (the measured optimum under drifting baselines). `nb`
// blocks per row in `nseg` segments of `seg`; on return seg is the length of
// segments 1, 2, ... and head that of segment 0.
// Samples a block's baseline window reaches past the block's end.
int32_t window_lead(int32_t baseline_len, int window) {
  return window == 1 ? std::max<int32_t>(0, (baseline_len - sps::kStride) / 2) : 0;
}

// Positions up to N + lead + 64 stay inside int32 arithmetic.
bool window_fits(int64_t nsamp, int32_t baseline_len, int window) {
  return nsamp + window_lead(baseline_len, window) + sps::kStride <= (int64_t)INT32_MAX - 8192;
}

void shorten_first_segment(int64_t nb, int64_t window, int32_t nseg, int32_t& seg, int32_t& head) {
  head = seg;
  if (nseg < 2) return;
  const int64_t shift = std::min<int64_t>(4 * window / sps::kStride, seg / 2);
  const int64_t seg2 = (nb + shift + nseg - 1) / nseg;
  const int64_t h = nb - (int64_t)(nseg - 1) * seg2;
  if (h >= 1 && h <= seg2) {
    seg = (int32_t)seg2;
    head = (int32_t)h;
  }
}

// Chain segments of a search's rows (automatic segmentation shortens the first).
void stats_segments_clipped(const sps_plan* p, int64_t nb, int32_t& seg, int32_t& head, int32_t& nseg) {
  seg = stats_seg_for(p, nb);
  nseg = (int32_t)((nb + seg - 1) / seg);
  head = seg;
  if (p->stats_seg == 0) shorten_first_segment(nb, std::min<int64_t>(p->baseline_len, p->nsamp), nseg, seg, head);
}

// Positions per detection segment for rows of `npos` positions (tuning only).
int detect_seg_for(const sps_plan* p, int64_t npos) {
  int64_t seg = p->detect_seg;
  if (seg <= 0) {
    // ~8192 workgroups; each segment >= 4 x max_width so the halo stays small
    const int64_t total = (int64_t)p->ndm * npos;
    seg = total / 8192;
    seg = std::max<int64_t>(seg, 4LL * p->max_width);
  }
  seg = ((seg + kDetectStep - 1) / kDetectStep) * kDetectStep;
  if (seg < kDetectStep) seg = kDetectStep;
  const int64_t nmax = (npos + kDetectStep - 1) / kDetectStep * kDetectStep;
  if (seg > nmax) seg = nmax;
  if (seg < kDetectStep) seg = kDetectStep;
  return (int)seg;
}

int auto_detect_seg(const sps_plan* p) { return detect_seg_for(p, p->nsamp); }

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

hipEvent_t take_event(sps_plan* p) {
  if (!p->ev_free->empty()) {
    hipEvent_t e = p->ev_free->back();
    p->ev_free->pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Records an event on `s` when timing is on; returns it (or null).
hipEvent_t mark(sps_plan* p, hipStream_t s) {
  if (!p->timing) return nullptr;
  hipEvent_t e = take_event(p);
  if (e && hipEventRecord(e, s) != hipSuccess) {
    (void)hipGetLastError();
    p->ev_free->push_back(e);
    return nullptr;
  }
  return e;
}

void span(sps_plan* p, int stage, hipEvent_t a, hipEvent_t b) {
  if (a && b) p->ev_pending->push_back({stage, {a, b}});
}

// Make room for the run summaries of multi-segment rows (host-synchronous).
int64_t frag_need(const sps_plan* p) {
  const int64_t seg = auto_detect_seg(p);
  const int64_t nseg = (p->nsamp + seg - 1) / seg;
  return nseg > 1 ? (int64_t)p->ndm * p->nw * nseg : 0;
}

bool plan_shape_ok(int32_t ndm, int64_t nsamp, int32_t max_width, int32_t baseline_len, float snr_thresh) {
  return ndm >= 1 && nsamp >= 1 && nsamp <= (int64_t)INT32_MAX - 8192 && is_pow2(max_width) &&
         max_width <= SPS_MAX_WIDTH_LIMIT && baseline_len >= 1 && baseline_len <= SPS_MAX_BASELINE_LEN &&
         std::isfinite(snr_thresh) && snr_thresh > 0.0f;
}

// Shape, widths and default tuning of a plan (no device memory, no events).
void plan_params(sps_plan* p, int32_t ndm, int64_t nsamp, int32_t max_width, int32_t baseline_len, float snr_thresh) {
  std::memset(p, 0, sizeof(*p));
  p->ndm = ndm;
  p->nsamp = (int32_t)nsamp;
  p->max_width = max_width;
  p->baseline_len = baseline_len;
  p->thresh = snr_thresh;
  p->nblocks = (int32_t)((nsamp + sps::kStride - 1) / sps::kStride);
  p->nw = 0;
  for (int w = 1; w <= max_width; w <<= 1) {
    p->sqrtw[p->nw] = std::sqrt((double)w);  // correctly rounded (IEEE sqrt)
    ++p->nw;
  }
  p->max_cands = 1LL << 24;
  p->hist_bins = 4096;
}

// Marks the end of a call's device work on `s` (plans with an event only).
int finish(sps_plan* p, hipStream_t s) {
  if (!p->done) return SPS_OK;
  if (hipEventRecord(p->done, s) != hipSuccess) {
    (void)hipGetLastError();
    return SPS_ERR_HIP;
  }
  p->pending = true;
  return SPS_OK;
}

int64_t domain_bound(int32_t max_width) {
  const int64_t b = (int64_t)INT32_MAX / (2LL * (max_width > 0 ? max_width : 1));
  return b < (1LL << 24) - 1 ? b : (1LL << 24) - 1;
}

// SPS_ATTR_VALIDATE: check n samples at x on the device and wait for the
// answer. SPS_OK, SPS_ERR_DOMAIN or SPS_ERR_HIP.
int check_domain(sps_plan* p, const float* x, int64_t n, hipStream_t s) {
  if (!p->validate) return SPS_OK;
  uint32_t h = 0;
  if (sps::launch_zero_u32(p->d_flag, 1, s) != hipSuccess ||
      sps::launch_validate(x, n, (float)domain_bound(p->max_width), p->d_flag, s) != hipSuccess ||
      hipMemcpyAsync(&h, p->d_flag, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    (void)hipGetLastError();
    return SPS_ERR_HIP;
  }
  return h ? SPS_ERR_DOMAIN : SPS_OK;
}

int ensure_frag(sps_plan* p) {
  const int64_t need = frag_need(p);
  if (need <= p->frag_cap) return SPS_OK;
  if (p->d_frag) {
    if (p->pending) (void)hipEventSynchronize(p->done);
    (void)hipFree(p->d_frag);
    p->d_frag = nullptr;
    p->frag_cap = 0;
  }
  if (hipMalloc(&p->d_frag, (size_t)need * sizeof(sps::RunSum)) != hipSuccess) {
    (void)hipGetLastError();
    p->d_frag = nullptr;
    return SPS_ERR_OOM;
  }
  p->frag_cap = need;
  return SPS_OK;
}

}  // namespace

static int launch_stats(sps_plan* p, const float* d_series, hipStream_t stream, int32_t* d_median,
                        int32_t* d_mad);
static int launch_wstats(sps_plan* p, const float* d_series, hipStream_t stream, const int32_t* d_median,
                         int32_t* center, int32_t* mad);

extern "C" {

int sps_last_error(void) { return g_last_error; }

const char* sps_error_string(int code) {
  switch (code) {
    case SPS_OK: return "success";
    case SPS_ERR_INVALID_ARG: return "invalid argument";
    case SPS_ERR_OOM: return "device memory allocation failed";
    case SPS_ERR_HIP: return "HIP runtime error";
    case SPS_ERR_OVERFLOW: return "candidate buffer overflow";
    case SPS_ERR_DOMAIN: return "input outside the supported domain";
    case SPS_ERR_SCRATCH: return "block larger than the allocation-free search's fixed scratch";
    default: return "unknown error";
  }
}

sps_plan* sps_plan_create(int32_t ndm, int64_t nsamp, int32_t max_width, int32_t baseline_len, float snr_thresh) {
  if (!plan_shape_ok(ndm, nsamp, max_width, baseline_len, snr_thresh)) {
    fail(SPS_ERR_INVALID_ARG);
    return nullptr;
  }
  sps_plan* p = new (std::nothrow) sps_plan;
  if (!p) {
    fail(SPS_ERR_OOM);
    return nullptr;
  }
  plan_params(p, ndm, nsamp, max_width, baseline_len, snr_thresh);
  p->ev_free = new (std::nothrow) std::vector<hipEvent_t>();
  p->ev_pending = new (std::nothrow) std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>>();
  if (!p->ev_free || !p->ev_pending) {
    delete p->ev_free;
    delete p->ev_pending;
    delete p;
    fail(SPS_ERR_OOM);
    return nullptr;
  }
  if (hipGetDevice(&p->device) != hipSuccess || hipEventCreateWithFlags(&p->done, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    delete p->ev_free;
    delete p->ev_pending;
    delete p;
    fail(SPS_ERR_HIP);
    return nullptr;
  }
  const size_t stats_bytes = (size_t)ndm * p->nblocks * sizeof(int32_t);
  if (hipMalloc(&p->d_med, stats_bytes) != hipSuccess || hipMalloc(&p->d_mad, stats_bytes) != hipSuccess ||
      hipMalloc(&p->d_flag, sizeof(uint32_t)) != hipSuccess ||
      hipMalloc(&p->d_wstat, 2 * (size_t)ndm * p->nw * sizeof(int32_t)) != hipSuccess) {
    (void)hipGetLastError();
    sps_plan_destroy(p);
    fail(SPS_ERR_OOM);
    return nullptr;
  }
  if (ensure_frag(p) != SPS_OK) {
    sps_plan_destroy(p);
    fail(SPS_ERR_OOM);
    return nullptr;
  }
  ok();
  return p;
}

void sps_plan_destroy(sps_plan* p) {
  if (!p) return;
  // only this plan's own work uses its scratch: wait for its last call, not the device
  if (p->pending) (void)hipEventSynchronize(p->done);
  if (p->done) (void)hipEventDestroy(p->done);
  if (p->d_med) (void)hipFree(p->d_med);
  if (p->d_mad) (void)hipFree(p->d_mad);
  if (p->d_frag) (void)hipFree(p->d_frag);
  if (p->d_plain) (void)hipFree(p->d_plain);
  if (p->d_flag) (void)hipFree(p->d_flag);
  if (p->d_wstat) (void)hipFree(p->d_wstat);
  if (p->ev_pending) {
    for (auto& e : *p->ev_pending) {
      (void)hipEventDestroy(e.second.first);
      (void)hipEventDestroy(e.second.second);
    }
    delete p->ev_pending;
  }
  if (p->ev_free) {
    for (auto e : *p->ev_free) (void)hipEventDestroy(e);
    delete p->ev_free;
  }
  delete p;
}

int sps_timing_read(sps_plan* p, double* ms_out, int64_t* nsearch) {
  if (!p || !ms_out || !nsearch) return fail(SPS_ERR_INVALID_ARG);
  for (auto& e : *p->ev_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(e.second.second) != hipSuccess ||
        hipEventElapsedTime(&ms, e.second.first, e.second.second) != hipSuccess) {
      (void)hipGetLastError();
      ms = 0.f;
    }
    p->stage_ms[e.first] += ms;
    // an event may close one span and open the next: return each once
    bool dup_a = false, dup_b = false;
    for (auto f : *p->ev_free) { dup_a |= f == e.second.first; dup_b |= f == e.second.second; }
    if (!dup_a) p->ev_free->push_back(e.second.first);
    if (!dup_b && e.second.second != e.second.first) p->ev_free->push_back(e.second.second);
  }
  p->ev_pending->clear();
  for (int i = 0; i < SPS_NSTAGES; ++i) {
    ms_out[i] = p->stage_ms[i];
    p->stage_ms[i] = 0.0;
  }
  *nsearch = p->nsearch;
  p->nsearch = 0;
  return ok();
}

int sps_plan_set(sps_plan* p, int attr, int64_t v) {
  if (!p) return fail(SPS_ERR_INVALID_ARG);
  switch (attr) {
    case SPS_ATTR_MAX_CANDS:
      if (v < 0 || v > (int64_t)UINT32_MAX) return fail(SPS_ERR_INVALID_ARG);
      p->max_cands = v;
      return ok();
    case SPS_ATTR_STATS_SEG:
      if (v < 0 || v > INT32_MAX) return fail(SPS_ERR_INVALID_ARG);
      p->stats_seg = (int32_t)v;
      return ok();
    case SPS_ATTR_DETECT_SEG:
      if (v < 0 || v > INT32_MAX || (v % kDetectStep) != 0) return fail(SPS_ERR_INVALID_ARG);
      p->detect_seg = (int32_t)v;
      if (ensure_frag(p) != SPS_OK) return fail(SPS_ERR_OOM);
      return ok();
    case SPS_ATTR_HIST_BINS:
      if (v != 4096 && v != 16384) return fail(SPS_ERR_INVALID_ARG);
      p->hist_bins = (int32_t)v;
      return ok();
    case SPS_ATTR_TIMING:
      if (v != 0 && v != 1) return fail(SPS_ERR_INVALID_ARG);
      p->timing = (int)v;
      return ok();
    case SPS_ATTR_VALIDATE:
      if (v != 0 && v != 1) return fail(SPS_ERR_INVALID_ARG);
      p->validate = (int)v;
      return ok();
    case SPS_ATTR_WINDOW:
      if ((v != 0 && v != 1) || !window_fits(p->nsamp, p->baseline_len, (int)v)) return fail(SPS_ERR_INVALID_ARG);
      p->window = (int32_t)v;
      return ok();
    case SPS_ATTR_NORM:
      if (v < 0 || v > 2) return fail(SPS_ERR_INVALID_ARG);
      p->norm = (int32_t)v;
      return ok();
    default:
      return fail(SPS_ERR_INVALID_ARG);
  }
}

int sps_plan_get(const sps_plan* p, int attr, int64_t* v) {
  if (!p || !v) return fail(SPS_ERR_INVALID_ARG);
  switch (attr) {
    case SPS_ATTR_MAX_CANDS: *v = p->max_cands; break;
    case SPS_ATTR_STATS_SEG: *v = auto_stats_seg(p); break;
    case SPS_ATTR_DETECT_SEG: *v = auto_detect_seg(p); break;
    case SPS_ATTR_HIST_BINS: *v = p->hist_bins; break;
    case SPS_ATTR_TIMING: *v = p->timing; break;
    case SPS_ATTR_VALIDATE: *v = p->validate; break;
    case SPS_ATTR_WINDOW: *v = p->window; break;
    case SPS_ATTR_NORM: *v = p->norm; break;
    case SPS_ATTR_NBLOCKS: *v = p->nblocks; break;
    case SPS_ATTR_BLOCK_STRIDE: *v = sps::kStride; break;
    case SPS_ATTR_NWIDTHS: *v = p->nw; break;
    default: return fail(SPS_ERR_INVALID_ARG);
  }
  return ok();
}

int sps_block_stats(sps_plan* p, const float* d_series, hipStream_t stream, int32_t* d_median, int32_t* d_mad) {
  if (!p || !d_series || !d_median || !d_mad) return fail(SPS_ERR_INVALID_ARG);
  hipEvent_t e0 = mark(p, stream);
  const int rc = launch_stats(p, d_series, stream, d_median, d_mad);
  span(p, 0, e0, mark(p, stream));
  if (rc != SPS_OK) return rc;
  if (finish(p, stream) != SPS_OK) return fail(SPS_ERR_HIP);
  return ok();
}

int sps_width_stats(sps_plan* p, const float* d_series, hipStream_t stream, int32_t* d_center, int32_t* d_mad) {
  if (!p || !d_series || !d_center || !d_mad) return fail(SPS_ERR_INVALID_ARG);
  // block medians into the plan's scratch (the residual's baseline), then the series' statistics
  const int32_t saved = p->norm;
  p->norm = 0;
  const int rc = launch_stats(p, d_series, stream, p->d_med, p->d_mad);
  p->norm = saved;
  if (rc != SPS_OK) return rc;
  if (launch_wstats(p, d_series, stream, p->d_med, d_center, d_mad) != SPS_OK) return g_last_error;
  if (finish(p, stream) != SPS_OK) return fail(SPS_ERR_HIP);
  return ok();
}

}  // extern "C"

static int launch_stats(sps_plan* p, const float* d_series, hipStream_t stream, int32_t* d_median, int32_t* d_mad) {
  sps::StatsArgs a;
  a.x = d_series;
  a.ld = p->nsamp;
  a.hist = nullptr;
  a.ldh = 0;
  a.Hx = 0;
  a.N = p->nsamp;
  a.L = p->baseline_len;
  a.lead = window_lead(p->baseline_len, p->window);
  a.nblocks = p->nblocks;
  a.kb_first = 0;
  stats_segments_clipped(p, p->nblocks, a.seg_blocks, a.head_blocks, a.nseg);
  a.nchains = p->ndm * a.nseg;
  a.tmin = nullptr;
  a.med = d_median;
  a.mad = d_mad;
  a.done = nullptr;
  if (sps::launch_block_stats(a, p->hist_bins, stream) != hipSuccess) return fail(SPS_ERR_HIP);
  if (p->norm == 1) {
    const sps::RowMadArgs r{d_series, p->nsamp, p->nsamp, p->nblocks, p->nblocks, p->ndm, d_median, d_mad};
    if (sps::launch_row_mad(r, stream) != hipSuccess) return fail(SPS_ERR_HIP);
  }
  return ok();
}

// Per-width scales (SPS_ATTR_NORM = 2): c_w and MAD_w of every (row, width)
// from the block medians into center / mad ([ndm][nw] each).
static int launch_wstats(sps_plan* p, const float* d_series, hipStream_t stream, const int32_t* d_median,
                         int32_t* center, int32_t* mad) {
  const sps::WidthStatsArgs w{d_series, p->nsamp, p->nsamp, p->nblocks, p->ndm, p->nw, d_median, center, mad};
  if (sps::launch_width_stats(w, stream) != hipSuccess) return fail(SPS_ERR_HIP);
  return ok();
}

// The fused search of one block: counter reset, block statistics into
// med/mad, fused detection (segments of seg_len positions; run summaries of
// segment edges in frag when a row has several segments), fix-up.
static int enqueue_search(sps_plan* p, const float* d_series, hipStream_t stream, sps_cand* d_cands,
                          uint32_t* d_ncand, int32_t* med, int32_t* mad, sps::RunSum* frag, int32_t seg_len) {
  hipEvent_t e0 = mark(p, stream);
  if (sps::launch_zero_u32(d_ncand, 1, stream) != hipSuccess) return SPS_ERR_HIP;
  hipEvent_t e1 = mark(p, stream);
  if (launch_stats(p, d_series, stream, med, mad) != SPS_OK) return g_last_error;
  const bool wnorm = p->norm == 2;
  int32_t* wc = wnorm ? p->d_wstat : nullptr;
  int32_t* wm = wnorm ? p->d_wstat + (size_t)p->ndm * p->nw : nullptr;
  if (wnorm && launch_wstats(p, d_series, stream, med, wc, wm) != SPS_OK) return g_last_error;
  hipEvent_t e2 = mark(p, stream);
  sps::DetectArgs d;
  d.seg_len = seg_len;
  d.nseg = (p->nsamp + seg_len - 1) / seg_len;
  d.x = d_series;
  d.ld = p->nsamp;
  d.hist = nullptr;
  d.ldh = 0;
  d.Hx = 0;
  d.seg_base = 0;
  d.e_first = 0;
  d.tmin = nullptr;
  d.sample_offset = 0;
  d.keep_edges = 0;
  d.N = p->nsamp;
  d.nblocks = p->nblocks;
  d.nw = p->nw;
  d.maxw = p->max_width;
  d.med = med;
  d.mad = mad;
  d.wmad = wm;
  d.theta = (double)p->thresh;
  // a per-width scale measures the filtered series itself: no sqrt(w)
  for (int j = 0; j < sps::kMaxWidths; ++j) d.sqrtw[j] = j < p->nw ? (wnorm ? 1.0 : p->sqrtw[j]) : 0.0;
  d.rows = p->ndm;
  d.row_offset = 0;
  d.cands = d_cands;
  d.ncand = d_ncand;
  d.cap = (uint32_t)p->max_cands;
  d.frag = frag;
  d.done = nullptr;
  d.done_target = 0;
  if (sps::launch_detect(d, stream) != hipSuccess) return SPS_ERR_HIP;
  hipEvent_t e3 = mark(p, stream);
  if (sps::launch_fixup(d, stream) != hipSuccess) return SPS_ERR_HIP;
  hipEvent_t e4 = mark(p, stream);
  span(p, 2, e0, e1);
  span(p, 0, e1, e2);
  span(p, 1, e2, e3);
  span(p, 2, e3, e4);
  if (p->timing) ++p->nsearch;
  return SPS_OK;
}

extern "C" {

int sps_search(sps_plan* p, const float* d_series, hipStream_t stream, sps_cand* d_cands, uint32_t* d_ncand) {
  if (!p || !d_series || !d_ncand || (!d_cands && p->max_cands > 0)) return fail(SPS_ERR_INVALID_ARG);
  const int32_t seg_len = auto_detect_seg(p);
  const int32_t nseg = (p->nsamp + seg_len - 1) / seg_len;
  if (nseg > 1 && (int64_t)p->ndm * p->nw * nseg > p->frag_cap) return fail(SPS_ERR_INVALID_ARG);
  {
    const int rc = check_domain(p, d_series, (int64_t)p->ndm * p->nsamp, stream);
    if (rc != SPS_OK) return fail(rc);
  }
  const int rc = enqueue_search(p, d_series, stream, d_cands, d_ncand, p->d_med, p->d_mad, p->d_frag, seg_len);
  if (rc != SPS_OK) return fail(rc);
  if (finish(p, stream) != SPS_OK) return fail(SPS_ERR_HIP);
  return ok();
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free search. Its scratch (block medians and MADs, run summaries
// of detection-segment edges) is one file-scope device array: every GPU the
// library runs on holds its own copy until the process ends, every call on a
// GPU shares that GPU's copy, and the array keeps the last call's contents.
// Host code never uses the array's name as an address: the device address is
// looked up once per device and kept in noalloc_ptr.

static __device__ __align__(256) unsigned char scratch[SPS_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex noalloc_mu;
void* noalloc_ptr[kMaxDevices];

// Device address of the current device's scratch (looked up on the first call per device).
int noalloc_scratch(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return SPS_ERR_HIP;
  }
  if (dev < 0 || dev >= kMaxDevices) return SPS_ERR_HIP;
  std::lock_guard<std::mutex> lock(noalloc_mu);
  if (!noalloc_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return SPS_ERR_HIP;
    }
    noalloc_ptr[dev] = ptr;
  }
  *out = noalloc_ptr[dev];
  return SPS_OK;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Layout of a search's scratch in the fixed array: medians, MADs, then run
// summaries. Detection segments follow the plan's rule, or cover whole rows
// (no summaries) when the summaries would not fit. false: too large.
bool noalloc_layout(const sps_plan* p, int32_t* seg_len, size_t* off_mad, size_t* off_frag) {
  const size_t stats = align256((size_t)p->ndm * p->nblocks * sizeof(int32_t));
  *off_mad = stats;
  *off_frag = 2 * stats;
  if (2 * stats > (size_t)SPS_NOALLOC_SCRATCH_BYTES) return false;
  int32_t seg = auto_detect_seg(p);
  const int64_t nseg = (p->nsamp + seg - 1) / seg;
  const size_t frag = nseg > 1 ? (size_t)p->ndm * p->nw * nseg * sizeof(sps::RunSum) : 0;
  if (2 * stats + frag > (size_t)SPS_NOALLOC_SCRATCH_BYTES)
    seg = (int32_t)(((int64_t)p->nsamp + kDetectStep - 1) / kDetectStep * kDetectStep);  // one segment per row
  *seg_len = seg;
  return true;
}

}  // namespace

extern "C" {

int sps_search_noalloc(int32_t ndm, int64_t nsamp, int32_t max_width, int32_t baseline_len, float snr_thresh,
                       const float* d_series, hipStream_t stream, sps_cand* d_cands, uint32_t* d_ncand,
                       int64_t max_cands) {
  if (!plan_shape_ok(ndm, nsamp, max_width, baseline_len, snr_thresh) || !d_series || !d_ncand || max_cands < 0 ||
      max_cands > (int64_t)UINT32_MAX || (!d_cands && max_cands > 0))
    return fail(SPS_ERR_INVALID_ARG);
  sps_plan p;  // parameters only: no device memory, no events
  plan_params(&p, ndm, nsamp, max_width, baseline_len, snr_thresh);
  p.max_cands = max_cands;
  int32_t seg_len = 0;
  size_t off_mad = 0, off_frag = 0;
  if (!noalloc_layout(&p, &seg_len, &off_mad, &off_frag)) return fail(SPS_ERR_SCRATCH);
  void* base = nullptr;
  {
    const int rc = noalloc_scratch(&base);
    if (rc != SPS_OK) return fail(rc);
  }
  // nothing in the scratch needs to start at zero: the statistics kernel writes
  // every block's median and MAD, and the detection kernel every run summary,
  // before anything reads them
  char* b = static_cast<char*>(base);
  const int rc = enqueue_search(&p, d_series, stream, d_cands, d_ncand, reinterpret_cast<int32_t*>(b),
                                reinterpret_cast<int32_t*>(b + off_mad), reinterpret_cast<sps::RunSum*>(b + off_frag),
                                seg_len);
  if (rc != SPS_OK) return fail(rc);
  return ok();
}

int sps_search_plain(sps_plan* p, const float* d_series, hipStream_t stream, sps_cand* d_cands, uint32_t* d_ncand) {
  if (!p || !d_series || !d_ncand || (!d_cands && p->max_cands > 0)) return fail(SPS_ERR_INVALID_ARG);
  if (p->norm == 2) return fail(SPS_ERR_INVALID_ARG);  // the per-stage path keeps per-block or per-row scales only
  {
    const int rc = check_domain(p, d_series, (int64_t)p->ndm * p->nsamp, stream);
    if (rc != SPS_OK) return fail(rc);
  }
  const int strip = 4096;  // positions per wave in the peak stage
  const int nstrip = (p->nsamp + strip - 1) / strip;
  const size_t n = (size_t)p->ndm * p->nsamp;
  const size_t bytes_r = n * 4, bytes_p = (size_t)p->ndm * (p->nsamp + 1) * 4, bytes_s = n * 4, bytes_f = n,
               bytes_frag = (size_t)p->ndm * nstrip * sizeof(sps::RunSum);
  auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
  const size_t need = al(bytes_r) + al(bytes_p) + al(bytes_s) + al(bytes_f) + al(bytes_frag);
  if (p->plain_bytes < need) {
    if (p->d_plain) {
      if (p->pending) (void)hipEventSynchronize(p->done);
      (void)hipFree(p->d_plain);
      p->d_plain = nullptr;
      p->plain_bytes = 0;
    }
    if (hipMalloc(&p->d_plain, need) != hipSuccess) {
      (void)hipGetLastError();
      p->d_plain = nullptr;
      return fail(SPS_ERR_OOM);
    }
    p->plain_bytes = need;
  }
  char* w = static_cast<char*>(p->d_plain);
  sps::PlainArgs a;
  a.x = d_series;
  a.N = p->nsamp;
  a.nblocks = p->nblocks;
  a.rows = p->ndm;
  a.med = p->d_med;
  a.mad = p->d_mad;
  a.r = reinterpret_cast<int32_t*>(w); w += al(bytes_r);
  a.P = reinterpret_cast<uint32_t*>(w); w += al(bytes_p);
  a.S = reinterpret_cast<int32_t*>(w); w += al(bytes_s);
  a.flag = reinterpret_cast<uint8_t*>(w); w += al(bytes_f);
  a.frag = reinterpret_cast<sps::RunSum*>(w);
  a.strip = strip;
  a.nstrip = nstrip;
  a.theta = (double)p->thresh;
  a.cands = d_cands;
  a.ncand = d_ncand;
  a.cap = (uint32_t)p->max_cands;
  hipEvent_t e0 = mark(p, stream);
  if (sps::launch_zero_u32(d_ncand, 1, stream) != hipSuccess) return fail(SPS_ERR_HIP);
  if (launch_stats(p, d_series, stream, p->d_med, p->d_mad) != SPS_OK) return g_last_error;
  if (sps::launch_plain_prepare(a, stream) != hipSuccess) return fail(SPS_ERR_HIP);
  for (int j = 0; j < p->nw; ++j) {
    a.w = 1 << j;
    a.sqrtw = p->sqrtw[j];
    if (sps::launch_plain_width(a, stream) != hipSuccess) return fail(SPS_ERR_HIP);
  }
  span(p, 3, e0, mark(p, stream));
  if (finish(p, stream) != SPS_OK) return fail(SPS_ERR_HIP);
  return ok();
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Streaming: gulp after gulp of one observation, the carried state on device.

constexpr int kGraphCache = 8;

struct sps_stream {
  sps_plan* plan;       // borrowed: gulp shape and tuning
  int32_t Hx;           // history samples kept per row (multiple of 1024)
  int32_t Hb;           // Hx / 64
  int32_t nbv;          // virtual blocks per row: Hb + nsamp / 64
  int32_t Nv;           // virtual samples per row: Hx + nsamp
  int32_t seg_base;     // first detection segment start (virtual)
  int32_t seg_len, nseg;
  int cur;              // which of the two history buffers is current
  float* hist[2];       // [ndm][Hx]
  int32_t* med[2];      // [ndm][nbv]
  int32_t* mad[2];
  sps::RunSum* carry;   // [ndm][nw]
  sps::RunSum* frag;    // [ndm][nw][nseg]
  int32_t* tmin;        // device: virtual index of the stream's first sample (clamped at 0)
  int64_t pushed;       // samples pushed so far
  // captured gulp steps, one per history parity, for each of a few recently
  // used (gulp, cands, ncand) buffer triples (least recently used replaced)
  hipStream_t cap_stream;
  struct GraphEntry {
    const void* key[3];
    int32_t norm;  // the scale the graph was captured with
    hipGraphExec_t exec[2];
    uint64_t last_use;
  } graphs[kGraphCache];
  uint64_t graph_clock;
  hipEvent_t done;      // end of the last push or flush (destroy waits for it)
  bool pending;
};

namespace {

struct StreamHeader {
  uint64_t magic;
  int64_t pushed;
  int32_t ndm, nsamp, Hx, nw, max_width, baseline_len;
  int32_t tmin;
  int32_t pad;
};
constexpr uint64_t kStreamMagic = 0x5350535354524D32ull;  // "SPSSTRM2"

// History length, virtual row and detection segments of a stream on plan p.
// Arithmetic a stream can run: the trailing window (a centred one would wait
// for the next gulp), with the block scale or one row scale per gulp (the
// per-width scale needs the whole filtered series).
bool stream_plan_ok(const sps_plan* p) { return p->window == 0 && p->norm != 2; }

bool stream_geometry(const sps_plan* p, sps_stream* s) {
  const int64_t need = std::max<int64_t>(p->baseline_len, p->max_width);
  s->Hx = (int32_t)((need + kDetectStep - 1) / kDetectStep * kDetectStep);
  s->Hb = s->Hx / sps::kStride;
  s->nbv = s->Hb + p->nsamp / sps::kStride;
  if ((int64_t)s->Hx + p->nsamp > (int64_t)INT32_MAX - 8192) return false;
  s->Nv = s->Hx + p->nsamp;
  // positions of a push are those whose window ends inside the gulp
  int64_t first = (int64_t)s->Hx + 1 - p->max_width;
  if (first < 0) first = 0;
  s->seg_base = (int32_t)(first / kDetectStep * kDetectStep);
  s->seg_len = detect_seg_for(p, s->Nv - s->seg_base);
  s->nseg = (s->Nv - s->seg_base + s->seg_len - 1) / s->seg_len;
  return true;
}

uint64_t stream_device_bytes(const sps_stream* s) {
  const sps_plan* p = s->plan;
  return 2ull * ((uint64_t)p->ndm * s->Hx * sizeof(float) + 2ull * p->ndm * s->nbv * sizeof(int32_t)) +
         (uint64_t)p->ndm * p->nw * (1 + s->nseg) * sizeof(sps::RunSum) + sizeof(int32_t);
}

uint64_t stream_state_bytes(const sps_stream* s) {
  const sps_plan* p = s->plan;
  return sizeof(StreamHeader) + (uint64_t)p->ndm * s->Hx * sizeof(float) +
         2ull * p->ndm * s->Hb * sizeof(int32_t) + (uint64_t)p->ndm * p->nw * sizeof(sps::RunSum);
}

sps::StreamArgs stream_args(sps_stream* s, const float* d_gulp, sps_cand* d_cands, uint32_t* d_ncand) {
  sps_plan* p = s->plan;
  sps::StreamArgs a;
  a.rows = p->ndm;
  a.nw = p->nw;
  a.nseg = s->nseg;
  a.Hx = s->Hx;
  a.Hb = s->Hb;
  a.ngulp = p->nsamp;
  a.nbv = s->nbv;
  a.frag = s->frag;
  a.carry = s->carry;
  a.gulp = d_gulp;
  a.hist_in = s->hist[s->cur];
  a.hist_out = s->hist[s->cur ^ 1];
  a.med_in = s->med[s->cur];
  a.mad_in = s->mad[s->cur];
  a.med_out = s->med[s->cur ^ 1];
  a.mad_out = s->mad[s->cur ^ 1];
  a.tmin = s->tmin;
  a.row_offset = 0;
  a.cands = d_cands;
  a.ncand = d_ncand;
  a.cap = (uint32_t)p->max_cands;
  return a;
}

void stream_free(sps_stream* s) {
  if (!s) return;
  for (int i = 0; i < 2; ++i) {
    if (s->hist[i]) (void)hipFree(s->hist[i]);
    if (s->med[i]) (void)hipFree(s->med[i]);
    if (s->mad[i]) (void)hipFree(s->mad[i]);
  }
  if (s->carry) (void)hipFree(s->carry);
  if (s->frag) (void)hipFree(s->frag);
  if (s->tmin) (void)hipFree(s->tmin);
  for (auto& e : s->graphs)
    for (int i = 0; i < 2; ++i)
      if (e.exec[i]) (void)hipGraphExecDestroy(e.exec[i]);
  if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
  if (s->done) (void)hipEventDestroy(s->done);
  delete s;
}

// Marks the end of a push or flush on `st`.
int stream_finish(sps_stream* s, hipStream_t st) {
  if (hipEventRecord(s->done, st) != hipSuccess) {
    (void)hipGetLastError();
    return SPS_ERR_HIP;
  }
  s->pending = true;
  return SPS_OK;
}

// Zero the carried state and put the stream start at the first sample of
// the next push (host-synchronous).
int stream_reset(sps_stream* s) {
  const sps_plan* p = s->plan;
  for (int i = 0; i < 2; ++i) {
    if (hipMemset(s->hist[i], 0, (size_t)p->ndm * s->Hx * sizeof(float)) != hipSuccess) return SPS_ERR_HIP;
    if (hipMemset(s->med[i], 0, (size_t)p->ndm * s->nbv * sizeof(int32_t)) != hipSuccess) return SPS_ERR_HIP;
    if (hipMemset(s->mad[i], 0, (size_t)p->ndm * s->nbv * sizeof(int32_t)) != hipSuccess) return SPS_ERR_HIP;
  }
  if (hipMemset(s->carry, 0, (size_t)p->ndm * p->nw * sizeof(sps::RunSum)) != hipSuccess) return SPS_ERR_HIP;
  const int32_t t0 = s->Hx;
  if (hipMemcpy(s->tmin, &t0, sizeof(t0), hipMemcpyHostToDevice) != hipSuccess) return SPS_ERR_HIP;
  s->cur = 0;
  s->pushed = 0;
  return SPS_OK;
}

}  // namespace

extern "C" {

int sps_stream_create(sps_plan* p, sps_stream** out) {
  if (!p || !out) return fail(SPS_ERR_INVALID_ARG);
  *out = nullptr;
  if (p->nsamp % sps::kStride != 0) return fail(SPS_ERR_INVALID_ARG);  // gulps must hold whole blocks
  if (!stream_plan_ok(p)) return fail(SPS_ERR_INVALID_ARG);
  sps_stream* s = new (std::nothrow) sps_stream;
  if (!s) return fail(SPS_ERR_OOM);
  std::memset(s, 0, sizeof(*s));
  s->plan = p;
  if (!stream_geometry(p, s)) {
    delete s;
    return fail(SPS_ERR_INVALID_ARG);
  }
  bool okm = true;
  for (int i = 0; i < 2 && okm; ++i) {
    okm = hipMalloc(&s->hist[i], (size_t)p->ndm * s->Hx * sizeof(float)) == hipSuccess &&
          hipMalloc(&s->med[i], (size_t)p->ndm * s->nbv * sizeof(int32_t)) == hipSuccess &&
          hipMalloc(&s->mad[i], (size_t)p->ndm * s->nbv * sizeof(int32_t)) == hipSuccess;
  }
  okm = okm && hipEventCreateWithFlags(&s->done, hipEventDisableTiming) == hipSuccess;
  okm = okm && hipMalloc(&s->carry, (size_t)p->ndm * p->nw * sizeof(sps::RunSum)) == hipSuccess &&
        hipMalloc(&s->frag, (size_t)p->ndm * p->nw * s->nseg * sizeof(sps::RunSum)) == hipSuccess &&
        hipMalloc(&s->tmin, sizeof(int32_t)) == hipSuccess;
  if (!okm) {
    (void)hipGetLastError();
    stream_free(s);
    return fail(SPS_ERR_OOM);
  }
  if (stream_reset(s) != SPS_OK) {
    stream_free(s);
    return fail(SPS_ERR_HIP);
  }
  *out = s;
  return ok();
}

void sps_stream_destroy(sps_stream* s) {
  if (!s) return;
  // only this stream's own pushes use its buffers: wait for the last one, not the device
  if (s->pending) (void)hipEventSynchronize(s->done);
  stream_free(s);
}

}  // extern "C"

namespace {

// Statistics of one gulp of stream s reading history buffer c: only the
// gulp's blocks, windows reaching back into the history.
sps::StatsArgs stream_stats_args(const sps_stream* s, const float* d_gulp, int c) {
  const sps_plan* p = s->plan;
  sps::StatsArgs a;
  a.x = d_gulp;
  a.ld = p->nsamp;
  a.hist = s->hist[c];
  a.ldh = s->Hx;
  a.Hx = s->Hx;
  a.N = s->Nv;
  a.L = p->baseline_len;
  a.lead = 0;  // streams use the trailing window only
  a.nblocks = s->nbv;
  a.kb_first = s->Hb;
  a.seg_blocks = stats_seg_for(p, s->nbv - s->Hb);
  a.head_blocks = a.seg_blocks;
  a.nseg = (s->nbv - s->Hb + a.seg_blocks - 1) / a.seg_blocks;
  a.nchains = p->ndm * a.nseg;
  a.tmin = s->tmin;
  a.med = s->med[c];
  a.mad = s->mad[c];
  a.done = nullptr;
  return a;
}

// One row scale per gulp (SPS_ATTR_NORM = 1): the row MAD of the gulp's
// residuals, written to the gulp's blocks of history buffer c.
sps::RowMadArgs stream_row_mad_args(const sps_stream* s, const float* d_gulp, int c) {
  const sps_plan* p = s->plan;
  return sps::RowMadArgs{d_gulp, p->nsamp, (int32_t)p->nsamp, s->nbv - s->Hb, s->nbv, p->ndm,
                         s->med[c] + s->Hb, s->mad[c] + s->Hb};
}

// Detection of one gulp of stream s reading history buffer c: window ends
// inside the gulp; runs at segment edges are left to k_stream_fold.
sps::DetectArgs stream_detect_args(const sps_stream* s, const float* d_gulp, sps_cand* d_cands, uint32_t* d_ncand,
                                   int c) {
  const sps_plan* p = s->plan;
  sps::DetectArgs d;
  d.x = d_gulp;
  d.ld = p->nsamp;
  d.hist = s->hist[c];
  d.ldh = s->Hx;
  d.Hx = s->Hx;
  d.N = s->Nv;
  d.nblocks = s->nbv;
  d.nw = p->nw;
  d.maxw = p->max_width;
  d.med = s->med[c];
  d.mad = s->mad[c];
  d.wmad = nullptr;  // streams use the per-block scale only
  d.theta = (double)p->thresh;
  for (int j = 0; j < sps::kMaxWidths; ++j) d.sqrtw[j] = j < p->nw ? p->sqrtw[j] : 0.0;
  d.seg_base = s->seg_base;
  d.seg_len = s->seg_len;
  d.nseg = s->nseg;
  d.rows = p->ndm;
  d.e_first = s->Hx + 1;
  d.tmin = s->tmin;
  d.sample_offset = s->Hx;
  d.keep_edges = 1;
  d.row_offset = 0;
  d.cands = d_cands;
  d.ncand = d_ncand;
  d.cap = (uint32_t)p->max_cands;
  d.frag = s->frag;
  d.done = nullptr;
  d.done_target = 0;
  return d;
}

// Enqueue one gulp step reading history buffer `c` (no host state changes;
// capturable: kernels only). `timed`: record tracing events.
int stream_enqueue(sps_stream* s, const float* d_gulp, hipStream_t stream, sps_cand* d_cands, uint32_t* d_ncand,
                   int c, bool timed) {
  sps_plan* p = s->plan;
  struct TimingGuard {  // tracing events are not recorded into captured graphs
    sps_plan* p;
    int saved;
    ~TimingGuard() { p->timing = saved; }
  } guard{p, p->timing};
  if (!timed) p->timing = 0;
  hipEvent_t e0 = mark(p, stream);
  if (sps::launch_zero_u32(d_ncand, 1, stream) != hipSuccess) return SPS_ERR_HIP;
  hipEvent_t e1 = mark(p, stream);
  const sps::StatsArgs a = stream_stats_args(s, d_gulp, c);
  if (sps::launch_block_stats(a, p->hist_bins, stream) != hipSuccess) return SPS_ERR_HIP;
  if (p->norm == 1 && sps::launch_row_mad(stream_row_mad_args(s, d_gulp, c), stream) != hipSuccess)
    return SPS_ERR_HIP;
  hipEvent_t e2 = mark(p, stream);
  const sps::DetectArgs d = stream_detect_args(s, d_gulp, d_cands, d_ncand, c);
  if (sps::launch_detect(d, stream) != hipSuccess) return SPS_ERR_HIP;
  hipEvent_t e3 = mark(p, stream);
  sps::StreamArgs sa = stream_args(s, d_gulp, d_cands, d_ncand);
  sa.hist_in = s->hist[c];
  sa.hist_out = s->hist[c ^ 1];
  sa.med_in = s->med[c];
  sa.mad_in = s->mad[c];
  sa.med_out = s->med[c ^ 1];
  sa.mad_out = s->mad[c ^ 1];
  if (sps::launch_stream_fold(sa, stream) != hipSuccess) return SPS_ERR_HIP;
  if (sps::launch_stream_advance(sa, stream) != hipSuccess) return SPS_ERR_HIP;
  hipEvent_t e4 = mark(p, stream);
  span(p, 2, e0, e1);
  span(p, 0, e1, e2);
  span(p, 1, e2, e3);
  span(p, 2, e3, e4);
  if (p->timing) ++p->nsearch;
  return SPS_OK;
}

}  // namespace

extern "C" {

int sps_stream_push(sps_stream* s, const float* d_gulp, hipStream_t stream, sps_cand* d_cands, uint32_t* d_ncand,
                    int64_t* gulp_offset) {
  if (!s || !d_gulp || !d_ncand || (!d_cands && s->plan->max_cands > 0)) return fail(SPS_ERR_INVALID_ARG);
  if (!stream_plan_ok(s->plan)) return fail(SPS_ERR_INVALID_ARG);  // attributes changed since create
  {
    const int rc = check_domain(s->plan, d_gulp, (int64_t)s->plan->ndm * s->plan->nsamp, stream);
    if (rc != SPS_OK) return fail(rc);
  }
  const int rc = stream_enqueue(s, d_gulp, stream, d_cands, d_ncand, s->cur, true);
  if (rc != SPS_OK) return fail(rc);
  if (stream_finish(s, stream) != SPS_OK) return fail(SPS_ERR_HIP);
  if (gulp_offset) *gulp_offset = s->pushed;
  s->pushed += s->plan->nsamp;
  s->cur ^= 1;
  return ok();
}

int sps_stream_push_graph(sps_stream* s, const float* d_gulp, hipStream_t stream, sps_cand* d_cands,
                          uint32_t* d_ncand, int64_t* gulp_offset) {
  if (!s || !d_gulp || !d_ncand || (!d_cands && s->plan->max_cands > 0)) return fail(SPS_ERR_INVALID_ARG);
  if (!stream_plan_ok(s->plan)) return fail(SPS_ERR_INVALID_ARG);  // attributes changed since create
  {
    const int rc = check_domain(s->plan, d_gulp, (int64_t)s->plan->ndm * s->plan->nsamp, stream);
    if (rc != SPS_OK) return fail(rc);
  }
  sps_stream::GraphEntry* hit = nullptr;
  for (auto& e : s->graphs)
    if (e.exec[0] && e.key[0] == d_gulp && e.key[1] == d_cands && e.key[2] == d_ncand && e.norm == s->plan->norm)
      hit = &e;
  if (!hit) {
    for (auto& e : s->graphs)
      if (!e.exec[0]) {
        hit = &e;
        break;
      }
    if (!hit) {
      hit = &s->graphs[0];
      for (auto& e : s->graphs)
        if (e.last_use < hit->last_use) hit = &e;
    }
    for (int i = 0; i < 2; ++i) {
      if (hit->exec[i]) (void)hipGraphExecDestroy(hit->exec[i]);
      hit->exec[i] = nullptr;
    }
    hit->key[0] = hit->key[1] = hit->key[2] = nullptr;
    if (!s->cap_stream && hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking) != hipSuccess)
      return fail(SPS_ERR_HIP);
    for (int i = 0; i < 2; ++i) {
      hipGraph_t g = nullptr;
      if (hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return fail(SPS_ERR_HIP);
      const int rc = stream_enqueue(s, d_gulp, s->cap_stream, d_cands, d_ncand, i, false);
      const hipError_t ec = hipStreamEndCapture(s->cap_stream, &g);
      if (rc != SPS_OK || ec != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        if (hit->exec[0]) (void)hipGraphExecDestroy(hit->exec[0]);
        hit->exec[0] = nullptr;
        return fail(SPS_ERR_HIP);
      }
      const hipError_t ei = hipGraphInstantiate(&hit->exec[i], g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ei != hipSuccess) {
        hit->exec[i] = nullptr;
        if (hit->exec[0]) (void)hipGraphExecDestroy(hit->exec[0]);
        hit->exec[0] = nullptr;
        (void)hipGetLastError();
        return fail(SPS_ERR_HIP);
      }
    }
    hit->key[0] = d_gulp;
    hit->key[1] = d_cands;
    hit->key[2] = d_ncand;
    hit->norm = s->plan->norm;
  }
  hit->last_use = ++s->graph_clock;
  if (hipGraphLaunch(hit->exec[s->cur], stream) != hipSuccess) return fail(SPS_ERR_HIP);
  if (stream_finish(s, stream) != SPS_OK) return fail(SPS_ERR_HIP);
  if (gulp_offset) *gulp_offset = s->pushed;
  s->pushed += s->plan->nsamp;
  s->cur ^= 1;
  return ok();
}

int sps_stream_flush(sps_stream* s, hipStream_t stream, sps_cand* d_cands, uint32_t* d_ncand, int64_t* end_offset) {
  if (!s || !d_ncand || (!d_cands && s->plan->max_cands > 0)) return fail(SPS_ERR_INVALID_ARG);
  if (sps::launch_zero_u32(d_ncand, 1, stream) != hipSuccess) return fail(SPS_ERR_HIP);
  const sps::StreamArgs sa = stream_args(s, nullptr, d_cands, d_ncand);
  if (sps::launch_stream_close(sa, stream) != hipSuccess) return fail(SPS_ERR_HIP);
  if (stream_finish(s, stream) != SPS_OK) return fail(SPS_ERR_HIP);
  if (end_offset) *end_offset = s->pushed;
  return ok();
}

int sps_stream_state_size(const sps_stream* s, uint64_t* bytes) {
  if (!s || !bytes) return fail(SPS_ERR_INVALID_ARG);
  *bytes = stream_state_bytes(s);
  return ok();
}

int sps_stream_save(sps_stream* s, hipStream_t stream, void* host_buf, uint64_t bytes) {
  if (!s || !host_buf || bytes < stream_state_bytes(s)) return fail(SPS_ERR_INVALID_ARG);
  if (hipStreamSynchronize(stream) != hipSuccess) return fail(SPS_ERR_HIP);
  const sps_plan* p = s->plan;
  StreamHeader h;
  std::memset(&h, 0, sizeof(h));
  h.magic = kStreamMagic;
  h.pushed = s->pushed;
  h.ndm = p->ndm; h.nsamp = p->nsamp; h.Hx = s->Hx; h.nw = p->nw;
  h.max_width = p->max_width; h.baseline_len = p->baseline_len;
  if (hipMemcpy(&h.tmin, s->tmin, sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess) return fail(SPS_ERR_HIP);
  char* o = static_cast<char*>(host_buf);
  std::memcpy(o, &h, sizeof(h));
  o += sizeof(h);
  const size_t hb = (size_t)p->ndm * s->Hx * sizeof(float);
  if (hipMemcpy(o, s->hist[s->cur], hb, hipMemcpyDeviceToHost) != hipSuccess) return fail(SPS_ERR_HIP);
  o += hb;
  const size_t mb = (size_t)s->Hb * sizeof(int32_t);
  if (hipMemcpy2D(o, mb, s->med[s->cur], (size_t)s->nbv * sizeof(int32_t), mb, p->ndm, hipMemcpyDeviceToHost) !=
      hipSuccess) return fail(SPS_ERR_HIP);
  o += mb * p->ndm;
  if (hipMemcpy2D(o, mb, s->mad[s->cur], (size_t)s->nbv * sizeof(int32_t), mb, p->ndm, hipMemcpyDeviceToHost) !=
      hipSuccess) return fail(SPS_ERR_HIP);
  o += mb * p->ndm;
  if (hipMemcpy(o, s->carry, (size_t)p->ndm * p->nw * sizeof(sps::RunSum), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(SPS_ERR_HIP);
  return ok();
}

int sps_stream_restore(sps_stream* s, hipStream_t stream, const void* host_buf, uint64_t bytes) {
  if (!s || !host_buf || bytes < stream_state_bytes(s)) return fail(SPS_ERR_INVALID_ARG);
  const sps_plan* p = s->plan;
  StreamHeader h;
  std::memcpy(&h, host_buf, sizeof(h));
  if (h.magic != kStreamMagic || h.ndm != p->ndm || h.nsamp != p->nsamp || h.Hx != s->Hx || h.nw != p->nw ||
      h.max_width != p->max_width || h.baseline_len != p->baseline_len || h.tmin < 0 || h.tmin > s->Hx)
    return fail(SPS_ERR_INVALID_ARG);
  if (hipStreamSynchronize(stream) != hipSuccess) return fail(SPS_ERR_HIP);
  const char* o = static_cast<const char*>(host_buf) + sizeof(h);
  const size_t hb = (size_t)p->ndm * s->Hx * sizeof(float);
  if (hipMemcpy(s->hist[s->cur], o, hb, hipMemcpyHostToDevice) != hipSuccess) return fail(SPS_ERR_HIP);
  o += hb;
  const size_t mb = (size_t)s->Hb * sizeof(int32_t);
  if (hipMemcpy2D(s->med[s->cur], (size_t)s->nbv * sizeof(int32_t), o, mb, mb, p->ndm, hipMemcpyHostToDevice) !=
      hipSuccess) return fail(SPS_ERR_HIP);
  o += mb * p->ndm;
  if (hipMemcpy2D(s->mad[s->cur], (size_t)s->nbv * sizeof(int32_t), o, mb, mb, p->ndm, hipMemcpyHostToDevice) !=
      hipSuccess) return fail(SPS_ERR_HIP);
  o += mb * p->ndm;
  if (hipMemcpy(s->carry, o, (size_t)p->ndm * p->nw * sizeof(sps::RunSum), hipMemcpyHostToDevice) != hipSuccess)
    return fail(SPS_ERR_HIP);
  if (hipMemcpy(s->tmin, &h.tmin, sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess) return fail(SPS_ERR_HIP);
  s->pushed = h.pushed;
  return ok();
}

}  // extern "C"

extern "C" {

int64_t sps_domain_bound(int32_t max_width) { return domain_bound(max_width); }

int sps_footprint(int32_t ndm, int64_t nsamp, int32_t max_width, int32_t baseline_len, int streaming,
                  uint64_t* bytes) {
  if (!bytes || ndm < 1 || nsamp < 1 || nsamp > (int64_t)INT32_MAX - 8192 || !is_pow2(max_width) ||
      max_width > SPS_MAX_WIDTH_LIMIT || baseline_len < 1 || baseline_len > SPS_MAX_BASELINE_LEN ||
      (streaming && nsamp % sps::kStride != 0))
    return fail(SPS_ERR_INVALID_ARG);
  sps_plan p;
  plan_params(&p, ndm, nsamp, max_width, baseline_len, 1.0f);
  uint64_t total = 2ull * ndm * p.nblocks * sizeof(int32_t) + (uint64_t)frag_need(&p) * sizeof(sps::RunSum);
  if (streaming) {
    sps_stream s;
    std::memset(&s, 0, sizeof(s));
    s.plan = &p;
    if (!stream_geometry(&p, &s)) return fail(SPS_ERR_INVALID_ARG);
    total += stream_device_bytes(&s);
  }
  *bytes = total;
  return ok();
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batch of independent blocks: one persistent launch per stage.

struct sps_batch {
  int device;
  int32_t stats_seg, detect_seg, hist_bins;
  int32_t window;      // SPS_ATTR_WINDOW for every item
  int32_t norm;        // SPS_ATTR_NORM for every item
  int32_t fused;       // SPS_ATTR_FUSED: statistics and detection in one persistent launch
  int32_t* d_ms;       // medians then MADs of every item (then per-width c_w and MAD_w with SPS_ATTR_NORM = 2)
  int64_t ms_cap;      // int32 records
  sps::RunSum* d_frag;
  int64_t frag_cap;
  char* d_tab;         // item descriptors, task offsets, counter pointers, queue heads
  char* h_tab;         // pinned staging of d_tab
  size_t tab_cap;
  hipEvent_t uploaded; // h_tab may be rewritten once this has completed
  hipEvent_t done;     // end of the last call's work
  bool pending;        // both events recorded at least once
  int grid_stats[2];   // resident workgroups: 4096 / 16384 bins (0 = not queried)
  int grid_detect[2];  // 13 widths / any
  int grid_search[2];  // fused kernel: 13 widths / any
};

namespace {

struct BatchShape {
  int idx;
  int32_t nblocks, nw;
  int32_t stats_seg, stats_nseg, stats_head;
  int32_t detect_seg, detect_nseg;
  int64_t ms_off, frag_off, ws_off;
};

bool item_valid(const sps_batch_item& it) {
  return it.d_series && it.d_ncand && it.ndm >= 1 && it.nsamp >= 1 && it.nsamp <= (int64_t)INT32_MAX - 8192 &&
         is_pow2(it.max_width) && it.max_width <= SPS_MAX_WIDTH_LIMIT && it.baseline_len >= 1 &&
         it.baseline_len <= SPS_MAX_BASELINE_LEN && std::isfinite(it.snr_thresh) && it.snr_thresh > 0.0f &&
         it.max_cands >= 0 && it.max_cands <= (int64_t)UINT32_MAX && (it.d_cands || it.max_cands == 0);
}

size_t align16(size_t v) { return (v + 15) & ~(size_t)15; }

// Row scales of a batch (SPS_ATTR_NORM = 1): one launch per item.
hipError_t launch_row_mads(const std::vector<sps::RowMadArgs>& v, hipStream_t s) {
  for (const sps::RowMadArgs& r : v) {
    const hipError_t e = sps::launch_row_mad(r, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Per-width scales of a batch (SPS_ATTR_NORM = 2): one launch per item.
hipError_t launch_width_stats_all(const std::vector<sps::WidthStatsArgs>& v, hipStream_t s) {
  for (const sps::WidthStatsArgs& w : v) {
    const hipError_t e = sps::launch_width_stats(w, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <class T>
int grow(T** p, int64_t* cap, int64_t need) {
  if (need <= *cap) return SPS_OK;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  *cap = 0;
  if (hipMalloc(reinterpret_cast<void**>(p), (size_t)need * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return SPS_ERR_OOM;
  }
  *cap = need;
  return SPS_OK;
}

// Workspace of a batch call: grows the scratch and the item tables (waiting
// for the context's earlier work first), queries the resident grids, orders
// `stream` after the previous call and waits until the pinned staging of the
// tables may be rewritten.
int batch_prepare(sps_batch* b, size_t tab_bytes, int64_t ms_need, int64_t frag_need, bool all13,
                  hipStream_t stream) {
  if (ms_need > b->ms_cap || frag_need > b->frag_cap || tab_bytes > b->tab_cap) {
    if (b->pending && hipEventSynchronize(b->done) != hipSuccess) return SPS_ERR_HIP;
    if (ms_need > 0 && grow(&b->d_ms, &b->ms_cap, ms_need) != SPS_OK) return SPS_ERR_OOM;
    if (frag_need > 0 && grow(&b->d_frag, &b->frag_cap, frag_need) != SPS_OK) return SPS_ERR_OOM;
    if (tab_bytes > b->tab_cap) {
      if (b->d_tab) (void)hipFree(b->d_tab);
      if (b->h_tab) (void)hipHostFree(b->h_tab);
      b->d_tab = nullptr;
      b->h_tab = nullptr;
      b->tab_cap = 0;
      const size_t cap = std::max<size_t>(tab_bytes, 64 * 1024);
      if (hipMalloc(reinterpret_cast<void**>(&b->d_tab), cap) != hipSuccess ||
          hipHostMalloc(reinterpret_cast<void**>(&b->h_tab), cap, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return SPS_ERR_OOM;
      }
      b->tab_cap = cap;
    }
  }
  const int bins = b->hist_bins == 16384 ? 1 : 0;
  if (!b->grid_stats[bins]) b->grid_stats[bins] = sps::block_stats_batch_grid(b->hist_bins);
  if (!b->grid_detect[all13 ? 0 : 1]) b->grid_detect[all13 ? 0 : 1] = sps::detect_batch_grid(all13 ? 13 : 0);
  if (b->grid_stats[bins] <= 0 || b->grid_detect[all13 ? 0 : 1] <= 0) return SPS_ERR_HIP;
  // order after the previous call (possibly on another stream), and wait
  // until the staging buffer is free again
  if (b->pending) {
    if (hipStreamWaitEvent(stream, b->done, 0) != hipSuccess) return SPS_ERR_HIP;
    if (hipEventSynchronize(b->uploaded) != hipSuccess) return SPS_ERR_HIP;
  }
  return SPS_OK;
}

}  // namespace

extern "C" {

int sps_batch_create(sps_batch** out) {
  if (!out) return fail(SPS_ERR_INVALID_ARG);
  *out = nullptr;
  sps_batch* b = new (std::nothrow) sps_batch;
  if (!b) return fail(SPS_ERR_OOM);
  std::memset(b, 0, sizeof(*b));
  b->hist_bins = 4096;
  b->fused = 1;
  if (hipGetDevice(&b->device) != hipSuccess ||
      hipEventCreateWithFlags(&b->uploaded, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->done, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    if (b->uploaded) (void)hipEventDestroy(b->uploaded);
    delete b;
    return fail(SPS_ERR_HIP);
  }
  *out = b;
  return ok();
}

int sps_batch_set(sps_batch* b, int attr, int64_t v) {
  if (!b) return fail(SPS_ERR_INVALID_ARG);
  switch (attr) {
    case SPS_ATTR_STATS_SEG:
      if (v < 0 || v > INT32_MAX) return fail(SPS_ERR_INVALID_ARG);
      b->stats_seg = (int32_t)v;
      return ok();
    case SPS_ATTR_DETECT_SEG:
      if (v < 0 || v > INT32_MAX || v % kDetectStep) return fail(SPS_ERR_INVALID_ARG);
      b->detect_seg = (int32_t)v;
      return ok();
    case SPS_ATTR_HIST_BINS:
      if (v != 4096 && v != 16384) return fail(SPS_ERR_INVALID_ARG);
      b->hist_bins = (int32_t)v;
      return ok();
    case SPS_ATTR_WINDOW:
      if (v != 0 && v != 1) return fail(SPS_ERR_INVALID_ARG);
      b->window = (int32_t)v;
      return ok();
    case SPS_ATTR_NORM:
      if (v < 0 || v > 2) return fail(SPS_ERR_INVALID_ARG);
      b->norm = (int32_t)v;
      return ok();
    case SPS_ATTR_FUSED:
      if (v != 0 && v != 1) return fail(SPS_ERR_INVALID_ARG);
      b->fused = (int32_t)v;
      return ok();
    default:
      return fail(SPS_ERR_INVALID_ARG);
  }
}

void sps_batch_destroy(sps_batch* b) {
  if (!b) return;
  if (b->pending) (void)hipEventSynchronize(b->done);
  if (b->d_ms) (void)hipFree(b->d_ms);
  if (b->d_frag) (void)hipFree(b->d_frag);
  if (b->d_tab) (void)hipFree(b->d_tab);
  if (b->h_tab) (void)hipHostFree(b->h_tab);
  (void)hipEventDestroy(b->uploaded);
  (void)hipEventDestroy(b->done);
  delete b;
}

int sps_batch_search(sps_batch* b, const sps_batch_item* items, int32_t n, hipStream_t stream) {
  if (!b || n < 0 || (n > 0 && !items)) return fail(SPS_ERR_INVALID_ARG);
  if (n == 0) return ok();
  for (int32_t i = 0; i < n; ++i)
    if (!item_valid(items[i]) || !window_fits(items[i].nsamp, items[i].baseline_len, b->window))
      return fail(SPS_ERR_INVALID_ARG);

  // Shapes. Chain and segment lengths follow the single-block rules, sized
  // for the whole batch so that the queue holds many more tasks than there
  // are resident workgroups.
  std::vector<BatchShape> sh((size_t)n);
  int64_t total_blocks = 0, total_samples = 0;
  for (int32_t i = 0; i < n; ++i) {
    total_blocks += (int64_t)items[i].ndm * ((items[i].nsamp + sps::kStride - 1) / sps::kStride);
    total_samples += (int64_t)items[i].ndm * items[i].nsamp;
  }
  int64_t ms_need = 0, frag_need = 0, fix_total = 0;
  bool all13 = true;
  for (int32_t i = 0; i < n; ++i) {
    const sps_batch_item& it = items[i];
    BatchShape& s = sh[(size_t)i];
    s.idx = i;
    s.nblocks = (int32_t)((it.nsamp + sps::kStride - 1) / sps::kStride);
    s.nw = 0;
    for (int w = 1; w <= it.max_width; w <<= 1) ++s.nw;
    all13 = all13 && s.nw == sps::kMaxWidths;
    int64_t seg;
    if (b->stats_seg > 0) {
      seg = b->stats_seg;
    } else {
      seg = (total_blocks + 4095) / 4096;
      seg = std::max<int64_t>(seg, std::max<int64_t>(64, (4LL * it.baseline_len + 63) / 64));
    }
    seg = std::max<int64_t>(1, std::min<int64_t>(seg, s.nblocks));
    s.stats_seg = (int32_t)seg;
    s.stats_nseg = (int32_t)((s.nblocks + seg - 1) / seg);
    s.stats_head = s.stats_seg;
    if (b->stats_seg == 0)
      shorten_first_segment(s.nblocks, std::min<int64_t>(it.baseline_len, it.nsamp), s.stats_nseg, s.stats_seg,
                            s.stats_head);
    int64_t dseg = b->detect_seg > 0 ? b->detect_seg : std::max<int64_t>(total_samples / 8192, 4LL * it.max_width);
    dseg = (dseg + kDetectStep - 1) / kDetectStep * kDetectStep;
    const int64_t nmax = std::max<int64_t>(kDetectStep, (it.nsamp + kDetectStep - 1) / kDetectStep * kDetectStep);
    dseg = std::max<int64_t>(kDetectStep, std::min<int64_t>(dseg, nmax));
    s.detect_seg = (int32_t)dseg;
    s.detect_nseg = (int32_t)((it.nsamp + dseg - 1) / dseg);
    s.ms_off = ms_need;
    ms_need += 2LL * it.ndm * s.nblocks;
    s.ws_off = ms_need;
    if (b->norm == 2) ms_need += 2LL * it.ndm * s.nw;
    s.frag_off = frag_need;
    if (s.detect_nseg > 1) {
      frag_need += (int64_t)it.ndm * s.nw * s.detect_nseg;
      fix_total += (int64_t)it.ndm * s.nw;
    }
  }
  // Fused launch (statistics chains then detection in one persistent kernel):
  // per row of every item a count of its finished chains, after the medians.
  const bool fused = b->fused == 1 && b->norm == 0 && b->hist_bins == 4096;
  int64_t total_rows = 0;
  for (int32_t i = 0; i < n; ++i) total_rows += items[i].ndm;
  const int64_t done_off = ms_need;
  if (fused) ms_need += total_rows;
  // task counts must fit the int32 queue
  int64_t stats_total = 0, detect_total = 0;
  for (const BatchShape& s : sh) {
    stats_total += (int64_t)items[s.idx].ndm * s.stats_nseg;
    detect_total += (int64_t)items[s.idx].ndm * s.detect_nseg;
  }
  if (stats_total > INT32_MAX / 2 || detect_total > INT32_MAX / 2 || fix_total > INT32_MAX / 2)
    return fail(SPS_ERR_INVALID_ARG);

  // Table layout.
  const size_t off_sa = 0;
  const size_t off_da = align16(off_sa + (size_t)n * sizeof(sps::StatsArgs));
  const size_t off_so = align16(off_da + (size_t)n * sizeof(sps::DetectArgs));
  const size_t off_do = align16(off_so + (size_t)(n + 1) * sizeof(int32_t));
  const size_t off_fo = align16(off_do + (size_t)(n + 1) * sizeof(int32_t));
  const size_t off_np = align16(off_fo + (size_t)(n + 1) * sizeof(int32_t));
  const size_t off_ct = align16(off_np + (size_t)n * sizeof(uint32_t*));
  const size_t tab_bytes = align16(off_ct + 2 * sizeof(uint32_t));

  {
    const int rc = batch_prepare(b, tab_bytes, ms_need, frag_need, all13, stream);
    if (rc != SPS_OK) return fail(rc);
  }
  const int bins = b->hist_bins == 16384 ? 1 : 0;

  char* h = b->h_tab;
  char* d = b->d_tab;
  auto* sa = reinterpret_cast<sps::StatsArgs*>(h + off_sa);
  auto* da = reinterpret_cast<sps::DetectArgs*>(h + off_da);
  auto* so = reinterpret_cast<int32_t*>(h + off_so);
  auto* dof = reinterpret_cast<int32_t*>(h + off_do);
  auto* fo = reinterpret_cast<int32_t*>(h + off_fo);
  auto* np = reinterpret_cast<uint32_t**>(h + off_np);

  std::vector<int64_t> row0((size_t)n);
  {
    int64_t r = 0;
    for (int32_t i = 0; i < n; ++i) {
      row0[(size_t)i] = r;
      r += items[i].ndm;
    }
  }
  // Stats queue: longest chains (warm-up window + segment) first.
  std::vector<BatchShape> ord = sh;
  std::stable_sort(ord.begin(), ord.end(), [&](const BatchShape& x, const BatchShape& y) {
    const int64_t cx = x.stats_seg + std::min<int64_t>(items[x.idx].baseline_len, items[x.idx].nsamp) / 64;
    const int64_t cy = y.stats_seg + std::min<int64_t>(items[y.idx].baseline_len, items[y.idx].nsamp) / 64;
    return cx > cy;
  });
  int32_t acc = 0;
  std::vector<sps::RowMadArgs> row_mads;
  std::vector<sps::WidthStatsArgs> width_stats;
  for (int32_t k = 0; k < n; ++k) {
    const BatchShape& s = ord[(size_t)k];
    const sps_batch_item& it = items[s.idx];
    sps::StatsArgs& a = sa[k];
    std::memset(&a, 0, sizeof(a));
    a.x = it.d_series;
    a.ld = it.nsamp;
    a.N = (int32_t)it.nsamp;
    a.L = it.baseline_len;
    a.lead = window_lead(it.baseline_len, b->window);
    a.nblocks = s.nblocks;
    a.kb_first = 0;
    a.seg_blocks = s.stats_seg;
    a.head_blocks = s.stats_head;
    a.nseg = s.stats_nseg;
    a.nchains = it.ndm * s.stats_nseg;
    a.tmin = nullptr;
    a.med = b->d_ms + s.ms_off;
    a.mad = b->d_ms + s.ms_off + (int64_t)it.ndm * s.nblocks;
    a.done = fused ? reinterpret_cast<uint32_t*>(b->d_ms + done_off + row0[(size_t)s.idx]) : nullptr;
    if (b->norm == 1) row_mads.push_back(sps::RowMadArgs{a.x, a.ld, a.N, a.nblocks, a.nblocks, it.ndm, a.med, a.mad});
    if (b->norm == 2)
      width_stats.push_back(sps::WidthStatsArgs{a.x, a.ld, a.N, a.nblocks, it.ndm, s.nw, a.med, b->d_ms + s.ws_off,
                                                b->d_ms + s.ws_off + (int64_t)it.ndm * s.nw});
    so[k] = acc;
    acc += a.nchains;
  }
  so[n] = acc;

  // Detect queue: longest segments (segment + widest halo) first; the fix-up
  // reads the same table.
  ord = sh;
  std::stable_sort(ord.begin(), ord.end(), [&](const BatchShape& x, const BatchShape& y) {
    const int64_t cx = std::min<int64_t>(x.detect_seg, items[x.idx].nsamp) + items[x.idx].max_width;
    const int64_t cy = std::min<int64_t>(y.detect_seg, items[y.idx].nsamp) + items[y.idx].max_width;
    return cx > cy;
  });
  acc = 0;
  int32_t facc = 0;
  for (int32_t k = 0; k < n; ++k) {
    const BatchShape& s = ord[(size_t)k];
    const sps_batch_item& it = items[s.idx];
    sps::DetectArgs& a = da[k];
    std::memset(&a, 0, sizeof(a));
    a.x = it.d_series;
    a.ld = it.nsamp;
    a.N = (int32_t)it.nsamp;
    a.nblocks = s.nblocks;
    a.nw = s.nw;
    a.maxw = it.max_width;
    a.med = b->d_ms + s.ms_off;
    a.mad = b->d_ms + s.ms_off + (int64_t)it.ndm * s.nblocks;
    a.wmad = b->norm == 2 ? b->d_ms + s.ws_off + (int64_t)it.ndm * s.nw : nullptr;
    a.theta = (double)it.snr_thresh;
    for (int j = 0; j < s.nw; ++j) a.sqrtw[j] = b->norm == 2 ? 1.0 : std::sqrt((double)(1 << j));
    a.seg_base = 0;
    a.seg_len = s.detect_seg;
    a.nseg = s.detect_nseg;
    a.rows = it.ndm;
    a.e_first = 0;
    a.tmin = nullptr;
    a.sample_offset = 0;
    a.keep_edges = 0;
    a.row_offset = 0;
    a.cands = it.d_cands;
    a.ncand = it.d_ncand;
    a.cap = (uint32_t)it.max_cands;
    a.frag = s.detect_nseg > 1 ? b->d_frag + s.frag_off : nullptr;
    a.done = fused ? reinterpret_cast<const uint32_t*>(b->d_ms + done_off + row0[(size_t)s.idx]) : nullptr;
    a.done_target = (uint32_t)s.stats_nseg;
    dof[k] = acc;
    acc += it.ndm * s.detect_nseg;
    fo[k] = facc;
    if (s.detect_nseg > 1) facc += it.ndm * s.nw;
  }
  dof[n] = acc;
  fo[n] = facc;
  for (int32_t i = 0; i < n; ++i) np[i] = items[i].d_ncand;

  if (hipMemcpyAsync(d, h, tab_bytes, hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipEventRecord(b->uploaded, stream) != hipSuccess) return fail(SPS_ERR_HIP);

  uint32_t* counters = reinterpret_cast<uint32_t*>(d + off_ct);
  sps::BatchStats bs{reinterpret_cast<const sps::StatsArgs*>(d + off_sa), reinterpret_cast<const int32_t*>(d + off_so),
                     n, so[n], counters};
  sps::BatchDetect bd{reinterpret_cast<const sps::DetectArgs*>(d + off_da),
                      reinterpret_cast<const int32_t*>(d + off_do), n, dof[n], counters + 1};
  const int wpg = b->hist_bins == 16384 ? 2 : 4;
  const int gs = (int)std::min<int64_t>(b->grid_stats[bins], (bs.total + wpg - 1) / wpg);
  const int gd = (int)std::min<int64_t>(b->grid_detect[all13 ? 0 : 1], bd.total);
  bool okl = sps::launch_batch_zero(reinterpret_cast<uint32_t* const*>(d + off_np), n, counters, stream) == hipSuccess;
  if (fused) {
    const int k13 = all13 ? 0 : 1;
    if (!b->grid_search[k13]) b->grid_search[k13] = sps::search_batch_grid(all13 ? 13 : 0);
    const int gf = (int)std::min<int64_t>(b->grid_search[k13], std::max<int64_t>((bs.total + 3) / 4, bd.total));
    okl = okl && b->grid_search[k13] > 0 &&
          sps::launch_zero_u32(reinterpret_cast<uint32_t*>(b->d_ms + done_off), (int)total_rows, stream) == hipSuccess &&
          sps::launch_search_batch(bs, bd, all13 ? 13 : 0, b->window == 1, gf, stream) == hipSuccess;
  } else {
    okl = okl && sps::launch_block_stats_batch(bs, b->hist_bins, b->window == 1, false, gs, stream) == hipSuccess &&
          launch_row_mads(row_mads, stream) == hipSuccess && launch_width_stats_all(width_stats, stream) == hipSuccess &&
          sps::launch_detect_batch(bd, all13 ? 13 : 0, false, gd, stream) == hipSuccess;
  }
  okl = okl && sps::launch_fixup_batch(bd, reinterpret_cast<const int32_t*>(d + off_fo), fo[n], stream) == hipSuccess &&
        hipEventRecord(b->done, stream) == hipSuccess;
  if (!okl) {
    (void)hipGetLastError();
    b->pending = true;
    return fail(SPS_ERR_HIP);
  }
  b->pending = true;
  return ok();
}

int sps_batch_push(sps_batch* b, sps_stream* const* streams, const float* const* d_gulps, int32_t n,
                   hipStream_t stream, sps_cand* const* d_cands, uint32_t* const* d_ncand, int64_t* gulp_offsets) {
  if (!b || n < 0 || (n > 0 && (!streams || !d_gulps || !d_cands || !d_ncand))) return fail(SPS_ERR_INVALID_ARG);
  if (n == 0) return ok();
  bool all13 = true;
  for (int32_t i = 0; i < n; ++i) {
    const sps_stream* s = streams[i];
    if (!s || !d_gulps[i] || !d_ncand[i] || (!d_cands[i] && s->plan->max_cands > 0)) return fail(SPS_ERR_INVALID_ARG);
    if (!stream_plan_ok(s->plan)) return fail(SPS_ERR_INVALID_ARG);
    for (int32_t k = 0; k < i; ++k)
      if (streams[k] == s) return fail(SPS_ERR_INVALID_ARG);  // one gulp per stream: the next needs this one's carry
    all13 = all13 && s->plan->nw == sps::kMaxWidths;
  }
  for (int32_t i = 0; i < n; ++i) {
    const int rc = check_domain(streams[i]->plan, d_gulps[i], (int64_t)streams[i]->plan->ndm * streams[i]->plan->nsamp,
                                stream);
    if (rc != SPS_OK) return fail(rc);
  }
  // Tables: statistics and detection arguments of every gulp, task offsets,
  // counter pointers, queue heads.
  const size_t off_sa = 0;
  const size_t off_da = align16(off_sa + (size_t)n * sizeof(sps::StatsArgs));
  const size_t off_so = align16(off_da + (size_t)n * sizeof(sps::DetectArgs));
  const size_t off_do = align16(off_so + (size_t)(n + 1) * sizeof(int32_t));
  const size_t off_np = align16(off_do + (size_t)(n + 1) * sizeof(int32_t));
  const size_t off_ct = align16(off_np + (size_t)n * sizeof(uint32_t*));
  const size_t tab_bytes = align16(off_ct + 2 * sizeof(uint32_t));
  {
    const int rc = batch_prepare(b, tab_bytes, 0, 0, all13, stream);
    if (rc != SPS_OK) return fail(rc);
  }
  const int bins = b->hist_bins == 16384 ? 1 : 0;
  char* h = b->h_tab;
  char* d = b->d_tab;
  auto* sa = reinterpret_cast<sps::StatsArgs*>(h + off_sa);
  auto* da = reinterpret_cast<sps::DetectArgs*>(h + off_da);
  auto* so = reinterpret_cast<int32_t*>(h + off_so);
  auto* dof = reinterpret_cast<int32_t*>(h + off_do);
  auto* np = reinterpret_cast<uint32_t**>(h + off_np);
  // queues ordered by task cost, largest first (chains: window + segment;
  // detection segments: segment + widest halo)
  std::vector<int32_t> ord((size_t)n);
  for (int32_t i = 0; i < n; ++i) ord[(size_t)i] = i;
  std::vector<sps::StatsArgs> st((size_t)n);
  std::vector<sps::DetectArgs> dt((size_t)n);
  for (int32_t i = 0; i < n; ++i) {
    st[(size_t)i] = stream_stats_args(streams[i], d_gulps[i], streams[i]->cur);
    dt[(size_t)i] = stream_detect_args(streams[i], d_gulps[i], d_cands[i], d_ncand[i], streams[i]->cur);
  }
  std::stable_sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) {
    return st[(size_t)x].seg_blocks + st[(size_t)x].L / 64 > st[(size_t)y].seg_blocks + st[(size_t)y].L / 64;
  });
  int32_t acc = 0;
  for (int32_t k = 0; k < n; ++k) {
    sa[k] = st[(size_t)ord[(size_t)k]];
    so[k] = acc;
    acc += sa[k].nchains;
  }
  so[n] = acc;
  std::stable_sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) {
    return dt[(size_t)x].seg_len + dt[(size_t)x].maxw > dt[(size_t)y].seg_len + dt[(size_t)y].maxw;
  });
  acc = 0;
  for (int32_t k = 0; k < n; ++k) {
    da[k] = dt[(size_t)ord[(size_t)k]];
    dof[k] = acc;
    acc += da[k].rows * da[k].nseg;
  }
  dof[n] = acc;
  for (int32_t i = 0; i < n; ++i) np[i] = d_ncand[i];
  if (hipMemcpyAsync(d, h, tab_bytes, hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipEventRecord(b->uploaded, stream) != hipSuccess) return fail(SPS_ERR_HIP);
  uint32_t* counters = reinterpret_cast<uint32_t*>(d + off_ct);
  sps::BatchStats bs{reinterpret_cast<const sps::StatsArgs*>(d + off_sa), reinterpret_cast<const int32_t*>(d + off_so),
                     n, so[n], counters};
  sps::BatchDetect bd{reinterpret_cast<const sps::DetectArgs*>(d + off_da),
                      reinterpret_cast<const int32_t*>(d + off_do), n, dof[n], counters + 1};
  const int wpg = b->hist_bins == 16384 ? 2 : 4;
  const int gs = (int)std::min<int64_t>(b->grid_stats[bins], (bs.total + wpg - 1) / wpg);
  const int gd = (int)std::min<int64_t>(b->grid_detect[all13 ? 0 : 1], bd.total);
  bool okl = sps::launch_batch_zero(reinterpret_cast<uint32_t* const*>(d + off_np), n, counters, stream) == hipSuccess &&
             sps::launch_block_stats_batch(bs, b->hist_bins, false, true, gs, stream) == hipSuccess;
  // streams with one row scale per gulp: the gulp's row MAD before detection
  for (int32_t i = 0; okl && i < n; ++i)
    if (streams[i]->plan->norm == 1)
      okl = sps::launch_row_mad(stream_row_mad_args(streams[i], d_gulps[i], streams[i]->cur), stream) == hipSuccess;
  okl = okl && sps::launch_detect_batch(bd, all13 ? 13 : 0, true, gd, stream) == hipSuccess;
  // each stream folds its open runs and rolls its history forward
  for (int32_t i = 0; okl && i < n; ++i) {
    const sps::StreamArgs fa = stream_args(streams[i], d_gulps[i], d_cands[i], d_ncand[i]);
    okl = sps::launch_stream_fold(fa, stream) == hipSuccess && sps::launch_stream_advance(fa, stream) == hipSuccess &&
          stream_finish(streams[i], stream) == SPS_OK;
  }
  okl = okl && hipEventRecord(b->done, stream) == hipSuccess;
  b->pending = true;
  if (!okl) {
    (void)hipGetLastError();
    return fail(SPS_ERR_HIP);
  }
  for (int32_t i = 0; i < n; ++i) {
    sps_stream* s = streams[i];
    if (gulp_offsets) gulp_offsets[i] = s->pushed;
    s->pushed += s->plan->nsamp;
    s->cur ^= 1;
  }
  return ok();
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Candidate clustering context: one device allocation carved into the
// scratch arrays of ClusterScratch.

struct sps_clusterer {
  uint32_t cap;
  void* mem;
  sps::ClusterScratch s;
  hipEvent_t done;  // end of the last run's work (destroy waits for it)
  bool pending;
};

extern "C" {

sps_clusterer* sps_cluster_create(uint32_t max_cands) {
  if (max_cands == 0) {
    fail(SPS_ERR_INVALID_ARG);
    return nullptr;
  }
  const size_t n = max_cands;
  const size_t cells = (size_t)sps::kClusterCells + 2;
  const size_t tiles = (size_t)sps::kClusterCells / 1024 + 1;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = (off + bytes + 255) & ~(size_t)255;
    return at;
  };
  const size_t o_sorted = take(16 * n), o_parent = take(4 * n), o_members = take(4 * n), o_snr = take(4 * n);
  const size_t o_slo = take(4 * n), o_shi = take(4 * n), o_dlo = take(4 * n), o_dhi = take(4 * n);
  const size_t o_tie = take(8 * n), o_count = take(4 * cells), o_cursor = take(4 * cells);
  const size_t o_bsum = take(4 * tiles), o_geo = take(32);
  sps_clusterer* k = new (std::nothrow) sps_clusterer;
  if (!k) {
    fail(SPS_ERR_OOM);
    return nullptr;
  }
  k->cap = max_cands;
  k->mem = nullptr;
  k->pending = false;
  if (hipEventCreateWithFlags(&k->done, hipEventDisableTiming) != hipSuccess) {
    delete k;
    fail(SPS_ERR_HIP);
    return nullptr;
  }
  if (hipMalloc(&k->mem, off) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipEventDestroy(k->done);
    delete k;
    fail(SPS_ERR_OOM);
    return nullptr;
  }
  char* b = static_cast<char*>(k->mem);
  k->s.sorted = reinterpret_cast<sps_cand*>(b + o_sorted);
  k->s.parent = reinterpret_cast<int32_t*>(b + o_parent);
  k->s.members = reinterpret_cast<uint32_t*>(b + o_members);
  k->s.snrbits = reinterpret_cast<uint32_t*>(b + o_snr);
  k->s.slo = reinterpret_cast<int32_t*>(b + o_slo);
  k->s.shi = reinterpret_cast<int32_t*>(b + o_shi);
  k->s.dlo = reinterpret_cast<uint32_t*>(b + o_dlo);
  k->s.dhi = reinterpret_cast<uint32_t*>(b + o_dhi);
  k->s.tie = reinterpret_cast<unsigned long long*>(b + o_tie);
  k->s.count = reinterpret_cast<uint32_t*>(b + o_count);
  k->s.cursor = reinterpret_cast<uint32_t*>(b + o_cursor);
  k->s.bsum = reinterpret_cast<uint32_t*>(b + o_bsum);
  k->s.geo = reinterpret_cast<int32_t*>(b + o_geo);
  ok();
  return k;
}

int sps_cluster_run(sps_clusterer* k, const sps_cand* d_cands, uint32_t n, int32_t time_tol, int32_t dm_tol,
                    int32_t width_tol, hipStream_t stream, sps_cluster_rec* d_out, uint32_t* d_nout) {
  if (!k || !d_nout || (n > 0 && (!d_cands || !d_out)) || n > k->cap || time_tol < 0 || dm_tol < 0 || width_tol < 0)
    return fail(SPS_ERR_INVALID_ARG);
  if (sps::launch_cluster(d_cands, n, time_tol, dm_tol, width_tol, k->s, d_out, d_nout, stream) != hipSuccess)
    return fail(SPS_ERR_HIP);
  if (hipEventRecord(k->done, stream) != hipSuccess) return fail(SPS_ERR_HIP);
  k->pending = true;
  return ok();
}

void sps_cluster_destroy(sps_clusterer* k) {
  if (!k) return;
  if (k->pending) (void)hipEventSynchronize(k->done);
  (void)hipEventDestroy(k->done);
  if (k->mem) (void)hipFree(k->mem);
  delete k;
}

}  // extern "C"

// ---------------------------------------------------------------- dedispersion

struct sps_dedisp {
  int32_t nchan, ndm, ndm_pad, dd, ngroups;
  int64_t nsamp_in, nsamp_out;
  void* d_mem;               // one allocation: span table, then offsets
  sps::DedispSpan* d_span;   // [nchan][ngroups]
  int32_t* d_base;           // [nchan][ndm_pad]
  hipEvent_t done;           // end of the last run's work (destroy waits for it)
  bool pending;
};

namespace {

constexpr double kDispersionConst = 4.148808e3;  // MHz^2 pc^-1 cm^3 s

// Largest spread of the delays of `dd` consecutive trials in any channel.
int64_t delay_spread(const std::vector<int32_t>& dt, int32_t nchan, int32_t ndm_pad, int32_t dd) {
  int64_t spread = 0;
  for (int32_t f = 0; f < nchan; ++f)
    for (int32_t g = 0; g < ndm_pad; g += dd) {
      const int32_t* p = &dt[(size_t)f * ndm_pad + g];
      int32_t lo = p[0], hi = p[0];
      for (int32_t j = 1; j < dd; ++j) {
        lo = std::min(lo, p[j]);
        hi = std::max(hi, p[j]);
      }
      spread = std::max<int64_t>(spread, (int64_t)hi - lo);
    }
  return spread;
}

}  // namespace

extern "C" {

int sps_dedisp_delays(int32_t nchan, const double* freqs_mhz, double f_ref_mhz, double tsamp_s, int32_t ndm,
                      const float* dms, int32_t* delays) {
  if (nchan < 1 || ndm < 1 || !freqs_mhz || !dms || !delays || !(tsamp_s > 0.0) || !std::isfinite(tsamp_s) ||
      !(f_ref_mhz > 0.0) || !std::isfinite(f_ref_mhz))
    return fail(SPS_ERR_INVALID_ARG);
  for (int32_t f = 0; f < nchan; ++f)
    if (!(freqs_mhz[f] > 0.0) || !(freqs_mhz[f] <= f_ref_mhz)) return fail(SPS_ERR_INVALID_ARG);
  for (int32_t d = 0; d < ndm; ++d)
    if (!(dms[d] >= 0.0f) || !std::isfinite(dms[d])) return fail(SPS_ERR_INVALID_ARG);
  const double ref = 1.0 / (f_ref_mhz * f_ref_mhz);
  for (int32_t d = 0; d < ndm; ++d) {
    const double dm = (double)dms[d];
    for (int32_t f = 0; f < nchan; ++f) {
      const double v = kDispersionConst * dm * (1.0 / (freqs_mhz[f] * freqs_mhz[f]) - ref) / tsamp_s;
      const double r = std::floor(v + 0.5);
      if (!(r <= (double)INT32_MAX)) return fail(SPS_ERR_INVALID_ARG);
      delays[(size_t)d * nchan + f] = (int32_t)r;
    }
  }
  return ok();
}

static sps_dedisp* dedisp_create(int32_t nchan, int64_t nsamp_in, int32_t ndm, const int32_t* delays);

sps_dedisp* sps_dedisp_create(int32_t nchan, int64_t nsamp_in, int32_t ndm, const int32_t* delays) {
  // the host tables are std::vector: an allocation failure must not cross the C boundary
  try {
    return dedisp_create(nchan, nsamp_in, ndm, delays);
  } catch (const std::bad_alloc&) {
    fail(SPS_ERR_OOM);
    return nullptr;
  }
}

static sps_dedisp* dedisp_create(int32_t nchan, int64_t nsamp_in, int32_t ndm, const int32_t* delays) {
  if (nchan < 1 || nchan > 65536 || ndm < 1 || nsamp_in < 1 || nsamp_in > (int64_t)INT32_MAX - 8192 || !delays) {
    fail(SPS_ERR_INVALID_ARG);
    return nullptr;
  }
  int32_t maxd = 0;
  for (int64_t i = 0; i < (int64_t)ndm * nchan; ++i) {
    if (delays[i] < 0) {
      fail(SPS_ERR_INVALID_ARG);
      return nullptr;
    }
    maxd = std::max(maxd, delays[i]);
  }
  if ((int64_t)maxd >= nsamp_in) {
    fail(SPS_ERR_INVALID_ARG);
    return nullptr;
  }
  // trials per workgroup: the most whose delays fit the LDS staging in every channel
  const int64_t room = 4LL * (sps::kDedispSpanWords - 1) - 1030;
  int32_t dd = 16;
  std::vector<int32_t> dt;
  int32_t ndm_pad = 0;
  for (;; dd /= 2) {
    ndm_pad = (ndm + dd - 1) / dd * dd;
    dt.assign((size_t)nchan * ndm_pad, 0);
    for (int32_t f = 0; f < nchan; ++f)
      for (int32_t d = 0; d < ndm_pad; ++d)
        dt[(size_t)f * ndm_pad + d] = delays[(size_t)std::min(d, ndm - 1) * nchan + f];
    if (dd == 1 || delay_spread(dt, nchan, ndm_pad, dd) <= room) break;
  }
  // Per (channel, trial group): the staged span at time tile 0 (a tile
  // starts a multiple of 4 bytes later, so only the first word moves) and
  // each trial's byte offset into it.
  const int32_t ngroups = ndm_pad / dd;
  std::vector<sps::DedispSpan> span((size_t)nchan * ngroups);
  std::vector<int32_t> base((size_t)nchan * ndm_pad);
  for (int32_t f = 0; f < nchan; ++f)
    for (int32_t g = 0; g < ngroups; ++g) {
      const int32_t* p = &dt[(size_t)f * ndm_pad + (size_t)g * dd];
      int32_t lo = p[0], hi = p[0];
      for (int32_t j = 1; j < dd; ++j) {
        lo = std::min(lo, p[j]);
        hi = std::max(hi, p[j]);
      }
      const int64_t src0 = (int64_t)f * nsamp_in + lo;  // first byte needed at tile 0
      const int32_t sh0 = (int32_t)(src0 & 3);
      sps::DedispSpan& sg = span[(size_t)f * ngroups + g];
      sg.w0 = src0 >> 2;
      sg.nw = (sh0 + (hi - lo) + 1024 + 3) / 4 + 1;  // <= kDedispSpanWords by the choice of dd
      sg.pad = 0;
      for (int32_t j = 0; j < dd; ++j) base[(size_t)f * ndm_pad + (size_t)g * dd + j] = sh0 + (p[j] - lo);
    }
  sps_dedisp* k = new (std::nothrow) sps_dedisp;
  if (!k) {
    fail(SPS_ERR_OOM);
    return nullptr;
  }
  k->nchan = nchan;
  k->ndm = ndm;
  k->ndm_pad = ndm_pad;
  k->dd = dd;
  k->ngroups = ngroups;
  k->nsamp_in = nsamp_in;
  k->nsamp_out = nsamp_in - maxd;
  k->d_mem = nullptr;
  k->pending = false;
  if (hipEventCreateWithFlags(&k->done, hipEventDisableTiming) != hipSuccess) {
    delete k;
    fail(SPS_ERR_HIP);
    return nullptr;
  }
  const size_t span_bytes = span.size() * sizeof(sps::DedispSpan), base_bytes = base.size() * sizeof(int32_t);
  if (hipMalloc(&k->d_mem, span_bytes + base_bytes) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipEventDestroy(k->done);
    delete k;
    fail(SPS_ERR_OOM);
    return nullptr;
  }
  k->d_span = static_cast<sps::DedispSpan*>(k->d_mem);
  k->d_base = reinterpret_cast<int32_t*>(static_cast<char*>(k->d_mem) + span_bytes);
  if (hipMemcpy(k->d_span, span.data(), span_bytes, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(k->d_base, base.data(), base_bytes, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(k->d_mem);
    (void)hipEventDestroy(k->done);
    delete k;
    fail(SPS_ERR_HIP);
    return nullptr;
  }
  ok();
  return k;
}

int64_t sps_dedisp_nsamp_out(const sps_dedisp* k) {
  if (!k) {
    fail(SPS_ERR_INVALID_ARG);
    return -1;
  }
  return k->nsamp_out;
}

int sps_dedisp_run(sps_dedisp* k, const uint8_t* d_fil, hipStream_t stream, float* d_out) {
  if (!k || !d_fil || !d_out || (reinterpret_cast<uintptr_t>(d_fil) & 3u)) return fail(SPS_ERR_INVALID_ARG);
  sps::DedispArgs a;
  a.fil32 = reinterpret_cast<const uint32_t*>(d_fil);
  a.ld = k->nsamp_in;
  a.total_bytes = (int64_t)k->nchan * k->nsamp_in;
  a.nfull = a.total_bytes / 4;
  a.nchan = k->nchan;
  a.ndm = k->ndm;
  a.ndm_pad = k->ndm_pad;
  a.nsamp_out = (int32_t)k->nsamp_out;
  a.dd = k->dd;
  a.ngroups = k->ngroups;
  const int64_t ntime = (k->nsamp_out + 1023) / 1024;
  const int64_t ntiles = ntime * a.ngroups;
  if (ntiles > (int64_t)INT32_MAX - 8) return fail(SPS_ERR_INVALID_ARG);
  a.ntiles = (int32_t)ntiles;
  a.per_xcd = (int32_t)((ntiles + 7) / 8);
  a.span = k->d_span;
  a.base = k->d_base;
  a.out = d_out;
  if (sps::launch_dedisp(a, stream) != hipSuccess) return fail(SPS_ERR_HIP);
  if (hipEventRecord(k->done, stream) != hipSuccess) return fail(SPS_ERR_HIP);
  k->pending = true;
  return ok();
}

int sps_zero_dm(const uint8_t* d_in, int32_t nchan, int64_t nsamp, int32_t offset, hipStream_t stream,
                uint8_t* d_out) {
  if (!d_in || !d_out || nchan < 1 || nchan > 65536 || nsamp < 1 || nsamp > (int64_t)INT32_MAX - 8192 || offset < 0 ||
      offset > 255)
    return fail(SPS_ERR_INVALID_ARG);
  // the output either is the input or does not overlap it
  const uintptr_t i0 = reinterpret_cast<uintptr_t>(d_in), o0 = reinterpret_cast<uintptr_t>(d_out);
  const uintptr_t bytes = (uintptr_t)nchan * (uintptr_t)nsamp;
  if (i0 != o0 && i0 < o0 + bytes && o0 < i0 + bytes) return fail(SPS_ERR_INVALID_ARG);
  sps::ZeroDmArgs a;
  a.in = d_in;
  a.out = d_out;
  a.nsamp = nsamp;
  a.nchan = nchan;
  a.offset = offset;
  if (sps::launch_zero_dm(a, stream) != hipSuccess) return fail(SPS_ERR_HIP);
  return ok();
}

int sps_chan_mask(const uint8_t* d_in, int32_t nchan, int64_t nsamp, int32_t k, hipStream_t stream, uint8_t* d_out,
                  uint8_t* d_stats) {
  if (!d_in || !d_out || !d_stats || nchan < 1 || nchan > 65536 || nsamp < 1 || nsamp > (int64_t)INT32_MAX - 8192 ||
      k < 0)
    return fail(SPS_ERR_INVALID_ARG);
  const uintptr_t i0 = reinterpret_cast<uintptr_t>(d_in), o0 = reinterpret_cast<uintptr_t>(d_out);
  const uintptr_t s0 = reinterpret_cast<uintptr_t>(d_stats);
  const uintptr_t bytes = (uintptr_t)nchan * (uintptr_t)nsamp, sbytes = 3 * (uintptr_t)nchan;
  if (i0 != o0 && i0 < o0 + bytes && o0 < i0 + bytes) return fail(SPS_ERR_INVALID_ARG);
  if ((s0 < i0 + bytes && i0 < s0 + sbytes) || (s0 < o0 + bytes && o0 < s0 + sbytes)) return fail(SPS_ERR_INVALID_ARG);
  sps::ChanMaskArgs a;
  a.in = d_in;
  a.out = d_out;
  a.stats = d_stats;
  a.nsamp = nsamp;
  a.nchan = nchan;
  a.k = k;
  if (sps::launch_chan_mask(a, stream) != hipSuccess) return fail(SPS_ERR_HIP);
  return ok();
}

void sps_dedisp_destroy(sps_dedisp* k) {
  if (!k) return;
  if (k->pending) (void)hipEventSynchronize(k->done);
  (void)hipEventDestroy(k->done);
  if (k->d_mem) (void)hipFree(k->d_mem);
  delete k;
}

}  // extern "C"
