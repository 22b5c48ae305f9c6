"""CPU oracle for the per-DM-trial single-pulse search (test infrastructure).

TEST INFRASTRUCTURE ONLY. Only the test suite, the package smoke check and the
benchmark's CPU-baseline leg may import this module. The product path (the HIP
library and its Python binding) never imports, links or calls it, and it
shares no code, table or helper with that path. The only common dependency is
the seeded input generator in ``synth``, which holds none of this arithmetic.

What is computed (Heimdall++, Section II-B "Pipeline Stages in Heimdall" and
Algorithm 1, the per-DM-trial loop): for every dedispersed DM trial, baseline
removal, normalisation, matched filtering with a bank of boxcars, and peak
detection above an S/N threshold, producing candidates (time, DM trial,
filter width, peak S/N). The paper names the stages but gives no formulas, so
the readings below are this project's (each is listed with its reason in the
design notes):

1. ``x_t`` is the integer value of sample t (inputs are integer-valued).
2. Blocks ``k = 0 .. ceil(N/S)-1`` of ``S`` samples; block k ends at
   ``e_k = min(kS+S, N)``. Its baseline window is the trailing, start-clipped
   ``W_k = x[max(0, e_k - L) : e_k]`` with ``n_k = |W_k|``.
3. Baseline ("baseline removal"): ``m_k`` = element of 0-based rank
   ``floor((n_k-1)/2)`` of sorted ``W_k`` (the lower median).
4. Noise scale ("normalisation"): ``MAD_k`` = element of the same rank of
   sorted ``|W_k - m_k|``; ``sigma_k = K * MAD_k`` with
   ``K = 1 / Phi^{-1}(3/4)``.
5. Residual ``r_t = x_t - m_{floor(t/S)}``; matched filter
   ``S_w(i) = sum_{t=i}^{i+w-1} r_t`` for ``w`` in 1, 2, 4, ..., max_width and
   ``0 <= i <= N - w``.
6. S/N of position i at width w uses the block ``k* = floor((i + floor(w/2))/S)``
   of the window's centre: if ``MAD_{k*} = 0`` the position is not above;
   otherwise ``snr = S_w(i) / ((K * MAD_{k*}) * sqrt(w))`` evaluated in IEEE
   double in exactly that order, and the position is above iff ``snr > theta``.
7. Peak detection: for each (row, width), every maximal run of consecutive
   above positions yields one candidate at its first arg-max:
   ``(dm_idx, sample=i*, width=w, snr=(float32) snr(i*))``.
8. Streaming is item 1-7 applied to the concatenation of the gulps; a batch is
   item 1-7 applied to every item on its own.
9. Centred-window variant (a plan option; the paper's "moving average" does
   not say where the window sits): the window of block k reaches ``lead =
   max(0, floor((L - S) / 2))`` samples past the block's end,
   ``W_k = x[max(0, e_k + lead - L) : min(N, e_k + lead)]``, so it is centred
   on the block (exactly when L - S is even); everything else is unchanged.
10. Row-normalisation variant (a plan option; Section II-B's "RMS scaling"
    read as one noise scale per DM trial and chunk): the residual of item 5
    is computed as before, and every block of the row takes the one value
    ``MAD_row`` = lower median of ``|r_t - c|`` over the whole row, where
    ``c`` is the lower median of ``r_t``; items 6-7 then use it in place of
    ``MAD_{k*}``. The medians ``m_k`` are unchanged. In a stream the chunk
    is the gulp (gulps hold whole blocks): every block of gulp g takes the
    ``MAD_row`` of the residuals ``r_t`` whose t lies in gulp g, the
    residuals being those of item 5 on the concatenation (trailing windows
    reach back into earlier gulps).
11. Per-width re-normalisation variant (a plan option; Section II-B's
    normalisation read as a scale for every filtered series, the way
    Heimdall re-normalises each boxcar output): the residual and boxcar sums
    of items 5 are unchanged; for each row and width w the filtered series
    ``T_w = {S_w(i) : 0 <= i <= N - w}`` gets its own robust scale,
    ``c_w`` = lower median of ``T_w`` and ``MAD_w`` = lower median of
    ``|S_w(i) - c_w|``, and item 6 becomes ``snr = S_w(i) / (K * MAD_w)`` in
    IEEE double (no sqrt(w): ``MAD_w`` already measures the filtered series);
    a width with ``MAD_w = 0`` has no above positions. The medians ``m_k``
    are unchanged; items 7-8 are unchanged.
"""
from __future__ import annotations

import math
from typing import Iterable, List, Optional, Sequence, Tuple

import numpy as np

# 1 / Phi^{-1}(3/4): makes the MAD a consistent estimator of a Gaussian's sigma.
K_MAD = 1.482602218505602
BLOCK_STRIDE = 64

CAND_DTYPE = np.dtype([("sample", "<i8"), ("dm_idx", "<u4"), ("width", "<u4"), ("snr", "<f4")])


def widths(max_width: int) -> List[int]:
    """The boxcar bank: powers of two 1 .. max_width (matched filtering, Section II-B)."""
    out, w = [], 1
    while w <= max_width:
        out.append(w)
        w *= 2
    return out


def to_int(x: np.ndarray) -> np.ndarray:
    """Reading 1: integer value of each (integer-valued) FP32 sample."""
    return np.asarray(x).astype(np.int64)


def lower_median(values: np.ndarray) -> int:
    """Element of 0-based rank floor((n-1)/2) of the sorted values."""
    n = values.size
    r = (n - 1) // 2
    return int(np.partition(values, r)[r])


def window_lead(baseline_len: int, stride: int = BLOCK_STRIDE, centered: bool = False) -> int:
    """Reading 9: samples the baseline window reaches past its block (0: trailing)."""
    return max(0, (baseline_len - stride) // 2) if centered else 0


def block_median_mad(x_row: np.ndarray, baseline_len: int, stride: int = BLOCK_STRIDE,
                     lead: int = 0) -> Tuple[np.ndarray, np.ndarray]:
    """Readings 2-4 (and 9 with lead > 0): per-block lower median and MAD of the window.

    Baseline removal and normalisation stages (Section II-B; Algorithm 1's
    per-trial kernels). Returns int64 arrays ``m`` and ``mad`` of length
    ``ceil(N / stride)``.
    """
    x_row = to_int(x_row)
    n = x_row.size
    nb = (n + stride - 1) // stride
    m = np.empty(nb, dtype=np.int64)
    mad = np.empty(nb, dtype=np.int64)
    for k in range(nb):
        end = min(k * stride + stride, n) + lead
        lo = max(0, end - baseline_len)
        e = min(n, end)
        window = x_row[lo:e]
        m[k] = lower_median(window)
        mad[k] = lower_median(np.abs(window - m[k]))
    return m, mad


def residual(x_row: np.ndarray, m: np.ndarray, stride: int = BLOCK_STRIDE) -> np.ndarray:
    """Reading 5, first half: r_t = x_t - m_{floor(t/S)} (baseline removal)."""
    x_row = to_int(x_row)
    t = np.arange(x_row.size)
    return x_row - m[t // stride]


def row_mad(r: np.ndarray) -> int:
    """Reading 10: lower median absolute deviation of the whole row's residual about its lower median."""
    c = lower_median(r)
    return lower_median(np.abs(r - c))


def width_mad(sw: np.ndarray) -> Tuple[int, int]:
    """Reading 11: lower median c_w of the filtered series and its lower MAD about c_w (0, 0 if empty)."""
    if sw.size == 0:
        return 0, 0
    c = lower_median(sw)
    return c, lower_median(np.abs(sw - c))


def snr_and_above_width(sw: np.ndarray, mad_w: int, theta: float) -> Tuple[np.ndarray, np.ndarray]:
    """Reading 11: FP64 S/N against the width's own scale, S_w(i) / (K * MAD_w); strict threshold.

    A width with MAD_w = 0 has no above positions (snr NaN)."""
    if mad_w <= 0:
        return np.full(sw.size, np.nan), np.zeros(sw.size, dtype=bool)
    den = K_MAD * float(mad_w)
    snr = sw.astype(np.float64) / den
    th = float(np.float32(theta))
    return snr, snr > th


def boxcar(r: np.ndarray, w: int) -> np.ndarray:
    """Reading 5, second half: S_w(i) = sum of r over [i, i+w), i = 0 .. N-w (matched filter)."""
    n = r.size
    if w > n:
        return np.zeros(0, dtype=np.int64)
    p = np.concatenate([np.zeros(1, dtype=np.int64), np.cumsum(r, dtype=np.int64)])
    return p[w:] - p[:-w]


def snr_and_above(sw: np.ndarray, mad: np.ndarray, w: int, theta: float,
                  stride: int = BLOCK_STRIDE) -> Tuple[np.ndarray, np.ndarray]:
    """Reading 6: FP64 S/N of each position and the strict threshold test.

    ``theta`` is the plan's threshold as passed through the C interface
    (FP32), widened to double. Positions whose centre block has MAD = 0 are
    never above; their snr entry is NaN.
    """
    i = np.arange(sw.size)
    kstar = (i + w // 2) // stride
    madk = mad[kstar]
    ok = madk > 0
    den = (K_MAD * madk.astype(np.float64)) * math.sqrt(float(w))
    with np.errstate(divide="ignore", invalid="ignore"):
        snr = sw.astype(np.float64) / den
    snr = np.where(ok, snr, np.nan)
    th = float(np.float32(theta))
    above = ok & (snr > th)
    return snr, above


def peaks(above: np.ndarray, snr: np.ndarray) -> List[Tuple[int, float]]:
    """Reading 7: one (first arg-max index, snr) per maximal run of above positions (peak detection)."""
    if above.size == 0 or not above.any():
        return []
    a = above.astype(np.int8)
    edges = np.diff(np.concatenate([[0], a, [0]]))
    starts = np.flatnonzero(edges == 1)
    ends = np.flatnonzero(edges == -1)
    out = []
    for s, e in zip(starts, ends):
        j = s + int(np.argmax(snr[s:e]))
        out.append((j, float(snr[j])))
    return out


def gulp_row_mads(r: np.ndarray, gulp_len: int, stride: int = BLOCK_STRIDE) -> np.ndarray:
    """Reading 10 in a stream: block k takes the row MAD of the residuals of the gulp holding it."""
    if gulp_len <= 0 or gulp_len % stride:
        raise ValueError("gulps hold whole blocks")
    nb = (r.size + stride - 1) // stride
    per_gulp = gulp_len // stride
    out = np.empty(nb, dtype=np.int64)
    for g0 in range(0, r.size, gulp_len):
        k0 = g0 // stride
        out[k0:k0 + per_gulp] = row_mad(r[g0:g0 + gulp_len])
    return out


def search_row(x_row: np.ndarray, dm_idx: int, max_width: int, baseline_len: int, theta: float,
               stride: int = BLOCK_STRIDE, with_stats: bool = False, lead: int = 0, row_norm: bool = False,
               width_norm: bool = False, gulp_len: int = 0):
    """Stages of one DM trial in the paper's order: baseline, normalise, filter, detect.

    ``gulp_len`` > 0 with ``row_norm``: one scale per gulp of that length
    (reading 10 in a stream)."""
    if row_norm and width_norm:
        raise ValueError("row_norm and width_norm are alternative readings")
    m, mad = block_median_mad(x_row, baseline_len, stride, lead)
    r = residual(x_row, m, stride)
    if row_norm and gulp_len > 0:
        mad = gulp_row_mads(r, gulp_len, stride)
    elif row_norm:
        mad = np.full(mad.size, row_mad(r), dtype=np.int64)
    cands = []
    for w in widths(max_width):
        sw = boxcar(r, w)
        if sw.size == 0:
            continue
        if width_norm:
            snr, above = snr_and_above_width(sw, width_mad(sw)[1], theta)
        else:
            snr, above = snr_and_above(sw, mad, w, theta, stride)
        for j, s in peaks(above, snr):
            cands.append((j, dm_idx, w, s))
    arr = np.array(cands, dtype=[("sample", "<i8"), ("dm_idx", "<u4"), ("width", "<u4"), ("snr", "<f8")])
    out = np.empty(arr.size, dtype=CAND_DTYPE)
    for f in ("sample", "dm_idx", "width"):
        out[f] = arr[f]
    out["snr"] = arr["snr"].astype(np.float32)
    if with_stats:
        return out, m, mad
    return out


def width_stats(x_row: np.ndarray, max_width: int, baseline_len: int, stride: int = BLOCK_STRIDE,
                lead: int = 0) -> Tuple[np.ndarray, np.ndarray]:
    """Reading 11's statistics of one row: c_w and MAD_w for every width (int64 arrays)."""
    m, _ = block_median_mad(x_row, baseline_len, stride, lead)
    r = residual(x_row, m, stride)
    cs, ms = [], []
    for w in widths(max_width):
        c, d = width_mad(boxcar(r, w))
        cs.append(c)
        ms.append(d)
    return np.array(cs, dtype=np.int64), np.array(ms, dtype=np.int64)


def sort_cands(c: np.ndarray) -> np.ndarray:
    """Canonical order (dm_idx, width, sample): candidate order is not part of the result."""
    if c.size == 0:
        return c
    return c[np.lexsort((c["sample"], c["width"], c["dm_idx"]))]


def search(block: np.ndarray, max_width: int, baseline_len: int, theta: float,
           rows: Optional[Iterable[int]] = None, stride: int = BLOCK_STRIDE,
           row_ids: Optional[Sequence[int]] = None, with_stats: bool = False, centered: bool = False,
           row_norm: bool = False, width_norm: bool = False, gulp_len: int = 0):
    """Search every row of ``block`` ([ndm][N]); candidates sorted (dm, width, sample).

    ``rows`` restricts the search to those rows of ``block``; ``row_ids``
    gives the DM index reported for each row of ``block`` (default: the row's
    position). With ``with_stats`` also returns int64 ``m`` and ``mad`` of
    shape ``[len(rows)][ceil(N/S)]``. ``centered``, ``row_norm`` and
    ``width_norm`` select readings 9, 10 and 11; ``gulp_len`` > 0 with
    ``row_norm`` takes one row scale per gulp of that length.
    """
    block = np.asarray(block)
    if block.ndim != 2:
        raise ValueError("block must be [ndm][nsamp]")
    rr = range(block.shape[0]) if rows is None else list(rows)
    parts, ms, mads = [], [], []
    for r in rr:
        d = r if row_ids is None else int(row_ids[r])
        c, m, mad = search_row(block[r], d, max_width, baseline_len, theta, stride, with_stats=True,
                               lead=window_lead(baseline_len, stride, centered), row_norm=row_norm,
                               width_norm=width_norm, gulp_len=gulp_len)
        parts.append(c)
        ms.append(m)
        mads.append(mad)
    cands = sort_cands(np.concatenate(parts)) if parts else np.empty(0, dtype=CAND_DTYPE)
    if with_stats:
        nb = (block.shape[1] + stride - 1) // stride
        return (cands, np.array(ms).reshape(-1, nb), np.array(mads).reshape(-1, nb))
    return cands


def search_stream(gulps: Sequence[np.ndarray], max_width: int, baseline_len: int, theta: float,
                  stride: int = BLOCK_STRIDE, row_norm: bool = False) -> np.ndarray:
    """Reading 8: streaming equals the one-shot search of the concatenated gulps (global sample index).

    ``row_norm``: reading 10 per gulp (the gulps must have one length)."""
    gulps = list(gulps)
    if row_norm and len({g.shape[1] for g in gulps}) > 1:
        raise ValueError("a stream's gulps have one length")
    return search(np.concatenate(gulps, axis=1), max_width, baseline_len, theta, stride=stride, row_norm=row_norm,
                  gulp_len=gulps[0].shape[1] if row_norm else 0)


def search_batch(items: Sequence[Tuple[np.ndarray, int, int, float]], stride: int = BLOCK_STRIDE) -> List[np.ndarray]:
    """Reading 8: a batch is every (block, max_width, baseline_len, theta) searched on its own."""
    return [search(b, mw, L, th, stride=stride) for (b, mw, L, th) in items]
