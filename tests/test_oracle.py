"""Pins for the CPU oracle: brute force, closed forms, invariants, statistics.

Each check is independent of the oracle's own code path (pure-Python sorts and
sums, the ``statistics`` module, closed-form S/N, Gaussian tail probabilities),
so that a dropped term, a wrong sign or index, or a transposed operand in the
oracle fails at least one of them.
"""
import math
import statistics

import numpy as np
import pytest
from scipy.stats import norm

import oracle
import synth

K = 1.482602218505602


def brute_stats(x, L, S):
    """Lower median and MAD of each trailing window by sorting Python lists."""
    n = len(x)
    ms, mads = [], []
    for k in range((n + S - 1) // S):
        e = min(k * S + S, n)
        w = sorted(x[max(0, e - L):e])
        r = (len(w) - 1) // 2
        m = w[r]
        d = sorted(abs(v - m) for v in w)[r]
        ms.append(m)
        mads.append(d)
    return ms, mads


def brute_search_row(x, dm, max_width, L, theta, S, row_norm=False, width_norm=False, gulp_len=0):
    """Whole search for one row with explicit loops only (row_norm: one MAD
    for the row, of the residual about its lower median, or with gulp_len
    one such MAD per gulp for the gulp's blocks; width_norm: one MAD per
    width, of the boxcar sums about their lower median, and no sqrt(w))."""
    ms, mads = brute_stats(x, L, S)
    n = len(x)
    r = [x[t] - ms[t // S] for t in range(n)]
    if row_norm:
        g = gulp_len if gulp_len else n
        mads = []
        for g0 in range(0, n, g):
            part = r[g0:g0 + g]
            c = sorted(part)[(len(part) - 1) // 2]
            d = sorted(abs(v - c) for v in part)[(len(part) - 1) // 2]
            mads += [d] * ((len(part) + S - 1) // S)
    th = float(np.float32(theta))
    out = []
    w = 1
    while w <= max_width:
        vals = []
        sums = [sum(r[i:i + w]) for i in range(n - w + 1)]
        if width_norm and sums:
            k = (len(sums) - 1) // 2
            cw = sorted(sums)[k]
            madw = sorted(abs(v - cw) for v in sums)[k]
        for i in range(n - w + 1):
            s = sums[i]
            mad = madw if width_norm else mads[(i + w // 2) // S]
            if mad == 0:
                vals.append(None)
                continue
            snr = s / (K * mad) if width_norm else s / ((K * mad) * math.sqrt(w))
            vals.append(snr if snr > th else None)
        i = 0
        while i < len(vals):
            if vals[i] is None:
                i += 1
                continue
            j, best, bi = i, vals[i], i
            while j < len(vals) and vals[j] is not None:
                if vals[j] > best:
                    best, bi = vals[j], j
                j += 1
            out.append((bi, dm, w, float(np.float32(best))))
            i = j
        w *= 2
    return sorted(out, key=lambda c: (c[1], c[2], c[0]))


def as_tuples(c):
    return [(int(a), int(b), int(w), float(s)) for a, b, w, s in zip(c["sample"], c["dm_idx"], c["width"], c["snr"])]


@pytest.mark.parametrize("n,L,S,seed", [(1, 5, 4, 0), (7, 3, 4, 1), (40, 9, 4, 2), (64, 64, 8, 3), (93, 17, 8, 4),
                                        (130, 1000, 16, 5), (257, 40, 64, 6), (300, 128, 64, 7)])
def test_median_mad_brute_force(n, L, S, seed):
    rng = np.random.default_rng(seed)
    x = rng.integers(-50, 50, size=n)
    # heavy ties in one half, spread values in the other
    x[: n // 2] = rng.integers(0, 3, size=n // 2)
    m, mad = oracle.block_median_mad(x.astype(np.float32), L, S)
    bm, bmad = brute_stats(x.tolist(), L, S)
    assert m.tolist() == bm
    assert mad.tolist() == bmad


def test_median_is_statistics_median_low_when_window_covers_row():
    # Special case L >= N: every window is a prefix; the last one is the row.
    rng = np.random.default_rng(11)
    for n in (63, 64, 100, 129):
        x = rng.integers(-1000, 1000, size=n)
        m, mad = oracle.block_median_mad(x, 10 * n, 64)
        ml = statistics.median_low(x.tolist())
        assert m[-1] == ml
        assert mad[-1] == statistics.median_low([abs(v - ml) for v in x.tolist()])
        # first block: prefix of length min(64, n)
        p = x[: min(64, n)].tolist()
        assert m[0] == statistics.median_low(p)


def test_boxcar_direct_sums():
    rng = np.random.default_rng(3)
    r = rng.integers(-100, 100, size=50)
    for w in (1, 2, 4, 8, 16, 32, 64):
        got = oracle.boxcar(r, w)
        want = [sum(r[i:i + w].tolist()) for i in range(len(r) - w + 1)] if w <= len(r) else []
        assert got.tolist() == want
        if w <= len(r):
            assert np.array_equal(got, np.convolve(r, np.ones(w, dtype=np.int64), "valid"))


@pytest.mark.parametrize("seed,n,L,S,maxw,theta", [(0, 200, 50, 8, 16, 1.5), (1, 333, 64, 16, 32, 1.2),
                                                    (2, 129, 500, 64, 64, 1.0), (3, 90, 7, 4, 8, 2.0)])
def test_search_row_brute_force(seed, n, L, S, maxw, theta):
    rng = np.random.default_rng(seed)
    x = rng.integers(0, 40, size=n)
    x[n // 3: n // 3 + 5] += 60  # a pulse so that wide widths fire too
    got = as_tuples(oracle.search_row(x, 5, maxw, L, theta, S))
    want = brute_search_row(x.tolist(), 5, maxw, L, theta, S)
    assert got == want
    assert len(got) > 0


def test_peaks_first_argmax_and_run_breaks():
    above = np.array([0, 1, 1, 1, 0, 1, 0, 0, 1, 1], dtype=bool)
    snr = np.array([9, 2, 5, 5, 9, 3, 9, 9, 7, 8], dtype=float)
    assert oracle.peaks(above, snr) == [(2, 5.0), (5, 3.0), (9, 8.0)]
    assert oracle.peaks(np.zeros(4, bool), snr[:4]) == []
    assert oracle.peaks(np.ones(3, bool), np.array([1.0, 1.0, 1.0])) == [(0, 1.0)]


def test_mad_zero_is_never_above():
    # Constant data: r == 0 exactly, MAD == 0, hence no candidates at all.
    x = np.full((3, 777), 12345.0, dtype=np.float32)
    c, m, mad = oracle.search(x, 64, 100, 0.5, with_stats=True)
    assert c.size == 0
    assert (m == 12345).all() and (mad == 0).all()
    assert (oracle.residual(x[0], m[0]) == 0).all()
    # MAD == 0 in one block breaks a run even if S is huge there
    snr, above = oracle.snr_and_above(np.array([100, 100, 100]), np.array([5, 0, 5]), 1, 1.0, stride=1)
    assert above.tolist() == [True, False, True]


def periodic_pulse_row(n, base, s, t0, w, amp):
    """Period-7 pattern (-2,-1,-1,0,1,1,2)*s with a zero run of 4w around a width-w pulse."""
    pat = np.array([-2, -1, -1, 0, 1, 1, 2]) * s
    x = base + pat[np.arange(n) % 7]
    x[t0 - 2 * w: t0 + 3 * w] = base
    x[t0: t0 + w] += amp
    return x


@pytest.mark.parametrize("w,expect", [(1, 6.744898), (4, 13.489795), (32, 38.154902)])
def test_snr_closed_form(w, expect):
    # m = base, MAD = s exactly, so the best candidate is at (t0, w) with snr = A sqrt(w) / (K s).
    base, s, amp, n, L = 32768, 100, 1000, 8192, 4096
    t0 = 6001
    x = periodic_pulse_row(n, base, s, t0, w, amp)
    c, m, mad = oracle.search(x[None, :].astype(np.float32), 64, L, 6.0, with_stats=True)
    assert (m == base).all()
    assert (mad == s).all()
    closed = amp * math.sqrt(w) / (K * s)
    assert abs(closed - expect) < 5e-6
    best = c[np.argmax(c["snr"])]
    assert (int(best["sample"]), int(best["width"])) == (t0, w)
    assert best["snr"] == np.float32(closed)
    # nothing fires away from the pulse: |S_w| <= 3s on the periodic pattern
    assert ((c["sample"] >= t0 - 64) & (c["sample"] < t0 + w + 64)).all()


def test_translation_invariance_bit_exact():
    b = synth.Block(ndm=3, nsamp=6000, max_width=64, baseline_len=1000, seed=77, n_pulses=3,
                    pulse_snr=(8, 20))
    x = synth.generate(b)
    c0 = oracle.search(x, 64, 1000, 5.0)
    c1 = oracle.search(x + np.float32(-20000), 64, 1000, 5.0)
    assert c0.size > 0
    assert np.array_equal(c0, c1)


def test_scale_invariance():
    b = synth.Block(ndm=2, nsamp=5000, max_width=32, baseline_len=700, seed=78, n_pulses=2,
                    pulse_snr=(8, 20))
    x = oracle.to_int(synth.generate(b)) - 32768
    c0 = oracle.search(x, 32, 700, 5.0)
    c3 = oracle.search(3 * x, 32, 700, 5.0)
    assert np.array_equal(c0[["sample", "dm_idx", "width"]], c3[["sample", "dm_idx", "width"]])
    np.testing.assert_allclose(c0["snr"], c3["snr"], rtol=1e-6)


@pytest.mark.slow
def test_noise_only_false_alarms_gaussian_tail():
    # Drift-free integer Gaussian noise, width 1: the number of above positions
    # (after the first L samples, whose windows are clipped) follows the
    # Gaussian tail count N_eff * Q(theta) to within Poisson scatter.
    b = synth.Block(ndm=6, nsamp=1 << 19, max_width=1, baseline_len=16384, seed=4242, drift_amp_sigma=0.0)
    x = synth.generate(b)
    for th in (4.0, 4.5):
        tot, neff = 0, 0
        for r in range(b.ndm):
            m, mad = oracle.block_median_mad(x[r], b.baseline_len)
            sw = oracle.boxcar(oracle.residual(x[r], m), 1)
            _, above = oracle.snr_and_above(sw, mad, 1, th)
            tot += int(above[b.baseline_len:].sum())
            neff += above.size - b.baseline_len
        lam = neff * norm.sf(th)
        z = (tot - lam) / math.sqrt(lam)
        assert abs(z) < 3.0, (th, tot, lam, z)  # within 3 Poisson sigmas of the tail count


def test_stream_equals_concatenation_and_batch_is_per_item():
    b = synth.Block(ndm=2, nsamp=4096, max_width=16, baseline_len=500, seed=5, n_pulses=2, pulse_snr=(8, 12))
    x = synth.generate(b)
    whole = oracle.search(x, 16, 500, 5.0)
    assert np.array_equal(oracle.search_stream([x[:, :1024], x[:, 1024:3072], x[:, 3072:]], 16, 500, 5.0), whole)
    res = oracle.search_batch([(x, 16, 500, 5.0), (x[:1, :2000], 8, 300, 4.0)])
    assert np.array_equal(res[0], whole)
    assert np.array_equal(res[1], oracle.search(x[:1, :2000], 8, 300, 4.0))


def test_widths_and_edges():
    assert oracle.widths(1) == [1]
    assert oracle.widths(64) == [1, 2, 4, 8, 16, 32, 64]
    # widths longer than the row give no positions
    x = np.arange(10, dtype=np.float32)
    c = oracle.search(x[None, :], 64, 5, 0.1)
    assert (c["width"] <= 10).all()
    # a single-sample row: MAD = 0, nothing
    assert oracle.search(np.ones((1, 1), np.float32), 4, 4, 0.1).size == 0


def brute_centred_stats(x, L, S):
    """Lower median and MAD of windows centred on each block's middle sample
    (c - L/2 .. c + L/2, clipped to the row), for rows of whole blocks."""
    n = len(x)
    ms, mads = [], []
    for k in range(n // S):
        c = k * S + S // 2
        w = sorted(x[max(0, c - L // 2):min(n, c + L // 2)])
        r = (len(w) - 1) // 2
        ms.append(w[r])
        mads.append(sorted(abs(v - w[r]) for v in w)[r])
    return ms, mads


@pytest.mark.parametrize("n,L,S,seed", [(64, 16, 8, 0), (96, 40, 8, 1), (256, 64, 64, 2), (512, 192, 64, 3),
                                        (640, 4096, 64, 4), (48, 20, 4, 5)])
def test_centred_window_brute_force(n, L, S, seed):
    # rows of whole blocks and L - S even: the window reaches (L - S) / 2 past
    # its block, i.e. it is centred on the block's middle
    rng = np.random.default_rng(seed)
    x = rng.integers(-50, 50, size=n)
    x[: n // 3] = rng.integers(0, 3, size=n // 3)
    lead = oracle.window_lead(L, S, centered=True)
    assert lead == (L - S) // 2
    m, mad = oracle.block_median_mad(x, L, S, lead)
    bm, bmad = brute_centred_stats(x.tolist(), L, S)
    assert m.tolist() == bm and mad.tolist() == bmad


def test_centred_window_time_reversal():
    # A centred window maps to a centred window under time reversal: block k
    # of the reversed row has the statistics of block nb-1-k of the row.
    rng = np.random.default_rng(21)
    for n, L in ((1024, 320), (2048, 1000), (640, 64)):
        x = rng.integers(-300, 300, size=n)
        lead = oracle.window_lead(L, 64, centered=True)
        m, mad = oracle.block_median_mad(x, L, 64, lead)
        mr, madr = oracle.block_median_mad(x[::-1].copy(), L, 64, lead)
        assert np.array_equal(mr, m[::-1]) and np.array_equal(madr, mad[::-1])


def test_centred_window_short_is_trailing():
    # L <= S: nothing to centre, the window is the trailing one
    assert oracle.window_lead(64, 64, centered=True) == 0 and oracle.window_lead(10, 64, centered=True) == 0
    x = np.random.default_rng(3).integers(-9, 9, size=500)
    a = oracle.search(x[None, :].astype(np.float32), 8, 40, 2.0, centered=True)
    b = oracle.search(x[None, :].astype(np.float32), 8, 40, 2.0)
    assert np.array_equal(a, b)


def test_centred_search_matches_explicit_loops():
    rng = np.random.default_rng(8)
    S, L = 64, 320
    x = rng.integers(-20, 20, size=640)
    x[300:306] += 60
    ms, mads = brute_centred_stats(x.tolist(), L, S)
    # the explicit search with these statistics (whole blocks, so every block is centred)
    th = 3.0
    got = oracle.search(x[None, :].astype(np.float32), 16, L, th, centered=True)
    r = [int(x[t]) - ms[t // S] for t in range(len(x))]
    out, w = [], 1
    while w <= 16:
        vals = []
        for i in range(len(x) - w + 1):
            mad = mads[(i + w // 2) // S]
            s = sum(r[i:i + w])
            v = s / ((K * mad) * math.sqrt(w)) if mad else None
            vals.append(v if v is not None and v > th else None)
        i = 0
        while i < len(vals):
            if vals[i] is None:
                i += 1
                continue
            j, bi = i, i
            while j < len(vals) and vals[j] is not None:
                if vals[j] > vals[bi]:
                    bi = j
                j += 1
            out.append((bi, 0, w, float(np.float32(vals[bi]))))
            i = j
        w *= 2
    assert as_tuples(got) == sorted(out, key=lambda c: (c[1], c[2], c[0]))
    assert len(out) > 0


@pytest.mark.parametrize("n,L,S,maxw,theta,seed", [(200, 50, 8, 16, 3.0, 0), (333, 90, 16, 32, 2.5, 1),
                                                   (97, 500, 8, 64, 2.0, 2), (640, 128, 64, 8, 3.5, 3)])
def test_row_norm_brute_force(n, L, S, maxw, theta, seed):
    rng = np.random.default_rng(100 + seed)
    x = rng.integers(-40, 40, size=n)
    x[n // 2:n // 2 + 4] += 150
    x[: n // 5] += 30  # a step: per-block and per-row scales differ
    got = oracle.search_row(x, 5, maxw, L, theta, S, row_norm=True)
    want = brute_search_row(x.tolist(), 5, maxw, L, theta, S, row_norm=True)
    assert as_tuples(oracle.sort_cands(got)) == want
    assert len(want) > 0
    _, _, mad = oracle.search_row(x, 5, maxw, L, theta, S, with_stats=True)
    _, _, rmad = oracle.search_row(x, 5, maxw, L, theta, S, with_stats=True, row_norm=True)
    assert np.all(rmad == rmad[0]) and not np.array_equal(mad, rmad)


@pytest.mark.parametrize("gulp,ngulps,L,S,maxw,theta,seed", [(64, 4, 50, 8, 16, 3.0, 0), (96, 3, 150, 16, 32, 2.5, 1),
                                                            (128, 2, 300, 64, 8, 3.0, 2), (40, 5, 17, 8, 64, 2.0, 3)])
def test_row_norm_per_gulp_brute_force(gulp, ngulps, L, S, maxw, theta, seed):
    # a stream takes one row scale per gulp; gulps of very different noise
    rng = np.random.default_rng(700 + seed)
    parts = [rng.integers(-a, a + 1, size=(2, gulp)) for a in (5, 60, 9, 200, 30)[:ngulps]]
    parts[-1][:, gulp // 2:gulp // 2 + 3] += 500
    got = oracle.search_stream([p.astype(np.float32) for p in parts], maxw, L, theta, stride=S, row_norm=True)
    x = np.concatenate(parts, axis=1)
    want = []
    for row in range(2):
        want += brute_search_row(x[row].tolist(), row, maxw, L, theta, S, row_norm=True, gulp_len=gulp)
    assert as_tuples(got) == sorted(want, key=lambda c: (c[1], c[2], c[0]))
    assert len(want) > 0


def test_row_norm_one_gulp_is_the_row_scale():
    rng = np.random.default_rng(71)
    x = rng.integers(-50, 51, size=(3, 640)).astype(np.float32)
    x[:, 300:305] += 400
    one = oracle.search_stream([x], 32, 200, 3.0, row_norm=True)
    assert np.array_equal(one, oracle.search(x, 32, 200, 3.0, row_norm=True))
    assert one.size > 0


def test_row_norm_per_gulp_scales_follow_each_gulp():
    # uniform integers on [-a, a] about a zero baseline: the MAD of a long gulp
    # is close to a/2, so the per-gulp scales track each gulp's noise
    rng = np.random.default_rng(72)
    n = 64 * 400
    x = np.concatenate([rng.integers(-a, a + 1, size=n) for a in (10, 100, 40)])
    m, _ = oracle.block_median_mad(x, 64 * 8)
    r = oracle.residual(x, m)
    mads = oracle.gulp_row_mads(r, n)
    per = n // 64
    for g, a in enumerate((10, 100, 40)):
        blk = mads[g * per:(g + 1) * per]
        assert np.all(blk == blk[0])
        assert abs(blk[0] - a / 2) <= 0.1 * a
    with pytest.raises(ValueError):
        oracle.gulp_row_mads(r, 100)  # gulps hold whole blocks
    with pytest.raises(ValueError):
        oracle.search_stream([x[None, :640].astype(np.float32), x[None, :704].astype(np.float32)], 8, 64, 3.0,
                             row_norm=True)


def test_row_norm_shift_and_scale_invariance():
    # adding a constant moves every median by it; doubling doubles every sum
    # and MAD exactly (binary floating point), so the S/N values are unchanged
    rng = np.random.default_rng(17)
    x = rng.integers(-500, 500, size=(3, 3000))
    x[:, 1000:1010] += 3000
    ref = oracle.search(x.astype(np.float32), 64, 700, 4.0, row_norm=True)
    assert ref.size > 0
    for y in (x + 12345, 2 * x, 2 * x - 77):
        assert np.array_equal(oracle.search(y.astype(np.float32), 64, 700, 4.0, row_norm=True), ref)


def test_row_norm_equals_block_norm_on_periodic_rows():
    # a row repeating one 64-sample pattern: every window of whole blocks holds
    # copies of the pattern, so each block's median and MAD are the pattern's,
    # the residual's row median is 0 and its row MAD is the block MAD
    rng = np.random.default_rng(23)
    pat = rng.integers(-30, 30, size=64)
    pat[17] += 400
    x = np.tile(pat, 40)[None, :].astype(np.float32)
    a, m, mad = oracle.search(x, 8, 64 * 5, 3.0, with_stats=True)
    b, _, rmad = oracle.search(x, 8, 64 * 5, 3.0, with_stats=True, row_norm=True)
    assert np.all(mad == mad[0, 0]) and np.array_equal(mad, rmad)
    assert a.size > 0 and np.array_equal(a, b)


def test_row_mad_closed_form():
    # residual of a constant-baseline row {0, 1, ..., n-1} shifted: about its median
    r = np.arange(11) - 3
    assert oracle.row_mad(r) == 3  # lower median 2, deviations 0..8 -> sorted rank 5 is 3
    assert oracle.row_mad(np.array([5, 5, 5, 9])) == 0
    assert oracle.row_mad(np.array([1, -1])) == 0  # lower median -1: deviations {2, 0}


# ---- reading 11: per-width re-normalisation ----

@pytest.mark.parametrize("n,L,S,maxw,theta,seed", [(50, 9, 4, 8, 1.5, 31), (130, 40, 8, 32, 2.0, 32),
                                                   (257, 100, 64, 64, 2.5, 33), (300, 64, 16, 128, 3.0, 34),
                                                   (97, 1000, 8, 256, 1.0, 35)])
def test_width_norm_brute_force(n, L, S, maxw, theta, seed):
    rng = np.random.default_rng(seed)
    x = rng.integers(-50, 50, size=n)
    x[n // 3: n // 3 + 5] += 300
    got, _, _ = oracle.search_row(x, 3, maxw, L, theta, S, with_stats=True, width_norm=True)
    want = brute_search_row(x.tolist(), 3, maxw, L, theta, S, width_norm=True)
    assert as_tuples(oracle.sort_cands(got)) == want
    assert len(want) > 0


def test_width_norm_closed_form_on_periodic_row():
    # Period-7 pattern p = (-2,-1,-1,0,1,1,2)*s, baseline exactly `base`
    # (zero run of 4w around a width-4 pulse of amplitude A): the boxcar sums
    # over whole pattern windows repeat with period 7 and, since the seven
    # values sum to 0, S_w has the distribution of S_{w mod 7}:
    #   w mod 7 = 1: {-2,-1,-1,0,1,1,2}s  -> c_w = 0, MAD_w = s
    #   w mod 7 = 2: {-3,-2,-1,1,2,3,0}s  -> c_w = 0, MAD_w = 2s
    #   w mod 7 = 4: {-4,-1,1,4,2,0,-2}s  -> c_w = 0, MAD_w = 2s
    # (the few windows touching the pulse or the zero run do not move these
    # ranks on a 28000-sample row). The pulse then gives snr = 4A/(K*2s) at
    # width 4 and A/(K*s) at width 1, both at its first sample.
    base, s, amp, n, L, w = 32768, 100, 1000, 28000, 4096, 4
    t0 = 14001
    x = periodic_pulse_row(n, base, s, t0, w, amp)
    c, mad = oracle.width_stats(x, 64, L)
    want_mad = {1: s, 2: 2 * s, 4: 2 * s, 8: s, 16: 2 * s, 32: 2 * s, 64: s}
    assert c.tolist() == [0] * 7
    assert mad.tolist() == [want_mad[v] for v in oracle.widths(64)]
    cands = oracle.search(x[None, :].astype(np.float32), 64, L, 6.0, width_norm=True)
    by_w = {int(cw): cands[cands["width"] == cw] for cw in (1, 4)}
    for cw, snr in ((1, amp / (K * s)), (4, 4 * amp / (K * 2 * s))):
        best = by_w[cw][np.argmax(by_w[cw]["snr"])]
        assert int(best["sample"]) == t0
        assert best["snr"] == np.float32(snr)
    assert abs(amp / (K * s) - 6.744898) < 5e-6 and abs(4 * amp / (K * 2 * s) - 13.489795) < 5e-6


def test_width_norm_shift_and_scale_invariance():
    # adding a constant moves every median (and no boxcar sum); doubling the
    # row doubles every sum and every MAD_w exactly, so no S/N changes
    rng = np.random.default_rng(41)
    x = rng.integers(-400, 400, size=(2, 4000))
    x[:, 2000:2016] += 900
    ref = oracle.search(x.astype(np.float32), 256, 900, 4.0, width_norm=True)
    assert ref.size > 0
    for y in (x + 5555, 2 * x, 2 * x - 31):
        assert np.array_equal(oracle.search(y.astype(np.float32), 256, 900, 4.0, width_norm=True), ref)


def test_width_norm_degenerate_cases():
    # constant row: every S_w is 0, MAD_w = 0, nothing is above
    x = np.full((1, 500), 77.0, dtype=np.float32)
    c, mad = oracle.width_stats(x[0], 16, 100)
    assert (c == 0).all() and (mad == 0).all()
    assert oracle.search(x, 16, 100, 0.5, width_norm=True).size == 0
    # widths longer than the row have no positions: statistics 0, no candidates
    c, mad = oracle.width_stats(np.arange(10), 64, 5)
    assert c[-1] == 0 and mad[-1] == 0
    with pytest.raises(ValueError):
        oracle.search(x, 16, 100, 0.5, width_norm=True, row_norm=True)
