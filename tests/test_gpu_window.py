"""GPU parity of the centred baseline window (SPS_ATTR_WINDOW = 1) against the oracle.

Medians and MADs bit-exact; candidates as in the trailing-window parity tests.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from parity import compare_cands, exact_equal

pytestmark = pytest.mark.gpu


def sps():
    from paper_2512_00398_amd import sps as m
    return m


def centred_search(x, max_width, L, theta, detect_seg=0, stats_seg=0, hist_bins=4096, plain=False):
    import torch
    m = sps()
    xd = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    ndm, n = x.shape
    with m.Plan(ndm, n, max_width, L, theta) as p:
        p.set(m.ATTR_WINDOW, 1)
        assert p.get(m.ATTR_WINDOW) == 1
        if detect_seg:
            p.set(m.ATTR_DETECT_SEG, detect_seg)
        if stats_seg:
            p.set(m.ATTR_STATS_SEG, stats_seg)
        p.set(m.ATTR_HIST_BINS, hist_bins)
        cands, ncand = p.alloc_cands()
        p.search(xd, cands, ncand, plain=plain)
        med, mad = p.block_stats(xd)
        torch.cuda.synchronize()
        return m.cands_to_numpy(cands, ncand, p.max_cands), med.cpu().numpy(), mad.cpu().numpy()


def check(x, max_width, L, theta, where, **kw):
    print("centred case %s shape=%s w=%d L=%d theta=%g %s" % (where, x.shape, max_width, L, theta, kw), flush=True)
    sys.stdout.flush()
    got, med, mad = centred_search(x, max_width, L, theta, **kw)
    ref, rm, rmad = oracle.search(x, max_width, L, theta, with_stats=True, centered=True)
    assert np.array_equal(med, rm), "%s: medians differ at %s" % (where, np.argwhere(med != rm)[:5])
    assert np.array_equal(mad, rmad), "%s: MADs differ at %s" % (where, np.argwhere(mad != rmad)[:5])
    assert compare_cands(got, ref, theta, where) == 0
    assert exact_equal(got, ref), where
    return got, ref


def test_centred_small_config():
    cfg = synth.config(1)["blocks"][0]
    x = synth.generate(cfg)
    got, ref = check(x, cfg.max_width, cfg.baseline_len, cfg.snr_thresh, "c1")
    # the placement changes the statistics, so the result differs from the trailing window's
    _, tm, _ = oracle.search(x[:2], cfg.max_width, cfg.baseline_len, cfg.snr_thresh, with_stats=True)
    _, cm, _ = oracle.search(x[:2], cfg.max_width, cfg.baseline_len, cfg.snr_thresh, with_stats=True, centered=True)
    assert not np.array_equal(tm, cm)
    assert ref.size > 1000


@pytest.mark.parametrize("stats_seg,detect_seg,bins", [(64, 1024, 4096), (333, 2048, 16384), (5, 0, 4096)])
def test_centred_tilings(stats_seg, detect_seg, bins):
    # short chain segments start inside the row, at windows clipped at both ends, and near the end
    rng = np.random.default_rng(40 + stats_seg)
    x = np.round(rng.normal(500, 25, size=(4, 20000)))
    x[:, 9000:9040] += 300
    x[2, 12000:] += 5000  # a step the centred window sees before the block reaches it
    check(x.astype(np.float32), 256, 3000, 4.0, "tiling-%d-%d-%d" % (stats_seg, detect_seg, bins),
          stats_seg=stats_seg, detect_seg=detect_seg, hist_bins=bins)


def test_centred_edge_cases_and_plain_path():
    rng = np.random.default_rng(41)
    # ragged rows, odd L - 64, L <= 64 (no lead), L longer than the row, maximum L
    for n, L, w in [(1, 5, 1), (63, 16, 16), (65, 129, 64), (1000, 64, 512), (1000, 100, 512), (3001, 701, 4096),
                    (5000, 12000, 256), (9000, 65535, 128)]:
        x = np.round(rng.normal(1000, 30, size=(3, n)))
        x[:, n // 2: n // 2 + 3] += 400
        x = x.astype(np.float32)
        check(x, w, L, 3.0, "ragged-%d-L%d" % (n, L))
        check(x, w, L, 3.0, "ragged-%d-L%d-plain" % (n, L), plain=True)
    # heavy ties and steps that move the median fast (recentring and the exact fallback)
    x = rng.integers(0, 3, size=(2, 9000)).astype(np.float32)
    x[1, 3000:] += 20000
    x[1, 6000:] -= 45000
    check(x, 128, 1000, 1.5, "ties-steps")
    x = np.round(rng.uniform(-4e6, 4e6, size=(2, 6000))).astype(np.float32)
    check(x, 256, 900, 2.5, "wide")


def test_centred_batch_equals_oracle():
    import torch
    m = sps()
    shapes = [(7, 3000, 64, 700, 5.0), (3, 65, 1, 1, 4.0), (5, 9000, 256, 16384, 4.5), (12, 20000, 1024, 3000, 6.0)]
    blocks = [synth.Block(ndm=nd, nsamp=n, max_width=w, baseline_len=L, snr_thresh=th, seed=700 + k, n_pulses=4,
                          pulse_width=(1, max(1, min(w, 256))), pulse_snr=(6.0, 25.0))
              for k, (nd, n, w, L, th) in enumerate(shapes)]
    xs_h = [synth.generate(b) for b in blocks]
    print("centred batch of %d items" % len(blocks), flush=True)
    with m.Batch() as b:
        b.set(m.ATTR_WINDOW, 1)
        items, outs = [], []
        for blk, x in zip(blocks, xs_h):
            cands = torch.empty((1 << 20, 4), dtype=torch.int32, device="cuda")
            ncand = torch.zeros((1,), dtype=torch.int32, device="cuda")
            outs.append((cands, ncand))
            items.append((torch.from_numpy(x).cuda(), blk.max_width, blk.baseline_len, blk.snr_thresh, cands, ncand))
        b.search(items)
        torch.cuda.synchronize()
        for k, (blk, x) in enumerate(zip(blocks, xs_h)):
            got = m.cands_to_numpy(*outs[k])
            a = np.empty(got.size, dtype=oracle.CAND_DTYPE)
            for f in ("sample", "dm_idx", "width", "snr"):
                a[f] = got[f]
            ref = oracle.search(x, blk.max_width, blk.baseline_len, blk.snr_thresh, centered=True)
            assert exact_equal(oracle.sort_cands(a), ref), "item %d" % k


def test_centred_window_attribute_rules():
    m = sps()
    with m.Plan(2, 4096, 64, 1000, 5.0) as p:
        assert p.get(m.ATTR_WINDOW) == 0
        with pytest.raises(m.SpsError):
            p.set(m.ATTR_WINDOW, 2)
        p.set(m.ATTR_WINDOW, 1)
        # a stream would need samples of the next gulp: refused
        with pytest.raises(m.SpsError):
            m.Stream(p)
        p.set(m.ATTR_WINDOW, 0)
        s = m.Stream(p)
        s.close()


@pytest.mark.parametrize("row_norm", [False, True])
def test_variants_full_size_sampled_rows(row_norm):
    # the 1024 x 2^20 block in the launch configuration the benchmark times
    # (bench.py --window centred [--norm row]); the oracle checks sampled rows
    import torch
    m = sps()
    cfg = synth.config(2)["blocks"][0]
    print("case c2 full size centred row_norm=%s: generate" % row_norm, flush=True)
    x = synth.generate(cfg)
    xd = torch.from_numpy(x).cuda()
    rows = [0, 700, 1023]
    with m.Plan(cfg.ndm, cfg.nsamp, cfg.max_width, cfg.baseline_len, cfg.snr_thresh) as p:
        p.set(m.ATTR_WINDOW, 1)
        p.set(m.ATTR_NORM, int(row_norm))
        cands, ncand = p.alloc_cands()
        p.search(xd, cands, ncand)
        med, mad = p.block_stats(xd)
        torch.cuda.synchronize()
        got = m.cands_to_numpy(cands, ncand, p.max_cands)
        med, mad = med.cpu().numpy(), mad.cpu().numpy()
    print("case c2 centred: oracle on rows %s (%d gpu candidates)" % (rows, got.size), flush=True)
    ref, rm, rmad = oracle.search(x, cfg.max_width, cfg.baseline_len, cfg.snr_thresh, rows=rows, with_stats=True,
                                  centered=True, row_norm=row_norm)
    assert np.array_equal(med[rows], rm) and np.array_equal(mad[rows], rmad)
    sel = np.isin(got["dm_idx"], rows)
    assert compare_cands(got[sel], ref, cfg.snr_thresh, "c2-centred-rows") == 0
    assert exact_equal(got[sel], ref)
    assert (got["sample"].astype(np.int64) + got["width"] <= cfg.nsamp).all()
