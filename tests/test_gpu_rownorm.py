"""GPU parity of the per-row noise scale (SPS_ATTR_NORM = 1) against the oracle.

Medians and MADs bit-exact (every block of a row reports the row's MAD);
candidates as in the per-block parity tests.
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


def run(x, max_width, L, theta, centred=False, plain=False, stats_seg=0):
    import torch
    m = sps()
    xd = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    ndm, n = x.shape
    with m.Plan(ndm, n, max_width, L, theta) as p:
        p.set(m.ATTR_NORM, 1)
        assert p.get(m.ATTR_NORM) == 1
        if centred:
            p.set(m.ATTR_WINDOW, 1)
        if stats_seg:
            p.set(m.ATTR_STATS_SEG, stats_seg)
        cands, ncand = p.alloc_cands()
        p.search(xd, cands, ncand, plain=plain)
        med, mad = p.block_stats(xd)
        torch.cuda.synchronize()
        return m.cands_to_numpy(cands, ncand, p.max_cands), med.cpu().numpy(), mad.cpu().numpy()


def check(x, max_width, L, theta, where, centred=False, **kw):
    print("row-norm case %s shape=%s w=%d L=%d theta=%g centred=%s %s" % (where, x.shape, max_width, L, theta,
                                                                        centred, kw), flush=True)
    sys.stdout.flush()
    got, med, mad = run(x, max_width, L, theta, centred=centred, **kw)
    ref, rm, rmad = oracle.search(x, max_width, L, theta, with_stats=True, centered=centred, row_norm=True)
    assert np.array_equal(med, rm), "%s: medians differ at %s" % (where, np.argwhere(med != rm)[:5])
    assert np.array_equal(mad, rmad), "%s: row MADs differ at %s" % (where, np.argwhere(mad != rmad)[:5])
    assert compare_cands(got, ref, theta, where) == 0
    assert exact_equal(got, ref), where
    return got, ref


def test_row_norm_small_config():
    cfg = synth.config(1)["blocks"][0]
    x = synth.generate(cfg)
    _, ref = check(x, cfg.max_width, cfg.baseline_len, cfg.snr_thresh, "c1")
    assert ref.size > 1000


def test_row_norm_edge_cases_and_plain_path():
    rng = np.random.default_rng(51)
    for n, L, w in [(1, 5, 1), (2, 5, 1), (63, 16, 16), (1000, 100, 512), (3001, 700, 4096), (70000, 4096, 256)]:
        x = np.round(rng.normal(1000, 30, size=(3, n)))
        x[:, n // 2: n // 2 + 3] += 400
        x = x.astype(np.float32)
        check(x, w, L, 3.0, "ragged-%d" % n)
        check(x, w, L, 3.0, "ragged-%d-plain" % n, plain=True)
    # constant rows: row MAD 0, no candidates; next to a noisy row
    x = np.full((2, 5000), 777.0, dtype=np.float32)
    x[1] = np.round(rng.normal(0, 5, size=5000))
    check(x, 64, 512, 2.0, "constant")
    # residuals far from 0 and spread wide: both selects leave their first window (radix path)
    t = np.arange(20000, dtype=np.float64)
    x = np.stack([np.round(2000.0 * (t % 7000)), np.round(rng.uniform(-4e6, 4e6, size=t.size))]).astype(np.float32)
    check(x, 64, 900, 2.5, "ramp-wide")
    # median inside the LDS window, MAD far outside it: 40% / 20% / 40% of the
    # samples at -1e5 / 0 / +1e5 (the deviations take their own select)
    lev = rng.choice(np.array([-1e5, 0.0, 1e5]), p=[0.4, 0.2, 0.4], size=(2, 12000))
    x = (lev + np.round(rng.normal(0, 20, size=lev.shape))).astype(np.float32)
    x[0, 5000:5004] += 6e5
    check(x, 32, 2000, 2.0, "three-level")
    # heavy ties and steps
    x = rng.integers(0, 3, size=(2, 9000)).astype(np.float32)
    x[1, 3000:] += 20000
    x[1, 6000:] -= 45000
    check(x, 128, 1000, 1.5, "ties-steps")
    # with the centred window too
    x = np.round(rng.normal(-8e6, 40, size=(3, 7000))).astype(np.float32)
    x[0, 4000:4010] += 900
    check(x, 64, 2000, 4.0, "centred", centred=True, stats_seg=9)


def test_row_norm_batch_equals_oracle():
    import torch
    m = sps()
    shapes = [(7, 3000, 64, 700, 5.0), (3, 65, 1, 1, 4.0), (5, 9000, 256, 16384, 4.5), (12, 20000, 1024, 3000, 6.0)]
    blocks = [synth.Block(ndm=nd, nsamp=n, max_width=w, baseline_len=L, snr_thresh=th, seed=900 + k, n_pulses=4,
                          pulse_width=(1, max(1, min(w, 256))), pulse_snr=(6.0, 25.0))
              for k, (nd, n, w, L, th) in enumerate(shapes)]
    xs_h = [synth.generate(b) for b in blocks]
    print("row-norm batch of %d items" % len(blocks), flush=True)
    with m.Batch() as b:
        b.set(m.ATTR_NORM, 1)
        items, outs = [], []
        for blk, x in zip(blocks, xs_h):
            cands = torch.empty((1 << 20, 4), dtype=torch.int32, device="cuda")
            ncand = torch.zeros((1,), dtype=torch.int32, device="cuda")
            outs.append((cands, ncand))
            items.append((torch.from_numpy(x).cuda(), blk.max_width, blk.baseline_len, blk.snr_thresh, cands, ncand))
        b.search(items)
        torch.cuda.synchronize()
        total = 0
        for k, (blk, x) in enumerate(zip(blocks, xs_h)):
            got = m.cands_to_numpy(*outs[k])
            a = np.empty(got.size, dtype=oracle.CAND_DTYPE)
            for f in ("sample", "dm_idx", "width", "snr"):
                a[f] = got[f]
            ref = oracle.search(x, blk.max_width, blk.baseline_len, blk.snr_thresh, row_norm=True)
            assert exact_equal(oracle.sort_cands(a), ref), "item %d" % k
            total += ref.size
        assert total > 0


def test_row_norm_attribute_rules():
    m = sps()
    with m.Plan(2, 4096, 64, 1000, 5.0) as p:
        assert p.get(m.ATTR_NORM) == 0
        with pytest.raises(m.SpsError):
            p.set(m.ATTR_NORM, 3)
        p.set(m.ATTR_NORM, 1)
        m.Stream(p).close()  # a stream takes one row scale per gulp


def test_row_norm_full_size_sampled_rows():
    # the 1024 x 2^20 block in the launch configuration the benchmark times
    # (bench.py --norm row); the oracle checks sampled rows
    import torch
    m = sps()
    cfg = synth.config(2)["blocks"][0]
    print("case c2 full size row_norm: generate", flush=True)
    x = synth.generate(cfg)
    xd = torch.from_numpy(x).cuda()
    rows = [3, 512, 1022]
    with m.Plan(cfg.ndm, cfg.nsamp, cfg.max_width, cfg.baseline_len, cfg.snr_thresh) as p:
        p.set(m.ATTR_NORM, 1)
        cands, ncand = p.alloc_cands()
        p.search(xd, cands, ncand)
        med, mad = p.block_stats(xd)
        torch.cuda.synchronize()
        got = m.cands_to_numpy(cands, ncand, p.max_cands)
        med, mad = med.cpu().numpy(), mad.cpu().numpy()
    print("case c2 row_norm: oracle on rows %s (%d gpu candidates)" % (rows, got.size), flush=True)
    ref, rm, rmad = oracle.search(x, cfg.max_width, cfg.baseline_len, cfg.snr_thresh, rows=rows, with_stats=True,
                                  row_norm=True)
    assert np.array_equal(med[rows], rm) and np.array_equal(mad[rows], rmad)
    assert all(np.all(mad[r] == mad[r, 0]) for r in range(cfg.ndm))
    sel = np.isin(got["dm_idx"], rows)
    assert compare_cands(got[sel], ref, cfg.snr_thresh, "c2-rownorm-rows") == 0
    assert exact_equal(got[sel], ref)
