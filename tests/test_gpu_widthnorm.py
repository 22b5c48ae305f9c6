"""GPU parity of the per-width noise scale (SPS_ATTR_NORM = 2) against the oracle.

The per-width medians c_w and MADs of the boxcar-filtered series are
bit-exact (sps_width_stats); candidates follow the parity rule and are
bitwise equal here.
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


def run(x, max_width, L, theta, detect_seg=0):
    import torch
    m = sps()
    xd = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    ndm, n = x.shape
    with m.Plan(ndm, n, max_width, L, theta) as p:
        p.set(m.ATTR_NORM, 2)
        assert p.get(m.ATTR_NORM) == 2
        if detect_seg:
            p.set(m.ATTR_DETECT_SEG, detect_seg)
        cands, ncand = p.alloc_cands()
        p.search(xd, cands, ncand)
        c, d = p.width_stats(xd)
        torch.cuda.synchronize()
        return m.cands_to_numpy(cands, ncand, p.max_cands), c.cpu().numpy(), d.cpu().numpy()


def oracle_width_stats(x, max_width, L):
    cs, ds = [], []
    for r in range(x.shape[0]):
        c, d = oracle.width_stats(x[r], max_width, L)
        cs.append(c)
        ds.append(d)
    return np.array(cs), np.array(ds)


def check(x, max_width, L, theta, where, **kw):
    print("width-norm case %s shape=%s w=%d L=%d theta=%g %s" % (where, x.shape, max_width, L, theta, kw),
          flush=True)
    sys.stdout.flush()
    got, c, d = run(x, max_width, L, theta, **kw)
    rc, rd = oracle_width_stats(x, max_width, L)
    assert np.array_equal(c, rc), "%s: medians c_w differ at %s" % (where, np.argwhere(c != rc)[:5])
    assert np.array_equal(d, rd), "%s: MAD_w differ at %s" % (where, np.argwhere(d != rd)[:5])
    ref = oracle.search(x, max_width, L, theta, width_norm=True)
    assert compare_cands(got, ref, theta, where) == 0
    assert exact_equal(got, ref), where
    return got, ref


def test_width_norm_small_config():
    cfg = synth.config(1)["blocks"][0]
    x = synth.generate(cfg)
    # the drift widens every filtered series, so its own scale leaves few candidates
    _, ref = check(x, cfg.max_width, cfg.baseline_len, cfg.snr_thresh, "c1")
    assert ref.size > 0


def test_width_norm_edge_cases():
    rng = np.random.default_rng(61)
    # ragged rows, rows shorter than some widths (those widths: c_w = MAD_w = 0,
    # no candidates), steps of 4096 samples and their tails, several segments
    for n, L, w, seg in [(1, 5, 1, 0), (2, 5, 2, 0), (3, 9, 4, 0), (63, 16, 64, 0), (1000, 100, 512, 0),
                         (4095, 700, 4096, 0), (4096, 700, 4096, 0), (4097, 700, 4096, 0),
                         (12289, 3000, 256, 1024), (70001, 4096, 4096, 8192)]:
        x = np.round(rng.normal(1000, 30, size=(3, n)))
        x[:, n // 2: n // 2 + 3] += 400
        check(x.astype(np.float32), w, L, 3.0, "ragged-%d" % n, detect_seg=seg)
    # constant rows: every filtered series constant, MAD_w 0, no candidates
    x = np.full((2, 5000), 777.0, dtype=np.float32)
    x[1] = np.round(rng.normal(0, 5, size=5000))
    check(x, 64, 512, 2.0, "constant")
    # a ramp and uniform noise over +-4e6: wide series, three selection levels
    t = np.arange(20000, dtype=np.float64)
    x = np.stack([np.round(2000.0 * (t % 7000)), np.round(rng.uniform(-4e6, 4e6, size=t.size))]).astype(np.float32)
    check(x, 64, 900, 2.5, "ramp-wide")
    # samples at the domain bound for the widest width (boxcar sums near +-2^31)
    b = sps().domain_bound(256)
    x = rng.choice(np.array([-b, b], dtype=np.float64), size=(2, 6000)).astype(np.float32)
    check(x, 256, 50, 1.0, "domain-bound")
    # heavy ties and steps
    x = rng.integers(0, 3, size=(2, 9000)).astype(np.float32)
    x[1, 3000:] += 20000
    x[1, 6000:] -= 45000
    check(x, 128, 1000, 1.5, "ties-steps")


def test_width_norm_batch_equals_alone_and_oracle():
    import torch
    m = sps()
    shapes = [(7, 3000, 64, 700, 5.0), (3, 65, 1, 1, 4.0), (5, 9000, 256, 16384, 4.5), (12, 20000, 1024, 3000, 6.0)]
    blocks = [synth.Block(ndm=nd, nsamp=n, max_width=w, baseline_len=L, snr_thresh=th, seed=950 + k, n_pulses=4,
                          pulse_width=(1, max(1, min(w, 256))), pulse_snr=(6.0, 25.0))
              for k, (nd, n, w, L, th) in enumerate(shapes)]
    xs_h = [synth.generate(b) for b in blocks]
    print("width-norm batch of %d items" % len(blocks), flush=True)
    with m.Batch() as b:
        b.set(m.ATTR_NORM, 2)
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
            alone, _, _ = run(x, blk.max_width, blk.baseline_len, blk.snr_thresh)
            assert exact_equal(got, alone), "item %d" % k
            a = np.empty(got.size, dtype=oracle.CAND_DTYPE)
            for f in ("sample", "dm_idx", "width", "snr"):
                a[f] = got[f]
            ref = oracle.search(x, blk.max_width, blk.baseline_len, blk.snr_thresh, width_norm=True)
            assert exact_equal(oracle.sort_cands(a), ref), "item %d" % k
            total += ref.size
        assert total > 0


def test_width_norm_attribute_rules():
    import torch
    m = sps()
    with m.Plan(2, 4096, 64, 1000, 5.0) as p:
        p.set(m.ATTR_NORM, 2)
        with pytest.raises(m.SpsError):
            m.Stream(p)  # a stream never sees the whole filtered series
        x = torch.zeros((2, 4096), dtype=torch.float32, device="cuda")
        cands, ncand = p.alloc_cands()
        with pytest.raises(m.SpsError):
            p.search(x, cands, ncand, plain=True)  # the per-stage path keeps block or row scales only
        p.search(x, cands, ncand)
        torch.cuda.synchronize()
        assert int(ncand.item()) == 0


def test_width_norm_full_size_sampled_rows():
    # the 1024 x 2^20 block in the launch configuration the benchmark times
    # (bench.py --norm width); the oracle checks sampled rows
    import torch
    m = sps()
    cfg = synth.config(2)["blocks"][0]
    print("case c2 full size width_norm: generate", flush=True)
    x = synth.generate(cfg)
    xd = torch.from_numpy(x).cuda()
    rows = [0, 511, 1023]
    with m.Plan(cfg.ndm, cfg.nsamp, cfg.max_width, cfg.baseline_len, cfg.snr_thresh) as p:
        p.set(m.ATTR_NORM, 2)
        cands, ncand = p.alloc_cands()
        p.search(xd, cands, ncand)
        c, d = p.width_stats(xd)
        torch.cuda.synchronize()
        got = m.cands_to_numpy(cands, ncand, p.max_cands)
        c, d = c.cpu().numpy(), d.cpu().numpy()
    print("case c2 width_norm: oracle on rows %s (%d gpu candidates)" % (rows, got.size), flush=True)
    rc, rd = oracle_width_stats(x[rows], cfg.max_width, cfg.baseline_len)
    assert np.array_equal(c[rows], rc) and np.array_equal(d[rows], rd)
    ref = oracle.search(x, cfg.max_width, cfg.baseline_len, cfg.snr_thresh, rows=rows, width_norm=True)
    sel = np.isin(got["dm_idx"], rows)
    assert compare_cands(got[sel], ref, cfg.snr_thresh, "c2-widthnorm-rows") == 0
    assert exact_equal(got[sel], ref)
