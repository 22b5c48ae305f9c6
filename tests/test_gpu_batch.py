"""GPU batch: many blocks in one persistent launch per stage.

Every item of a batch must give exactly what the oracle gives for that block
alone, and what a single-block search gives; tuning, reuse of the context and
the order of items must not change anything.
"""
import numpy as np
import pytest

import oracle
import synth
from parity import compare_cands, exact_equal

pytestmark = pytest.mark.gpu


def sps():
    from paper_2512_00398_amd import sps as m
    return m


def run_batch(blocks, xs, tune=None, batch=None, order=None):
    import torch
    m = sps()
    own = batch is None
    b = m.Batch() if own else batch
    for attr, v in (tune or {}).items():
        b.set(attr, v)
    outs = []
    items = []
    for blk, x in zip(blocks, xs):
        cands = torch.empty((1 << 20, 4), dtype=torch.int32, device="cuda")
        ncand = torch.full((1,), 12345, dtype=torch.int32, device="cuda")
        outs.append((cands, ncand))
        items.append((x, blk.max_width, blk.baseline_len, blk.snr_thresh, cands, ncand))
    idx = list(range(len(items))) if order is None else order
    print("batch of %d items %s tune=%s" % (len(items), [tuple(x.shape) for x in xs], tune), flush=True)
    b.search([items[i] for i in idx])
    torch.cuda.synchronize()
    res = [m.cands_to_numpy(c, n) for c, n in outs]
    if own:
        b.close()
    return res


def as_oracle(c):
    a = np.empty(c.size, dtype=oracle.CAND_DTYPE)
    a["sample"], a["dm_idx"], a["width"], a["snr"] = c["sample"], c["dm_idx"], c["width"], c["snr"]
    return oracle.sort_cands(a)


def mixed_blocks():
    shapes = [(7, 3000, 64, 700, 5.0), (16, 16384, 4096, 4096, 5.5), (3, 65, 1, 1, 4.0),
              (5, 9000, 256, 16384, 4.5), (1, 4096, 4096, 100, 5.0), (12, 20000, 1024, 3000, 6.0)]
    out = []
    for k, (ndm, n, w, L, th) in enumerate(shapes):
        out.append(synth.Block(ndm=ndm, nsamp=n, max_width=w, baseline_len=L, snr_thresh=th, seed=500 + k,
                               n_pulses=4, pulse_width=(1, max(1, min(w, 256))), pulse_snr=(6.0, 25.0)))
    return out


def test_batch_equals_oracle_per_item():
    import torch
    blocks = mixed_blocks()
    xs_h = [synth.generate(b) for b in blocks]
    xs = [torch.from_numpy(x).cuda() for x in xs_h]
    got = run_batch(blocks, xs)
    total = 0
    for k, (b, x) in enumerate(zip(blocks, xs_h)):
        ref = oracle.search(x, b.max_width, b.baseline_len, b.snr_thresh)
        g = as_oracle(got[k])
        assert compare_cands(g, ref, b.snr_thresh, "item %d" % k) == 0
        assert exact_equal(g, ref), "item %d" % k
        total += ref.size
    assert total > 0


def test_batch_tilings_order_and_reuse():
    import torch
    m = sps()
    blocks = mixed_blocks()
    xs = [torch.from_numpy(synth.generate(b)).cuda() for b in blocks]
    base = run_batch(blocks, xs)
    # multi-segment rows (fix-up path), short chains, wide histogram
    for tune in ({m.ATTR_DETECT_SEG: 1024, m.ATTR_STATS_SEG: 64}, {m.ATTR_DETECT_SEG: 4096},
                 {m.ATTR_HIST_BINS: 16384, m.ATTR_STATS_SEG: 1}):
        got = run_batch(blocks, xs, tune=tune)
        for k in range(len(blocks)):
            assert exact_equal(as_oracle(got[k]), as_oracle(base[k])), (tune, k)
    # reversed order, and one context reused for a large then a smaller batch
    got = run_batch(blocks, xs, order=list(reversed(range(len(blocks)))))
    for k in range(len(blocks)):
        assert exact_equal(as_oracle(got[k]), as_oracle(base[k])), ("reversed", k)
    with m.Batch() as ctx:
        run_batch(blocks, xs, batch=ctx)
        got = run_batch(blocks[:3], xs[:3], batch=ctx)
        for k in range(3):
            assert exact_equal(as_oracle(got[k]), as_oracle(base[k])), ("reuse", k)
    # a single-block search gives the same
    for k, (b, x) in enumerate(zip(blocks, xs)):
        with m.Plan(b.ndm, b.nsamp, b.max_width, b.baseline_len, b.snr_thresh) as p:
            c, n = p.alloc_cands(1 << 20)
            p.search(x, c, n)
            torch.cuda.synchronize()
            assert exact_equal(as_oracle(m.cands_to_numpy(c, n)), as_oracle(base[k])), ("alone", k)


def test_batch_invalid_item_rejected_nothing_enqueued():
    import torch
    m = sps()
    x = torch.zeros((2, 128), dtype=torch.float32, device="cuda")
    c = torch.empty((16, 4), dtype=torch.int32, device="cuda")
    n = torch.full((1,), 77, dtype=torch.int32, device="cuda")
    with m.Batch() as b:
        for bad in ((x, 3, 10, 5.0, c, n), (x, 4, 0, 5.0, c, n), (x, 4, 10, 0.0, c, n), (x, 8192, 10, 5.0, c, n)):
            with pytest.raises(m.SpsError):
                b.search([(x, 4, 10, 5.0, c, n), bad])
        torch.cuda.synchronize()
        assert int(n.item()) == 77
        b.search([])


def test_batch_workload_files_sampled():
    # Files of the many-file workload (full shapes: up to 2048 x 2^20 samples,
    # widths 1..4096, window 16384), batched; every file equals its
    # single-block search, and sampled rows equal the oracle.
    import torch
    m = sps()
    cfg = synth.config(4)
    pick = [0, 5, 11, 17, 23, 29]
    blocks = [cfg["blocks"][i] for i in pick]
    xs = [torch.from_numpy(synth.generate(b)).cuda() for b in blocks]
    items, outs = [], []
    for b, x in zip(blocks, xs):
        cands = torch.empty((1 << 24, 4), dtype=torch.int32, device="cuda")
        ncand = torch.zeros((1,), dtype=torch.int32, device="cuda")
        outs.append((cands, ncand))
        items.append((x, b.max_width, b.baseline_len, b.snr_thresh, cands, ncand))
    print("workload batch", [(b.ndm, b.nsamp) for b in blocks], flush=True)
    with m.Batch() as ctx:
        ctx.search(items)
        torch.cuda.synchronize()
    for k, (b, x) in enumerate(zip(blocks, xs)):
        got = as_oracle(m.cands_to_numpy(*outs[k]))
        with m.Plan(b.ndm, b.nsamp, b.max_width, b.baseline_len, b.snr_thresh) as p:
            c, n = p.alloc_cands()
            p.search(x, c, n)
            torch.cuda.synchronize()
            assert exact_equal(got, as_oracle(m.cands_to_numpy(c, n))), ("alone", k)
        rows = [0, b.ndm - 1]
        xr = synth.generate(b, rows=rows)
        for j, r in enumerate(rows):
            ref = oracle.search(xr[j:j + 1], b.max_width, b.baseline_len, b.snr_thresh)
            ref["dm_idx"] = r
            sel = got[got["dm_idx"] == r]
            assert compare_cands(sel, ref, b.snr_thresh, "file %d row %d" % (pick[k], r)) == 0
            assert exact_equal(sel, ref), (k, r)


def test_fused_launch_equals_per_stage_launches_and_oracle():
    # SPS_ATTR_FUSED = 1 (the default) runs the statistics chains and the
    # detection tasks in one persistent launch, each task waiting for its
    # row's chains; 0 runs one launch per stage. Both give each block's own
    # result, also with the centred window, more chains than resident waves,
    # and settings that fall back to per-stage launches (16384 bins).
    import torch
    m = sps()
    blocks = mixed_blocks()
    xs = [torch.from_numpy(synth.generate(b)).cuda() for b in blocks]
    refs = [oracle.search(x.cpu().numpy(), b.max_width, b.baseline_len, b.snr_thresh) for b, x in zip(blocks, xs)]
    for tune in ({m.ATTR_FUSED: 1}, {m.ATTR_FUSED: 0}, {m.ATTR_FUSED: 1, m.ATTR_STATS_SEG: 64},
                 {m.ATTR_FUSED: 1, m.ATTR_HIST_BINS: 16384}, {m.ATTR_FUSED: 1, m.ATTR_DETECT_SEG: 1024}):
        got = run_batch(blocks, xs, tune=tune)
        for k, (g, r) in enumerate(zip(got, refs)):
            assert exact_equal(as_oracle(g), r), (tune, k)
    # slow chains: rows too spread for the histogram take the exact select
    # block by block, so their detection tasks wait far longer than the rest
    rng = np.random.default_rng(77)
    spread = np.round(rng.uniform(-4e6, 4e6, size=(6, 9000))).astype(np.float32)
    spread[:, 4000:4003] += 8e6
    sb = synth.Block(ndm=6, nsamp=9000, max_width=64, baseline_len=3000, snr_thresh=1.5, seed=1)
    sref = oracle.search(spread, 64, 3000, 1.5)
    for fused in (1, 0):
        got = run_batch(blocks + [sb], xs + [torch.from_numpy(spread).cuda()], tune={m.ATTR_FUSED: fused})
        assert exact_equal(as_oracle(got[-1]), sref), ("spread", fused)
        for k, (g, r) in enumerate(zip(got[:-1], refs)):
            assert exact_equal(as_oracle(g), r), ("with spread", fused, k)
    assert sref.size > 0
    for fused in (1, 0):
        got = run_batch(blocks, xs, tune={m.ATTR_FUSED: fused, m.ATTR_WINDOW: 1})
        for k, (g, b, x) in enumerate(zip(got, blocks, xs)):
            ref = oracle.search(x.cpu().numpy(), b.max_width, b.baseline_len, b.snr_thresh, centered=True)
            assert exact_equal(as_oracle(g), ref), ("centred", fused, k)
    with pytest.raises(m.SpsError):
        with m.Batch() as b:
            b.set(m.ATTR_FUSED, 2)


def test_fused_equals_per_stage_on_random_batches():
    # Seeded random batches of uneven blocks (rows, lengths, widths, windows,
    # thresholds, chain and segment lengths): the one-launch form must give
    # bit-identical results to one launch per stage, and small items the
    # oracle's.
    import torch
    m = sps()
    rng = np.random.default_rng(2026)
    checked = 0
    for trial in range(8):
        nitems = int(rng.integers(1, 7))
        blocks = []
        for k in range(nitems):
            w = 1 << int(rng.integers(0, 13))
            n = int(rng.integers(64, 40000))
            blocks.append(synth.Block(ndm=int(rng.integers(1, 12)), nsamp=n, max_width=w,
                                      baseline_len=int(rng.integers(1, 20000)), snr_thresh=float(rng.uniform(3.0, 6.0)),
                                      seed=3000 + 10 * trial + k, n_pulses=3, pulse_width=(1, max(1, min(w, 128))),
                                      pulse_snr=(6.0, 20.0)))
        xs = [torch.from_numpy(synth.generate(b)).cuda() for b in blocks]
        tune = {}
        if rng.random() < 0.5:
            tune[m.ATTR_STATS_SEG] = int(rng.choice([1, 16, 64, 500]))
        if rng.random() < 0.5:
            tune[m.ATTR_DETECT_SEG] = int(rng.choice([1024, 3072, 8192]))
        if rng.random() < 0.3:
            tune[m.ATTR_WINDOW] = 1
        print("random batch %d: %d items %s tune=%s" % (trial, nitems, [(b.ndm, b.nsamp, b.max_width) for b in blocks],
                                                      tune), flush=True)
        fused = run_batch(blocks, xs, tune={**tune, m.ATTR_FUSED: 1})
        staged = run_batch(blocks, xs, tune={**tune, m.ATTR_FUSED: 0})
        for k in range(nitems):
            assert exact_equal(as_oracle(fused[k]), as_oracle(staged[k])), (trial, k)
            b = blocks[k]
            if b.ndm * b.nsamp <= 60000:
                ref = oracle.search(xs[k].cpu().numpy(), b.max_width, b.baseline_len, b.snr_thresh,
                                    centered=tune.get(m.ATTR_WINDOW, 0) == 1)
                assert exact_equal(as_oracle(fused[k]), ref), (trial, k)
                checked += 1
    assert checked > 0
