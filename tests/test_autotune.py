"""Autotuner host logic (CPU) and, on the GPU, that tuning leaves results unchanged."""
import numpy as np
import pytest

from paper_2512_00398_amd import autotune


def test_shape_key_classes():
    a = autotune.shape_key("gfx950", 1000, 1000000, 4096, 16384)
    assert a == autotune.shape_key("gfx950", 1024, 1 << 20, 4096, 16384) == "gfx950|ndm1024|n1048576|w4096|L16384"
    assert a != autotune.shape_key("gfx950", 1025, 1 << 20, 4096, 16384)
    assert a != autotune.shape_key("gfx942", 1024, 1 << 20, 4096, 16384)


def test_candidate_configs_in_range():
    c = autotune.candidate_configs(1024, 1 << 20, 4096, 16384)
    assert c["stats_seg"][0] == 0 and c["detect_seg"][0] == 0
    assert all(s % 1024 == 0 and s >= 4 * 4096 for s in c["detect_seg"][1:])
    assert all(0 < s < (1 << 20) // 64 for s in c["stats_seg"][1:])
    assert sorted(c["hist_bins"]) == [4096, 16384]
    small = autotune.candidate_configs(4, 1000, 64, 100)
    assert small["detect_seg"] == [0]


def test_digest_is_order_independent_and_sensitive():
    rng = np.random.default_rng(1)
    a = rng.integers(0, 1 << 31, size=(1000, 4), dtype=np.int64).astype(np.int32)
    d = autotune.digest(a)
    assert d == autotune.digest(a[rng.permutation(1000)])
    b = a.copy()
    b[17, 3] ^= 1
    assert d != autotune.digest(b)
    c = a.copy()
    c[[3, 4], 0] = c[[4, 3], 0]  # swap one field between two records
    assert d != autotune.digest(c)
    assert autotune.digest(a[:0]) == 0


def test_cache_roundtrip(tmp_path):
    p = str(tmp_path / "sub" / "t.json")
    assert autotune.load_cache(p) == {}
    key = autotune.shape_key("gfx950", 64, 16384, 64, 4096)
    autotune.save_cache({key: {"config": {"stats_seg": 256, "detect_seg": 0, "hist_bins": 4096}}}, p)
    assert autotune.lookup(64, 16384, 64, 4096, "gfx950", p) == {"stats_seg": 256, "detect_seg": 0,
                                                                 "hist_bins": 4096}
    assert autotune.lookup(64, 16384, 64, 4096, "gfx942", p) is None
    autotune.save_cache({key: {"config": {"bogus": 1}}}, p)
    with pytest.raises(ValueError):
        autotune.lookup(64, 16384, 64, 4096, "gfx950", p)


@pytest.mark.gpu
def test_tuned_plan_gives_oracle_result(tmp_path):
    import torch
    import oracle
    import synth
    from parity import exact_equal
    from paper_2512_00398_amd import sps
    b = synth.Block(ndm=48, nsamp=1 << 17, max_width=1024, baseline_len=4096, snr_thresh=5.5, seed=4242,
                    n_pulses=8, pulse_width=(1, 512), pulse_snr=(6.0, 30.0))
    x = synth.generate(b)
    xd = torch.from_numpy(x).cuda()
    path = str(tmp_path / "tune.json")
    with sps.Plan(b.ndm, b.nsamp, b.max_width, b.baseline_len, b.snr_thresh) as p:
        res = autotune.tune(p, xd, steps=1, path=path)
        assert res["tried"] > 3 and res["ms"] <= res["default_ms"]
    with sps.Plan(b.ndm, b.nsamp, b.max_width, b.baseline_len, b.snr_thresh) as p:
        cfg = autotune.apply(p, path=path)
        assert cfg == res["config"]
        c, n = p.alloc_cands()
        p.search(xd, c, n)
        torch.cuda.synchronize()
        got = sps.cands_to_numpy(c, n)
    ref = oracle.search(x, b.max_width, b.baseline_len, b.snr_thresh)
    g = np.empty(got.size, dtype=oracle.CAND_DTYPE)
    g["sample"], g["dm_idx"], g["width"], g["snr"] = got["sample"], got["dm_idx"], got["width"], got["snr"]
    assert exact_equal(oracle.sort_cands(g), ref)


def test_batch_key_is_a_multiset_of_shape_classes():
    a = autotune.batch_key("gfx950", [(256, 1 << 16, 4096, 16384), (1000, 1 << 20, 4096, 16384),
                                      (256, 60000, 4096, 16384)])
    b = autotune.batch_key("gfx950", [(1024, 1 << 20, 4096, 16384), (256, 65536, 4096, 16384),
                                      (200, 65000, 4096, 16384)])
    assert a == b == "gfx950|batch|1xndm1024|n1048576|w4096|L16384;2xndm256|n65536|w4096|L16384"
    assert a != autotune.batch_key("gfx950", [(256, 1 << 16, 4096, 16384), (1000, 1 << 20, 4096, 16384)])


def test_batch_candidate_configs_fit_the_items():
    shapes = [(256, 1 << 16, 4096, 16384), (2048, 1 << 20, 4096, 16384)]
    c = autotune.batch_candidate_configs(shapes)
    assert c["stats_seg"][0] == 0 and c["detect_seg"][0] == 0
    assert all(s >= 4 * 4096 and s < (1 << 20) for s in c["detect_seg"][1:])
    assert all(s < (1 << 20) // 64 for s in c["stats_seg"][1:])
    assert sorted(c["hist_bins"]) == [4096, 16384]
    assert sorted(c["fused"]) == [0, 1]


@pytest.mark.gpu
def test_tuned_batch_keeps_every_item_result(tmp_path):
    import torch
    import oracle
    import synth
    from paper_2512_00398_amd import sps
    shapes = [(4, 30000, 1024, 3000, 6.0), (9, 9000, 256, 16384, 5.0), (2, 70000, 4096, 4096, 6.0)]
    blocks = [synth.Block(ndm=nd, nsamp=n, max_width=w, baseline_len=L, snr_thresh=th, seed=330 + k, n_pulses=4,
                          pulse_width=(1, 256), pulse_snr=(6.0, 25.0)) for k, (nd, n, w, L, th) in enumerate(shapes)]
    xs = [synth.generate(b) for b in blocks]
    items = []
    for b, x in zip(blocks, xs):
        cands = torch.empty((1 << 20, 4), dtype=torch.int32, device="cuda")
        ncand = torch.zeros((1,), dtype=torch.int32, device="cuda")
        items.append((torch.from_numpy(x).cuda(), b.max_width, b.baseline_len, b.snr_thresh, cands, ncand))
    path = str(tmp_path / "tune.json")
    print("tune batch of %d items" % len(items), flush=True)
    with sps.Batch() as bt:
        res = autotune.tune_batch(bt, items, steps=1, path=path)  # raises if any configuration changes a result
        assert res["tried"] > 1 and res["ms"] <= res["default_ms"]
        bt.search(items)
        torch.cuda.synchronize()
        for (x, w, L, th, c, n), xh in zip(items, xs):
            got = sps.cands_to_numpy(c, n)
            ref = oracle.search(xh, w, L, th)
            assert got.size == ref.size and np.array_equal(got["sample"].astype(np.int64), ref["sample"])
    with sps.Batch() as bt2:
        cfg = autotune.apply_batch(bt2, [(int(x.shape[0]), int(x.shape[1]), w, L) for (x, w, L, _, _, _) in items],
                                   path=path)
        assert cfg == res["config"]
