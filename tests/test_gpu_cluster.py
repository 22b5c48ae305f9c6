"""GPU parity of candidate clustering against the CPU oracle (exact)."""
import numpy as np
import pytest

import synth
from oracle import CAND_DTYPE
from oracle import cluster_oracle as co

pytestmark = pytest.mark.gpu

FIELDS = ("sample", "dm_idx", "width", "snr", "members", "sample_lo", "sample_hi", "dm_lo", "dm_hi")


def _sps():
    from paper_2512_00398_amd import sps
    return sps


def _random_cands(rng, n, t_lo, t_span, ndm, nw, ties=False):
    s = rng.integers(t_lo, t_lo + t_span, size=4 * n)
    d = rng.integers(0, ndm, size=4 * n)
    w = 1 << rng.integers(0, nw, size=4 * n)
    key = np.stack([s, d, w], 1)
    _, first = np.unique(key, axis=0, return_index=True)
    first = np.sort(first)[:n]
    c = np.empty(first.size, dtype=CAND_DTYPE)
    c["sample"], c["dm_idx"], c["width"] = s[first], d[first], w[first]
    c["snr"] = (rng.integers(6, 9, size=first.size) if ties else rng.uniform(6, 40, size=first.size)).astype(np.float32)
    return c[rng.permutation(c.size)]


def gpu_cluster(c, tt, dt, wt):
    import torch
    sps = _sps()
    rec = np.zeros((max(1, c.size), 4), dtype=np.int32)
    if c.size:
        rec[:c.size, 0] = c["sample"].astype(np.int32)
        rec[:c.size, 1] = c["dm_idx"].astype(np.uint32).view(np.int32)
        rec[:c.size, 2] = c["width"].astype(np.uint32).view(np.int32)
        rec[:c.size, 3] = c["snr"].astype(np.float32).view(np.int32)
    d = torch.from_numpy(rec).cuda()
    with sps.Clusterer(max(1, c.size)) as k:
        out, nout = k.alloc_out(max(1, c.size))
        k.run(d, c.size, tt, dt, wt, out, nout)
        torch.cuda.synchronize()
        return sps.clusters_to_numpy(out, nout)


def check(c, tt, dt, wt, what):
    print("case %s n=%d tol=(%d,%d,%d)" % (what, c.size, tt, dt, wt), flush=True)
    got = gpu_cluster(c, tt, dt, wt)
    ref = co.cluster(c, tt, dt, wt)
    assert got.size == ref.size, what
    for f in FIELDS:
        assert np.array_equal(got[f].astype(np.int64) if f != "snr" else got[f], ref[f].astype(np.int64) if f != "snr" else ref[f]), (what, f)
    return got


@pytest.mark.parametrize("seed", range(6))
def test_random_sets_match_oracle(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(50, 20000))
    c = _random_cands(rng, n, int(rng.integers(-5000, 5000)), int(rng.integers(100, 200000)), 300, 13, ties=bool(seed % 2))
    tt, dt, wt = int(rng.integers(0, 40)), int(rng.integers(0, 8)), int(rng.integers(0, 4))
    check(c, tt, dt, wt, "random-%d" % seed)


def test_edge_cases():
    rng = np.random.default_rng(7)
    check(np.empty(0, dtype=CAND_DTYPE), 3, 3, 3, "empty")
    check(_random_cands(rng, 1, 0, 10, 5, 3), 3, 3, 3, "one")
    c = _random_cands(rng, 3000, 12345, 1, 400, 13)  # one sample for all
    check(c, 0, 1, 0, "same-sample")
    check(c, 0, 1000, 20, "same-sample-one-cluster")
    c = _random_cands(rng, 5000, -2 ** 31 + 10, 2 ** 32 - 100, 50, 4)  # whole int32 range: wide cells
    check(c, 5, 3, 1, "int32-range")
    c = _random_cands(rng, 4000, 0, 100000, 100, 13, ties=True)
    check(c, 1 << 30, 1 << 20, 31, "unbounded")
    c = _random_cands(rng, 6000, -7, 3000, (1 << 27) - 1, 13)  # DM range beyond the cell table: wide DM cells
    c["dm_idx"][::7] = c["dm_idx"][::7] % 64  # and a dense corner that links
    c = c[np.unique(np.stack([c["sample"], c["dm_idx"], c["width"]], 1), axis=0, return_index=True)[1]]
    check(c, 9, 5, 1, "dm-range")


def test_search_output_small_config():
    import torch
    sps = _sps()
    b = synth.config(1)["blocks"][0]
    x = torch.from_numpy(synth.generate(b)).cuda()
    got = sps.search(x, b.max_width, b.baseline_len, b.snr_thresh)
    c = np.empty(got.size, dtype=CAND_DTYPE)
    for f in ("sample", "dm_idx", "width", "snr"):
        c[f] = got[f]
    for tols in ((0, 0, 0), (16, 2, 1), (64, 4, 2), (1024, 64, 6)):
        check(c, *tols, "c1 search")


def test_search_output_large_block_rows():
    # candidates of the 1024 x 2^20 block (drift flood), the first 104 DM rows
    # (about a million candidates in large friends-of-friends components)
    import torch
    sps = _sps()
    b = synth.config(2)["blocks"][0]
    rows = 104
    x = torch.from_numpy(synth.generate(b, rows=range(rows))).cuda()
    got = sps.search(x, b.max_width, b.baseline_len, b.snr_thresh)
    c = np.empty(got.size, dtype=CAND_DTYPE)
    for f in ("sample", "dm_idx", "width", "snr"):
        c[f] = got[f]
    assert c.size > 500000
    check(c, 32, 3, 2, "c2 rows")


def test_clusterer_rejects_bad_arguments():
    import torch
    sps = _sps()
    with sps.Clusterer(100) as k:
        cands = torch.zeros((200, 4), dtype=torch.int32, device="cuda")
        out, nout = k.alloc_out(200)
        with pytest.raises(sps.SpsError):
            k.run(cands, 150, 1, 1, 1, out, nout)  # beyond the context's capacity
        with pytest.raises(sps.SpsError):
            k.run(cands, 10, -1, 1, 1, out, nout)
