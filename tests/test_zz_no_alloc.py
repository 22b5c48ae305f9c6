"""The allocation-free search (sps_search_noalloc) against the plan-based
search (sps_search) through the C ABI: the same candidates, on two calls in a
row with the second input smaller, and on a block whose run summaries do not
fit the fixed scratch (one detection segment per row). Blocks too large for
the scratch are refused before any device work."""
import numpy as np
import pytest

import oracle
import synth
from parity import compare_cands, exact_equal


def _sps():
    from paper_2512_00398_amd import sps
    return sps


def test_noalloc_refuses_blocks_beyond_the_scratch_without_device():
    sps = _sps()
    lib = sps.load()
    # 513 rows of 2^20 samples need 2 x 513 x 16384 x 4 bytes of medians and MADs (> 64 MiB)
    rc = lib.sps_search_noalloc(513, 1 << 20, 4096, 16384, 6.0, 1, None, 1, 1, 16)
    assert rc == sps.SPS_ERR_SCRATCH
    assert lib.sps_last_error() == sps.SPS_ERR_SCRATCH
    assert "scratch" in sps.error_string(sps.SPS_ERR_SCRATCH)
    # invalid shapes and pointers are argument errors, checked first
    assert lib.sps_search_noalloc(0, 1024, 64, 100, 6.0, 1, None, 1, 1, 16) == sps.SPS_ERR_INVALID_ARG
    assert lib.sps_search_noalloc(4, 1024, 64, 100, 6.0, None, None, 1, 1, 16) == sps.SPS_ERR_INVALID_ARG
    assert lib.sps_search_noalloc(4, 1024, 64, 100, 6.0, 1, None, None, 1, 16) == sps.SPS_ERR_INVALID_ARG
    assert lib.sps_search_noalloc(4, 1024, 64, 100, 6.0, 1, None, 1, 1, -1) == sps.SPS_ERR_INVALID_ARG


def _plan_search(xd, max_width, L, theta, cap):
    import torch
    sps = _sps()
    ndm, n = xd.shape
    with sps.Plan(ndm, n, max_width, L, theta) as p:
        p.set(sps.ATTR_MAX_CANDS, cap)
        cands, ncand = p.alloc_cands()
        p.search(xd, cands, ncand)
        torch.cuda.synchronize()
        return sps.cands_to_numpy(cands, ncand, cap)


def _noalloc_search(xd, max_width, L, theta, cands, ncand):
    import torch
    sps = _sps()
    sps.search_noalloc(xd, max_width, L, theta, cands, ncand)
    torch.cuda.synchronize()
    return sps.cands_to_numpy(cands, ncand, cands.shape[0])


@pytest.mark.gpu
def test_noalloc_equals_plan_search_twice_second_smaller():
    import torch
    cap = 1 << 20
    # one candidate buffer for both calls: the second call's results replace the first's
    cands = torch.empty((cap, 4), dtype=torch.int32, device="cuda")
    ncand = torch.zeros((1,), dtype=torch.int32, device="cuda")
    cases = [
        ("small configuration 64 x 16384", synth.config(1)["blocks"][0]),
        ("ragged 12 x 9001", synth.Block(ndm=12, nsamp=9001, max_width=256, baseline_len=2500, seed=515,
                                         n_pulses=6, pulse_width=(1, 128), pulse_snr=(6.0, 30.0))),
    ]
    for where, b in cases:
        print("case noalloc %s w=%d L=%d" % (where, b.max_width, b.baseline_len), flush=True)
        x = synth.generate(b)
        xd = torch.from_numpy(x).cuda()
        got = _noalloc_search(xd, b.max_width, b.baseline_len, b.snr_thresh, cands, ncand)
        ref = _plan_search(xd, b.max_width, b.baseline_len, b.snr_thresh, cap)
        assert exact_equal(got, ref), where
        # and both against the oracle, to the parity rule
        compare_cands(got, oracle.search(x, b.max_width, b.baseline_len, b.snr_thresh), b.snr_thresh, where)


@pytest.mark.gpu
def test_noalloc_whole_row_segments_when_summaries_do_not_fit():
    import torch
    # 512 x 2^20: medians and MADs take the whole 64 MiB, so each row is
    # detected in one segment (the plan splits rows into several)
    ndm, n = 512, 1 << 20
    g = torch.Generator(device="cuda")
    g.manual_seed(20251207)
    print("case noalloc 512 x 2^20 (whole-row segments)", flush=True)
    t = torch.arange(n, device="cuda", dtype=torch.float32)
    drift = torch.round(2048.0 * torch.sin(2.0 * np.pi * t / 8192.0))
    xd = torch.round(torch.randn((ndm, n), generator=g, device="cuda") * 1024.0 + 32768.0) + drift
    del t, drift
    cap = 1 << 24
    cands = torch.empty((cap, 4), dtype=torch.int32, device="cuda")
    ncand = torch.zeros((1,), dtype=torch.int32, device="cuda")
    got = _noalloc_search(xd, 4096, 16384, 6.0, cands, ncand)
    del cands, ncand
    ref = _plan_search(xd, 4096, 16384, 6.0, cap)
    print("candidates %d" % got.size, flush=True)
    assert got.size > 0
    assert exact_equal(got, ref)
