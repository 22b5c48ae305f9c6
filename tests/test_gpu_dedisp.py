"""GPU parity of incoherent dedispersion against the oracle (exact integer sums)."""
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import dedisp_oracle as dd
from synth import filterbank as fb
from parity import exact_equal

pytestmark = pytest.mark.gpu


def sps():
    from paper_2512_00398_amd import sps as m
    return m


def gpu_dedisperse(fil, tab):
    import torch
    m = sps()
    nchan, nin = fil.shape
    with m.Dedisperser(nchan, nin, tab) as k:
        out = k.run(torch.from_numpy(np.ascontiguousarray(fil)).cuda())
        torch.cuda.synchronize()
        return out.cpu().numpy()


def check(fil, tab, where):
    print("dedisp case %s nchan=%d nsamp_in=%d ndm=%d max delay=%d" % (where, fil.shape[0], fil.shape[1], tab.shape[0],
                                                                     int(tab.max())), flush=True)
    sys.stdout.flush()
    got = gpu_dedisperse(fil, tab)
    ref = dd.dedisperse(fil, tab)
    assert got.shape == ref.shape, where
    assert np.array_equal(got.astype(np.int64), ref), "%s: differs at %s" % (where, np.argwhere(got != ref)[:5])
    return got


def test_small_band_parity():
    f, fref = fb.band(64)
    dms = np.linspace(0, 400, 40).astype(np.float32)
    tab = dd.delays(f, fref, 1e-4, dms)
    fil = fb.filterbank(64, 6000 + int(tab.max()), seed=3, pulses=[(700, 4, 30), (2500, 1, 90)], tracks=tab[[11, 30]])
    check(fil, tab, "band-64")


def test_ragged_shapes_and_flushes():
    rng = np.random.default_rng(5)
    # odd byte counts (partial last word), channels past a 256-channel flush,
    # trials not a multiple of the group, output rows not a multiple of 4 or 1024
    for nchan, nin, ndm in [(1, 1, 1), (3, 9, 2), (300, 4999, 37), (600, 2051, 17), (257, 1030, 16)]:
        maxd = max(0, nin // 3)
        tab = np.sort(rng.integers(0, maxd + 1, size=(ndm, nchan)), axis=0)
        fil = rng.integers(0, 256, size=(nchan, nin)).astype(np.uint8)
        check(fil, tab, "ragged-%d-%d-%d" % (nchan, nin, ndm))
    # every byte 255: the 16-bit pair sums reach their largest value before each flush
    fil = np.full((700, 3000), 255, dtype=np.uint8)
    tab = np.sort(rng.integers(0, 500, size=(20, 700)), axis=0)
    got = check(fil, tab, "saturated")
    assert np.all(got == 255 * 700)


def test_wide_spread_uses_smaller_trial_groups():
    # delays of neighbouring trials far apart: the library groups fewer trials per workgroup
    rng = np.random.default_rng(6)
    nchan, nin, ndm = 48, 70000, 21
    tab = np.zeros((ndm, nchan), dtype=np.int64)
    tab[:, :] = (np.arange(ndm) * 3000)[:, None] + rng.integers(0, 50, size=(ndm, nchan))
    fil = rng.integers(0, 256, size=(nchan, nin)).astype(np.uint8)
    check(fil, tab, "wide-spread")


@pytest.mark.parametrize("spread", [0, 1, 700, 1526, 3000, 7157, 7158, 7159])
def test_trial_group_spread_edges(spread):
    # The spread of the delays of 16 neighbouring trials in a channel decides
    # the trials per workgroup: 16 up to 7158 samples (at 7158 the largest
    # staged span, 2048 words), then fewer. Channels are offset from one
    # another and the rows have an odd length, so the spans start at every
    # byte alignment.
    rng = np.random.default_rng(spread + 11)
    nchan, ndm = 6, 37
    ramp = np.round(np.linspace(0, spread, 16)).astype(np.int64)
    tab = np.zeros((ndm, nchan), dtype=np.int64)
    for f in range(nchan):
        tab[:, f] = ramp[np.arange(ndm) % 16] + 3 * f + (np.arange(ndm) // 16)
    nin = 2 * 1024 + 500 + int(tab.max())
    nin += 1 - nin % 2
    fil = rng.integers(0, 256, size=(nchan, nin)).astype(np.uint8)
    check(fil, tab, "spread-%d" % spread)


def test_dedispersed_pulse_found_by_search():
    # producer and consumer on the device: a dispersed pulse comes back at its
    # DM and time through sps_search, as the oracle finds it
    import torch
    m = sps()
    nchan, ndm = 128, 64
    f, fref = fb.band(nchan)
    dms = np.linspace(0, 600, ndm).astype(np.float32)
    tsamp = 98.304e-6
    tab = m.dedisp_delays(f, fref, tsamp, dms)
    assert np.array_equal(tab.astype(np.int64), dd.delays(f, fref, tsamp, dms))
    k_dm, t0, w = 41, 9000, 8
    nin = 40000 + int(tab.max())
    fil = fb.filterbank(nchan, nin, seed=9, pulses=[(t0, w, 12)], tracks=tab[[k_dm]])
    with m.Dedisperser(nchan, nin, tab) as k:
        x = k.run(torch.from_numpy(fil).cuda())
        with m.Plan(ndm, k.nsamp_out, 64, 4096, 8.0) as p:
            cands, ncand = p.alloc_cands()
            p.search(x, cands, ncand)
            torch.cuda.synchronize()
            got = m.cands_to_numpy(cands, ncand, p.max_cands)
        xs = x.cpu().numpy()
    ref_x = dd.dedisperse(fil, tab.astype(np.int64))
    assert np.array_equal(xs.astype(np.int64), ref_x)
    ref = oracle.search(ref_x.astype(np.float32), 64, 4096, 8.0)
    assert exact_equal(got, ref)
    best = ref[np.argmax(ref["snr"])]
    assert best["dm_idx"] == k_dm and abs(int(best["sample"]) - t0) <= w and best["width"] == w


def test_full_size_sampled_rows():
    # the benchmark's workload: 1024 channels over 1050-1450 MHz, 49.152 us,
    # 1024 trials over DM 0-1000, 2^18 output samples; the oracle checks sampled rows
    import torch
    m = sps()
    nchan, ndm, nout = 1024, 1024, 1 << 18
    f, fref = fb.band(nchan)
    dms = np.linspace(0, 1000, ndm).astype(np.float32)
    tab = m.dedisp_delays(f, fref, 49.152e-6, dms)
    nin = nout + int(tab.max())
    print("dedisp full size: generate %d x %d" % (nchan, nin), flush=True)
    fil = fb.filterbank(nchan, nin, seed=12, pulses=[(50000, 16, 20), (200000, 2, 60)], tracks=tab[[300, 900]])
    with m.Dedisperser(nchan, nin, tab) as k:
        assert k.nsamp_out == nout
        out = k.run(torch.from_numpy(fil).cuda())
        torch.cuda.synchronize()
        rows = [0, 300, 777, 1023]
        got = out[rows].cpu().numpy()
    ref = dd.dedisperse(fil, tab[rows].astype(np.int64))
    assert np.array_equal(got.astype(np.int64), ref[:, :nout])
