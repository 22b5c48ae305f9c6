"""GPU parity of broadband (zero-DM) RFI excision against the oracle (exact bytes)."""
import sys

import numpy as np
import pytest

import oracle
from oracle import dedisp_oracle as dd
from oracle import rfi_oracle as ro
from synth import filterbank as fb
from parity import exact_equal

pytestmark = pytest.mark.gpu


def sps():
    from paper_2512_00398_amd import sps as m
    return m


def run(fil, offset, in_place=False):
    import torch
    m = sps()
    x = torch.from_numpy(np.ascontiguousarray(fil)).cuda()
    out = m.zero_dm(x, offset, out=x if in_place else None)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("nchan,nsamp,offset", [(1, 1, 0), (3, 7, 255), (64, 1000, 64), (100, 1003, 30),
                                                (1000, 4096, 128), (7, 257, 1),
                                                # the read-once kernel's channels per wave (4, 16, 64) at their
                                                # limits, one 252-sample tile and its neighbours; over 1024
                                                # channels the two-pass kernel
                                                (65, 503, 10), (256, 252, 200), (257, 253, 0), (1024, 259, 64),
                                                (1025, 300, 64), (16, 251, 3), (17, 505, 255),
                                                # odd channel counts per wave and short rows of a tile or two
                                                (33, 125, 7), (129, 123, 200), (513, 130, 1), (1023, 249, 64),
                                                (48, 124, 9)])
def test_zero_dm_parity(nchan, nsamp, offset):
    print("zero-dm case nchan=%d nsamp=%d offset=%d" % (nchan, nsamp, offset), flush=True)
    sys.stdout.flush()
    rng = np.random.default_rng(nchan * 7 + nsamp)
    fil = rng.integers(0, 256, size=(nchan, nsamp)).astype(np.uint8)
    ref = ro.zero_dm(fil, offset)
    assert np.array_equal(run(fil, offset), ref)
    assert np.array_equal(run(fil, offset, in_place=True), ref)


def test_overlapping_output_rejected():
    import torch
    m = sps()
    base = torch.zeros(500, dtype=torch.uint8, device="cuda")
    x = base[:400].view(4, 100)
    with pytest.raises(m.SpsError):
        m.zero_dm(x, 0, out=base[50:450].view(4, 100))  # same size, shifted by 50 bytes: overlaps
    with pytest.raises(m.SpsError):
        m.zero_dm(x, 300)


def test_zero_dm_before_dedispersion_removes_broadband_burst():
    # an undispersed burst in every channel shows up at every trial DM; after
    # the zero-DM filter the dedispersed block has no trace of it, and the
    # dispersed pulse is still the brightest candidate
    import torch
    m = sps()
    nchan, ndm = 128, 48
    f, fref = fb.band(nchan)
    dms = np.linspace(0, 500, ndm).astype(np.float32)
    tab = m.dedisp_delays(f, fref, 98.304e-6, dms)
    nin = 30000 + int(tab.max())
    fil = fb.filterbank(nchan, nin, seed=21, pulses=[(12000, 8, 14)], tracks=tab[[30]])
    burst = fil.astype(np.int64)
    burst[:, 20000:20016] += 60  # broadband, DM 0
    fil = np.minimum(burst, 255).astype(np.uint8)
    x = torch.from_numpy(fil).cuda()
    m.zero_dm(x, 64, out=x)
    with m.Dedisperser(nchan, nin, tab) as k:
        blk = k.run(x)
        with m.Plan(ndm, k.nsamp_out, 64, 4096, 7.0) as p:
            cands, ncand = p.alloc_cands()
            p.search(blk, cands, ncand)
            torch.cuda.synchronize()
            got = m.cands_to_numpy(cands, ncand, p.max_cands)
    clean = ro.zero_dm(fil, 64)
    assert np.array_equal(x.cpu().numpy(), clean)
    ref = oracle.search(dd.dedisperse(clean, tab.astype(np.int64)).astype(np.float32), 64, 4096, 7.0)
    assert exact_equal(got, ref)
    best = ref[np.argmax(ref["snr"])]
    assert best["dm_idx"] == 30 and abs(int(best["sample"]) - 12000) <= 8
    # nothing from the burst: no candidate near the burst time at DM 0
    near = ref[(ref["dm_idx"] == 0) & (np.abs(ref["sample"].astype(np.int64) - 20000) < 64)]
    assert near.size == 0


def test_zero_dm_full_size():
    # the benchmark filterbank shape: 1024 channels x 298,529 samples
    import torch
    m = sps()
    nchan, nsamp = 1024, 298529
    print("zero-dm full size %d x %d" % (nchan, nsamp), flush=True)
    fil = fb.filterbank(nchan, nsamp, seed=31)
    fil[:, 5000:5003] = 250
    out = run(fil, 64)
    assert np.array_equal(out, ro.zero_dm(fil, 64))


def run_mask(fil, k, in_place=False):
    import torch
    m = sps()
    x = torch.from_numpy(np.ascontiguousarray(fil)).cuda()
    out, st = m.chan_mask(x, k, out=x if in_place else None)
    torch.cuda.synchronize()
    return out.cpu().numpy(), st.cpu().numpy()


@pytest.mark.parametrize("nchan,nsamp,k", [(1, 1, 0), (2, 5, 0), (64, 3000, 3), (37, 1001, 2), (300, 4096, 0),
                                           # rows of 2 and 3 bytes (one partial word each), and rows long
                                           # enough for the statistics' four-word steps with a tail
                                           (5, 2, 0), (6, 3, 1), (9, 4097 * 4 + 3, 1)])
def test_chan_mask_parity(nchan, nsamp, k):
    print("chan-mask case nchan=%d nsamp=%d k=%d" % (nchan, nsamp, k), flush=True)
    rng = np.random.default_rng(nchan + 3 * nsamp)
    fil = np.clip(np.rint(rng.normal(64, 6, size=(nchan, nsamp))), 0, 255).astype(np.uint8)
    for f in range(0, nchan, 7):  # noisy channels
        fil[f] = np.clip(np.rint(rng.normal(90, 40, size=nsamp)), 0, 255).astype(np.uint8)
    ref, mu, sg, fl = ro.channel_mask(fil, k)
    for in_place in (False, True):
        out, st = run_mask(fil, k, in_place)
        assert np.array_equal(st[:, 0], mu) and np.array_equal(st[:, 1], sg)
        assert np.array_equal(st[:, 2].astype(bool), fl)
        assert np.array_equal(out, ref)


def test_chan_mask_then_zero_dm_full_size():
    # the benchmark filterbank shape with 20 noisy channels: mask, then zero-DM, as one pre-dedispersion pass
    import torch
    m = sps()
    nchan, nsamp = 1024, 298529
    print("chan-mask full size %d x %d" % (nchan, nsamp), flush=True)
    fil = fb.filterbank(nchan, nsamp, seed=41)
    rng = np.random.default_rng(41)
    bad = rng.choice(nchan, size=20, replace=False)
    for f in bad:
        fil[f] = np.clip(np.rint(rng.normal(100, 50, size=nsamp)), 0, 255).astype(np.uint8)
    ref, mu, sg, fl = ro.channel_mask(fil, 4)
    assert set(np.flatnonzero(fl).tolist()) == set(bad.tolist())
    x = torch.from_numpy(fil).cuda()
    out, st = m.chan_mask(x, 4, out=x)
    z = m.zero_dm(out, 64)
    torch.cuda.synchronize()
    assert np.array_equal(st.cpu().numpy()[:, 2].astype(bool), fl)
    assert np.array_equal(z.cpu().numpy(), ro.zero_dm(ref, 64))


@pytest.mark.parametrize("nchan,nsamp", [(13, 1001), (5, 4096), (3, 7), (40, 257)])
def test_rfi_on_buffers_at_odd_byte_offsets(nchan, nsamp):
    # inputs and outputs that start 1 to 5 bytes into their buffer (every
    # row, the first included, starts inside a 4-byte word), in and out of
    # place; at the same alignment mod 4 zero-DM takes its read-once kernel,
    # otherwise the two-pass one; the channel copy works in 16-byte chunks at
    # the same alignment mod 16, otherwise in 4-byte words
    import torch
    m = sps()
    print("rfi odd offsets nchan=%d nsamp=%d" % (nchan, nsamp), flush=True)
    rng = np.random.default_rng(nchan * 31 + nsamp)
    fil = np.clip(np.rint(rng.normal(64, 6, size=(nchan, nsamp))), 0, 255).astype(np.uint8)
    fil[::4] = np.clip(np.rint(rng.normal(90, 40, size=(len(range(0, nchan, 4)), nsamp))), 0, 255).astype(np.uint8)
    fil[:, nsamp // 2] = 255
    size = nchan * nsamp

    def at(offset, src=None):
        base = torch.full((size + 8,), 7, dtype=torch.uint8, device="cuda")
        v = base[offset:offset + size].view(nchan, nsamp)
        if src is not None:
            v.copy_(torch.from_numpy(src))
        return base, v

    zref = ro.zero_dm(fil, 40)
    mref, mu, sg, fl = ro.channel_mask(fil, 2)
    for oi, oo in ((1, 3), (3, 1), (1, 0), (0, 3), (1, 1), (3, 3), (2, 2), (0, 4), (5, 1)):
        bi, xi = at(oi, fil)
        bo, xo = at(oo)
        m.zero_dm(xi, 40, out=xo)
        torch.cuda.synchronize()
        assert np.array_equal(xo.cpu().numpy(), zref), (oi, oo)
        assert np.array_equal(xi.cpu().numpy(), fil), (oi, oo)  # input untouched
        guard = bo.cpu().numpy()
        assert (guard[:oo] == 7).all() and (guard[oo + size:] == 7).all(), (oi, oo)  # nothing past the ends
        bo, xo = at(oo)
        out, st = m.chan_mask(xi, 2, out=xo)
        torch.cuda.synchronize()
        assert np.array_equal(xo.cpu().numpy(), mref), ("mask", oi, oo)
        assert np.array_equal(st.cpu().numpy()[:, 0], mu) and np.array_equal(st.cpu().numpy()[:, 1], sg)
        guard = bo.cpu().numpy()
        assert (guard[:oo] == 7).all() and (guard[oo + size:] == 7).all(), ("mask", oi, oo)
    for off in (1, 3):
        bi, xi = at(off, fil)
        m.zero_dm(xi, 40, out=xi)  # in place
        torch.cuda.synchronize()
        assert np.array_equal(xi.cpu().numpy(), zref), ("in place", off)
        guard = bi.cpu().numpy()
        assert (guard[:off] == 7).all() and (guard[off + size:] == 7).all(), ("in place", off)
        bi, xi = at(off, fil)
        m.chan_mask(xi, 2, out=xi)
        torch.cuda.synchronize()
        assert np.array_equal(xi.cpu().numpy(), mref), ("mask in place", off)
