"""Pins of the dedispersion oracle (CPU): the delay law's textbook values,
monotonicity, brute force, a dispersed pulse summed back into one sample,
DM 0 as the plain channel sum, linearity and time shifts."""
import math

import numpy as np
import pytest

from oracle import dedisp_oracle as dd
from synth import filterbank as fb


def test_delay_textbook_value():
    # 4.15 ms x DM x nu_GHz^-2 against an infinitely high reference; here the
    # reference is 1e9 MHz (its term is 1e-18 of the channel's)
    t = dd.delays([1000.0], 1e9, 1e-6, [1.0])
    assert t[0, 0] == 4149  # 4148.808 us at 1 GHz, DM 1
    t = dd.delays([400.0], 1e9, 1e-3, [100.0])
    assert t[0, 0] == round(4.148808e3 * 100 / 400.0 ** 2 / 1e-3)  # 2593 ms at 400 MHz, DM 100
    assert abs(t[0, 0] - 2593) <= 1


def test_delay_monotone_and_zero_at_reference():
    f, fref = fb.band(64)
    dms = np.linspace(0, 800, 17).astype(np.float32)
    t = dd.delays(f, fref, 64e-6, dms)
    assert np.all(t[0] == 0)  # DM 0
    assert np.all(np.diff(t, axis=0) >= 0)  # more DM, more delay
    assert np.all(np.diff(t, axis=1) >= 0)  # channels listed from the top down: lower frequency, more delay
    assert dd.delays([1400.0], 1400.0, 1e-4, [500.0])[0, 0] == 0
    # linear in DM up to the rounding of each value
    t1 = dd.delays(f, fref, 64e-6, [100.0])
    t2 = dd.delays(f, fref, 64e-6, [200.0])
    assert np.all(np.abs(t2 - 2 * t1) <= 1)
    with pytest.raises(ValueError):
        dd.delays([1500.0], 1450.0, 1e-4, [1.0])


def test_brute_force_tiny():
    rng = np.random.default_rng(3)
    nchan, nin = 5, 40
    fil = rng.integers(0, 256, size=(nchan, nin)).astype(np.uint8)
    delay = np.array([[0, 0, 0, 0, 0], [0, 1, 2, 3, 5], [0, 2, 4, 7, 9]])
    got = dd.dedisperse(fil, delay)
    nout = nin - 9
    assert got.shape == (3, nout)
    for d in range(3):
        for t in range(nout):
            s = 0
            for f in range(nchan):
                s += int(fil[f][t + delay[d][f]])
            assert got[d, t] == s


def test_dm_zero_is_channel_sum():
    fil = np.random.default_rng(4).integers(0, 256, size=(16, 300)).astype(np.uint8)
    got = dd.dedisperse(fil, np.zeros((1, 16), dtype=np.int64))
    assert np.array_equal(got[0], fil.astype(np.int64).sum(axis=0))


def test_dispersed_pulse_sums_back_at_its_dm():
    f, fref = fb.band(32)
    dms = np.linspace(0, 300, 31).astype(np.float32)
    tab = dd.delays(f, fref, 2e-4, dms)
    k, t0, amp = 17, 50, 3
    fil = np.zeros((32, 50 + int(tab.max()) + 200), dtype=np.uint8)
    for c in range(32):
        fil[c, t0 + tab[k, c]] = amp
    out = dd.dedisperse(fil, tab)
    assert out[k, t0] == 32 * amp
    assert out[k].sum() == 32 * amp and np.count_nonzero(out[k]) == 1
    # any other trial whose delays differ from the pulse's track leaves channels behind
    for d in range(len(dms)):
        if np.any(tab[d] != tab[k]):
            assert out[d].max() < 32 * amp


def test_linearity_and_time_shift():
    rng = np.random.default_rng(5)
    a = rng.integers(0, 128, size=(8, 500)).astype(np.uint8)
    b = rng.integers(0, 128, size=(8, 500)).astype(np.uint8)
    tab = np.sort(rng.integers(0, 60, size=(6, 8)), axis=1)
    assert np.array_equal(dd.dedisperse(a + b, tab), dd.dedisperse(a, tab) + dd.dedisperse(b, tab))
    s = 17
    sh = np.zeros_like(a)
    sh[:, s:] = a[:, :-s]
    full, shifted = dd.dedisperse(a, tab), dd.dedisperse(sh, tab)
    assert np.array_equal(shifted[:, s:], full[:, :-s])


def test_generator_places_pulses_on_tracks():
    f, fref = fb.band(16)
    tab = dd.delays(f, fref, 1e-4, [0.0, 150.0])
    x = fb.filterbank(16, 3000, seed=1, sigma=0.0, pulses=[(100, 3, 40)], tracks=tab[1:2])
    out = dd.dedisperse(x, tab)
    base = 16 * 64
    assert out[1, 100] == base + 16 * 40 and out[1, 102] == base + 16 * 40 and out[1, 103] == base
