"""Pins of the zero-DM oracle (CPU): brute force, removal of an undispersed
impulse, survival of a dispersed pulse, constant input, rounding of the
level, clipping."""
import numpy as np
import pytest

from oracle import dedisp_oracle as dd
from oracle import rfi_oracle as ro
from synth import filterbank as fb


def test_brute_force_tiny():
    rng = np.random.default_rng(1)
    fil = rng.integers(0, 256, size=(7, 30)).astype(np.uint8)
    got = ro.zero_dm(fil, 40)
    for t in range(30):
        col = [int(fil[f][t]) for f in range(7)]
        s = sum(col)
        # mean rounded half up: the integer nearest s/7, ties upward
        z = int(s / 7 + 0.5) if (2 * s) % 14 != 7 else (s // 7) + 1
        for f in range(7):
            assert got[f][t] == min(255, max(0, col[f] - z + 40))


def test_level_rounds_half_up():
    fil = np.array([[1, 2, 0], [2, 2, 1]], dtype=np.uint8)  # means 1.5, 2, 0.5
    assert ro.zero_dm_level(fil).tolist() == [2, 2, 1]


def test_undispersed_impulse_is_removed_exactly():
    rng = np.random.default_rng(2)
    fil = rng.integers(60, 70, size=(32, 400)).astype(np.uint8)
    hit = fil.copy()
    hit[:, 123] += 50  # the same 50 in every channel at one time: a DM-0 burst
    a, b = ro.zero_dm(fil, 64), ro.zero_dm(hit, 64)
    assert np.array_equal(a, b)


def test_dispersed_pulse_survives_and_constant_input_goes_to_offset():
    f, fref = fb.band(64)
    tab = dd.delays(f, fref, 1e-4, [0.0, 400.0])
    fil = fb.filterbank(64, 9000, seed=3, sigma=0.0, pulses=[(300, 2, 40)], tracks=tab[1:2])
    out = ro.zero_dm(fil, 64)
    # one channel per time sample carries the sweep: it keeps most of its excess
    back = dd.dedisperse(out, tab)
    assert back[1, 300] - 64 * 64 >= 64 * 40 - 64 * 2
    assert np.all(ro.zero_dm(np.full((5, 9), 200, dtype=np.uint8), 17) == 17)


def test_clipping_and_offset_range():
    fil = np.array([[0, 255], [255, 0]], dtype=np.uint8)  # means 127.5 -> 128
    out = ro.zero_dm(fil, 0)
    assert out.tolist() == [[0, 127], [127, 0]]
    with pytest.raises(ValueError):
        ro.zero_dm(fil, 256)


def test_channel_stats_brute_force():
    rng = np.random.default_rng(7)
    fil = rng.integers(0, 256, size=(6, 41)).astype(np.uint8)
    fil[2] = rng.integers(100, 103, size=41)
    mu, sg = ro.channel_stats(fil)
    for f in range(6):
        row = sorted(int(v) for v in fil[f])
        m = row[20]
        assert mu[f] == m
        assert sg[f] == sorted(abs(v - m) for v in row)[20]


def test_noisy_channels_are_flagged_and_replaced_by_their_median():
    rng = np.random.default_rng(8)
    fil = np.clip(np.rint(rng.normal(64, 6, size=(64, 3000))), 0, 255).astype(np.uint8)
    bad = [5, 40, 41]
    for f in bad:  # narrowband interference: strongly fluctuating power
        fil[f] = np.clip(np.rint(rng.normal(90, 40, size=3000)), 0, 255).astype(np.uint8)
    out, mu, sg, fl = ro.channel_mask(fil, 3)
    assert sorted(np.flatnonzero(fl).tolist()) == bad
    for f in bad:
        assert np.all(out[f] == mu[f])
    keep = np.setdiff1d(np.arange(64), bad)
    assert np.array_equal(out[keep], fil[keep])


def test_channel_mask_closed_cases():
    # identical channels: S = 0 and no channel exceeds M; nothing is flagged
    fil = np.tile(np.arange(50, dtype=np.uint8), (8, 1))
    out, _, _, fl = ro.channel_mask(fil, 0)
    assert not fl.any() and np.array_equal(out, fil)
    # k = 0: every channel above the median MAD is flagged
    fil = np.stack([np.tile(np.array([100 - d, 100, 100 + d], dtype=np.uint8), 7) for d in (1, 2, 3, 4, 5)])
    _, _, sg, fl = ro.channel_mask(fil, 0)
    assert sg.tolist() == [1, 2, 3, 4, 5] and fl.tolist() == [False, False, False, True, True]
