"""The seeded input generator: published Philox answers, Gaussian table, determinism."""
import numpy as np
import pytest
from scipy.stats import norm

import synth


def test_philox4x64_known_answers():
    # Random123's published known-answer vector for philox4x64-10, counter 0 / key 0.
    got = [int(v) for v in synth.philox((0, 0, 0, 0), (0, 0))]
    assert got == [0x16554D9ECA36314C, 0xDB20FE9D672D0FDC, 0xD7E772CEE186176B, 0x7E68B68AEC7BA23B]
    # numpy's Philox (also philox4x64-10) bumps its counter before each block.
    key = np.array([123456789, 987654321], dtype=np.uint64)
    bg = np.random.Philox(key=key, counter=np.array([41, 0, 0, 0], dtype=np.uint64))
    ref = bg.random_raw(8)
    ours = synth.philox((42, 0, 0, 0), (123456789, 987654321), nblocks=2)
    assert np.array_equal(ours, ref)


def test_integer_gaussian_table():
    sigma = 1024.0
    u = synth.philox((0, 0, 7, 0), (1, 2), nblocks=1 << 17)
    g = synth.int_gauss(sigma, u).astype(np.float64)
    assert abs(g.mean()) < 4 * sigma / np.sqrt(g.size)
    assert abs(g.std() / np.sqrt(sigma ** 2 + 1 / 12) - 1) < 0.01
    # empirical CDF of round(N(0, sigma^2)) at a few integers
    for k in (-2048, -1024, 0, 700, 2500):
        p = (g <= k).mean()
        assert abs(p - norm.cdf((k + 0.5) / sigma)) < 4 * np.sqrt(0.25 / g.size)
    # monotone in u: the largest and smallest words hit the clamped tails
    ext = synth.int_gauss(sigma, np.array([0, 2 ** 64 - 1], dtype=np.uint64))
    assert ext[0] == -8 * 1024 and ext[1] == 8 * 1024


def test_generate_is_coordinate_deterministic():
    b = synth.config(1)["blocks"][0]
    x = synth.generate(b, nthreads=3)
    assert np.array_equal(x, synth.generate(b, nthreads=1))
    sub = synth.generate(b, t0=1001, nsamp=333, rows=[5, 2, 63])
    assert np.array_equal(sub, x[[5, 2, 63], 1001:1334])
    assert np.all(x == np.round(x))
    assert np.abs(x).max() < 2 ** 24


def test_pulses_do_not_overlap_and_straddle():
    b = synth.config(3)["blocks"][0].with_(ndm=64, n_pulses=40)
    ps = synth.pulses(b)
    assert len(ps) == 40
    for i, p in enumerate(ps):
        for q in ps[:i]:
            assert (p.row + p.nrows <= q.row or q.row + q.nrows <= p.row or p.t0 + p.width <= q.t0
                    or q.t0 + q.width <= p.t0)
    gulp = b.straddle_period
    straddling = [p for p in ps if p.t0 // gulp != (p.t0 + p.width - 1) // gulp]
    assert len(straddling) >= 15


def test_configs_shapes():
    assert synth.config(1)["blocks"][0].ndm == 64
    c4 = synth.config(4)["blocks"]
    assert len(c4) == 32
    assert {b.ndm for b in c4} <= {256, 512, 1024, 2048}
    assert {b.nsamp for b in c4} <= {1 << k for k in range(16, 21)}
    c5 = synth.config(5)["blocks"]
    assert len(c5) == 16 and all(512 <= b.ndm <= 2048 for b in c5)
    with pytest.raises(ValueError):
        synth.config(6)
