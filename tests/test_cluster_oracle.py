"""Pins of the clustering oracle (CPU): brute force, closed forms, invariants."""
import itertools

import numpy as np
import pytest

from oracle import CAND_DTYPE
from oracle import cluster_oracle as co


def _cands(rows):
    c = np.empty(len(rows), dtype=CAND_DTYPE)
    for k, (s, d, w, q) in enumerate(rows):
        c[k] = (s, d, w, q)
    return c


def _random_cands(rng, n, t_span, ndm, nw, ties=False):
    seen, rows = set(), []
    while len(rows) < n:
        key = (int(rng.integers(0, t_span)), int(rng.integers(0, ndm)), 1 << int(rng.integers(0, nw)))
        if key in seen:
            continue
        seen.add(key)
        q = float(rng.integers(6, 9)) if ties else float(np.float32(rng.uniform(6, 30)))
        rows.append(key + (q,))
    return _cands(rows)


def _brute_force(c, tt, dt, wt):
    """All pairs, breadth-first components, best member by a full scan."""
    n = c.size
    lw = [int(w).bit_length() - 1 for w in c["width"]]

    def linked(a, b):
        return (abs(int(c["sample"][a]) - int(c["sample"][b])) <= tt and abs(int(c["dm_idx"][a]) - int(c["dm_idx"][b])) <= dt
                and abs(lw[a] - lw[b]) <= wt)

    comp = [-1] * n
    groups = []
    for a in range(n):
        if comp[a] >= 0:
            continue
        comp[a] = len(groups)
        members, frontier = [a], [a]
        while frontier:
            x = frontier.pop()
            for y in range(n):
                if comp[y] < 0 and linked(x, y):
                    comp[y] = comp[a]
                    members.append(y)
                    frontier.append(y)
        groups.append(members)
    recs = []
    for g in groups:
        best = g[0]
        for m in g[1:]:
            kb = (-float(c["snr"][best]), int(c["dm_idx"][best]), int(c["width"][best]), int(c["sample"][best]))
            km = (-float(c["snr"][m]), int(c["dm_idx"][m]), int(c["width"][m]), int(c["sample"][m]))
            if km < kb:
                best = m
        recs.append((int(c["sample"][best]), int(c["dm_idx"][best]), int(c["width"][best]), float(c["snr"][best]), len(g),
                     min(int(c["sample"][m]) for m in g), max(int(c["sample"][m]) for m in g),
                     min(int(c["dm_idx"][m]) for m in g), max(int(c["dm_idx"][m]) for m in g)))
    out = np.array(recs, dtype=co.CLUSTER_DTYPE) if recs else np.empty(0, dtype=co.CLUSTER_DTYPE)
    return co.sort_clusters(out)


@pytest.mark.parametrize("seed", range(8))
def test_cluster_matches_brute_force(seed):
    rng = np.random.default_rng(seed)
    c = _random_cands(rng, int(rng.integers(20, 160)), 400, 40, 6, ties=bool(seed % 2))
    tt, dt, wt = int(rng.integers(0, 12)), int(rng.integers(0, 5)), int(rng.integers(0, 3))
    got = co.cluster(c, tt, dt, wt)
    ref = _brute_force(c, tt, dt, wt)
    assert got.size == ref.size
    assert np.array_equal(got, ref)


def test_zero_tolerance_keeps_every_candidate():
    rng = np.random.default_rng(11)
    c = _random_cands(rng, 300, 50, 10, 4)  # dense, but (sample, dm, width) are distinct
    got = co.cluster(c, 0, 0, 0)
    assert got.size == c.size
    assert np.all(got["members"] == 1)
    ref = c[np.lexsort((c["sample"], c["width"], c["dm_idx"]))]
    for f in ("sample", "dm_idx", "width", "snr"):
        assert np.array_equal(got[f], ref[f])


def test_unbounded_tolerance_gives_one_cluster_at_the_global_best():
    rng = np.random.default_rng(12)
    c = _random_cands(rng, 200, 10000, 500, 13, ties=True)
    got = co.cluster(c, 1 << 40, 1 << 20, 20)
    assert got.size == 1
    r = got[0]
    assert r["members"] == c.size
    assert r["snr"] == c["snr"].max()
    top = c[c["snr"] == c["snr"].max()]
    first = top[np.lexsort((top["sample"], top["width"], top["dm_idx"]))][0]
    assert (r["sample"], r["dm_idx"], r["width"]) == (first["sample"], first["dm_idx"], first["width"])
    assert (r["sample_lo"], r["sample_hi"]) == (c["sample"].min(), c["sample"].max())
    assert (r["dm_lo"], r["dm_hi"]) == (c["dm_idx"].min(), c["dm_idx"].max())


def test_links_chain_transitively():
    # each candidate within time_tol of the next; the ends are far apart
    c = _cands([(10 * k, k % 3, 4, 7.0 + (k == 5)) for k in range(12)])
    got = co.cluster(c, 10, 2, 0)
    assert got.size == 1 and got[0]["members"] == 12 and got[0]["sample"] == 50
    # one missing link splits it
    got = co.cluster(c, 9, 2, 0)
    assert got.size == 12


def test_each_tolerance_is_a_separate_closed_bound():
    base = (100, 5, 8, 9.0)
    for other, tols, linked in [((103, 5, 8, 7.0), (3, 0, 0), True), ((104, 5, 8, 7.0), (3, 0, 0), False),
                                ((100, 7, 8, 7.0), (0, 2, 0), True), ((100, 8, 8, 7.0), (0, 2, 0), False),
                                ((100, 5, 32, 7.0), (0, 0, 2), True), ((100, 5, 64, 7.0), (0, 0, 2), False),
                                ((97, 3, 2, 7.0), (3, 2, 2), True)]:
        got = co.cluster(_cands([base, other]), *tols)
        assert got.size == (1 if linked else 2), (other, tols)


def test_permutation_invariance():
    rng = np.random.default_rng(5)
    c = _random_cands(rng, 500, 3000, 64, 8)
    ref = co.cluster(c, 6, 3, 1)
    for _ in range(3):
        assert np.array_equal(co.cluster(c[rng.permutation(c.size)], 6, 3, 1), ref)


def test_members_partition_the_input():
    rng = np.random.default_rng(9)
    c = _random_cands(rng, 800, 2000, 100, 10)
    for tols in itertools.product((0, 4, 30), (0, 3), (0, 1)):
        got = co.cluster(c, *tols)
        assert int(got["members"].sum()) == c.size
