"""Comparison helpers for GPU-vs-oracle parity (test support, no GPU code)."""
import multiprocessing as mp
import os

import numpy as np

SNR_RTOL = 1e-4        # per-candidate S/N tolerance
EDGE_REL = 1e-3        # candidates with |snr - theta| <= EDGE_REL * theta may differ


def keyset(c):
    return set(zip(c["dm_idx"].tolist(), c["width"].tolist(), c["sample"].tolist()))


def compare_cands(gpu, ref, theta, where=""):
    """Assert two candidate arrays agree to the parity rule; return the number of exemptions.

    Sets must be identical except for candidates whose S/N lies within
    EDGE_REL*theta of the threshold; matched candidates agree in S/N within
    SNR_RTOL (relative).
    """
    g = {k: s for k, s in zip(zip(gpu["dm_idx"].tolist(), gpu["width"].tolist(), gpu["sample"].tolist()),
                              gpu["snr"].tolist())}
    r = {k: s for k, s in zip(zip(ref["dm_idx"].tolist(), ref["width"].tolist(), ref["sample"].tolist()),
                              ref["snr"].tolist())}
    only_g = [k for k in g if k not in r]
    only_r = [k for k in r if k not in g]
    edge = EDGE_REL * theta
    bad_g = [(k, g[k]) for k in only_g if abs(g[k] - theta) > edge]
    bad_r = [(k, r[k]) for k in only_r if abs(r[k] - theta) > edge]
    assert not bad_g and not bad_r, "%s: %d extra on GPU %s, %d missing %s" % (
        where, len(bad_g), bad_g[:5], len(bad_r), bad_r[:5])
    common = [k for k in g if k in r]
    if common:
        gs = np.array([g[k] for k in common], dtype=np.float64)
        rs = np.array([r[k] for k in common], dtype=np.float64)
        rel = np.abs(gs - rs) / np.maximum(np.abs(rs), 1e-30)
        assert rel.max() <= SNR_RTOL, "%s: snr rel err %g at %s" % (where, rel.max(), common[int(rel.argmax())])
    return len(only_g) + len(only_r)


def exact_equal(a, b):
    """Sorted candidate arrays identical in every field (bitwise S/N)."""
    if a.size != b.size:
        return False
    return (np.array_equal(a["sample"].astype(np.int64), b["sample"].astype(np.int64))
            and np.array_equal(a["dm_idx"], b["dm_idx"]) and np.array_equal(a["width"], b["width"])
            and np.array_equal(a["snr"].view(np.uint32), b["snr"].view(np.uint32)))


def _oracle_row(args):
    x_row, row_id, max_width, L, theta, kw = args
    import oracle
    return oracle.search(x_row[None, :], max_width, L, theta, row_ids=[row_id], with_stats=True, **kw)


def oracle_rows(x, rows, max_width, L, theta, **kw):
    """oracle.search(x, ..., rows=rows, with_stats=True, **kw), one process per
    row (at most 16): returns candidates sorted (dm, width, sample) and the
    stacked block medians and MADs of the rows, in the order given."""
    import oracle
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        cores = os.cpu_count() or 1
    procs = max(1, min(16, cores, len(rows)))
    tasks = [(np.ascontiguousarray(x[r]), int(r), max_width, L, theta, kw) for r in rows]
    with mp.get_context("spawn").Pool(procs) as pool:
        res = pool.map(_oracle_row, tasks)
    cands = oracle.sort_cands(np.concatenate([c for c, _, _ in res]))
    return cands, np.concatenate([m for _, m, _ in res]), np.concatenate([d for _, _, d in res])
