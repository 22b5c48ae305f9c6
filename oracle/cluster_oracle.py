"""CPU oracle for candidate merging and clustering (test infrastructure).

TEST INFRASTRUCTURE ONLY. Only the test suite and the benchmark may import
this module; the HIP library and its binding never do, and nothing here is
shared with them.

What is computed (Heimdall++, Section II-B "Candidate Merging and
Clustering", Section III's discussion of that stage, and the last step of
Algorithm 1): candidates that lie close together in time, DM trial and
filter width are grouped, and each group is reported once, by its candidate
of highest S/N. The paper gives no tolerances and no grouping rule, so the
reading is this project's:

1. Two candidates a and b are linked when |sample_a - sample_b| <= time_tol,
   |dm_a - dm_b| <= dm_tol and |log2 width_a - log2 width_b| <= width_tol
   (all three, closed intervals; tolerances are non-negative integers).
2. Clusters are the connected components of the link graph (a
   friends-of-friends grouping: a chain of links joins a cluster).
3. Each cluster is reported by its member of largest S/N; among equal S/N
   the one with the smallest (dm, width, sample). The record also carries
   the member count and the cluster's sample and DM extents.
"""
from __future__ import annotations

import numpy as np
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

CLUSTER_DTYPE = np.dtype([("sample", "<i8"), ("dm_idx", "<u4"), ("width", "<u4"), ("snr", "<f4"),
                          ("members", "<u4"), ("sample_lo", "<i8"), ("sample_hi", "<i8"),
                          ("dm_lo", "<u4"), ("dm_hi", "<u4")])


def _log2w(width: np.ndarray) -> np.ndarray:
    w = np.asarray(width, dtype=np.int64)
    if np.any(w <= 0) or np.any(w & (w - 1)):
        raise ValueError("widths must be powers of two")
    return np.round(np.log2(w)).astype(np.int64)


def links(cands: np.ndarray, time_tol: int, dm_tol: int, width_tol: int):
    """Reading 1: every linked pair (i, j), i < j, as two index arrays.

    Candidates are visited in sample order; each is compared with the later
    ones whose sample lies within time_tol (found by a sorted search)."""
    n = cands.size
    s = np.asarray(cands["sample"], dtype=np.int64)
    d = np.asarray(cands["dm_idx"], dtype=np.int64)
    lw = _log2w(cands["width"])
    order = np.argsort(s, kind="stable")
    ss = s[order]
    end = np.searchsorted(ss, ss + time_tol, side="right")
    ii, jj = [], []
    for a in range(n):
        b = np.arange(a + 1, end[a])
        if b.size == 0:
            continue
        ia, ib = order[a], order[b]
        ok = (np.abs(d[ib] - d[ia]) <= dm_tol) & (np.abs(lw[ib] - lw[ia]) <= width_tol)
        ii.append(np.full(int(ok.sum()), ia))
        jj.append(ib[ok])
    if not ii:
        return np.empty(0, np.int64), np.empty(0, np.int64)
    return np.concatenate(ii).astype(np.int64), np.concatenate(jj).astype(np.int64)


def labels(cands: np.ndarray, time_tol: int, dm_tol: int, width_tol: int) -> np.ndarray:
    """Reading 2: connected-component label of every candidate (0 .. nclusters-1)."""
    n = cands.size
    if n == 0:
        return np.empty(0, np.int64)
    i, j = links(cands, time_tol, dm_tol, width_tol)
    g = coo_matrix((np.ones(i.size, dtype=np.int8), (i, j)), shape=(n, n))
    _, lab = connected_components(g, directed=False)
    return lab.astype(np.int64)


def cluster(cands: np.ndarray, time_tol: int, dm_tol: int, width_tol: int) -> np.ndarray:
    """Readings 1-3: one record per cluster, sorted by (dm, width, sample) of its best member."""
    if min(time_tol, dm_tol, width_tol) < 0:
        raise ValueError("tolerances must be >= 0")
    n = cands.size
    out = np.empty(0, dtype=CLUSTER_DTYPE)
    if n == 0:
        return out
    lab = labels(cands, time_tol, dm_tol, width_tol)
    s = np.asarray(cands["sample"], dtype=np.int64)
    d = np.asarray(cands["dm_idx"], dtype=np.int64)
    w = np.asarray(cands["width"], dtype=np.int64)
    q = np.asarray(cands["snr"], dtype=np.float32)
    # best member: largest snr, then smallest (dm, width, sample)
    order = np.lexsort((s, w, d, -q.astype(np.float64), lab))
    first = np.ones(n, dtype=bool)
    first[1:] = lab[order][1:] != lab[order][:-1]
    best = order[first]
    nc = best.size
    out = np.empty(nc, dtype=CLUSTER_DTYPE)
    out["sample"], out["dm_idx"], out["width"], out["snr"] = s[best], d[best], w[best], q[best]
    blab = lab[best]
    out["members"] = np.bincount(lab, minlength=nc)[blab]
    lo = np.full(nc, np.iinfo(np.int64).max); hi = np.full(nc, np.iinfo(np.int64).min)
    np.minimum.at(lo, lab, s); np.maximum.at(hi, lab, s)
    dlo = np.full(nc, np.iinfo(np.int64).max); dhi = np.full(nc, -1)
    np.minimum.at(dlo, lab, d); np.maximum.at(dhi, lab, d)
    out["sample_lo"], out["sample_hi"] = lo[blab], hi[blab]
    out["dm_lo"], out["dm_hi"] = dlo[blab], dhi[blab]
    return sort_clusters(out)


def sort_clusters(c: np.ndarray) -> np.ndarray:
    """Canonical order of cluster records: (dm, width, sample) of the best member."""
    if c.size == 0:
        return c
    return c[np.lexsort((c["sample"], c["width"], c["dm_idx"]))]
