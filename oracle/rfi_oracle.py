"""CPU oracle for broadband (zero-DM) RFI excision (test infrastructure).

TEST INFRASTRUCTURE ONLY. Only the test suite and the benchmark may import
this module; the HIP library and its binding never do, and nothing here is
shared with them.

What is computed (Heimdall++, Section II-B "RFI Mitigation", the stage before
dedispersion in Algorithm 1): interference that spans every channel arrives
at all frequencies at once, i.e. it is undispersed (DM 0), and is removed by
subtracting each time sample's level across the band. The paper names the
strategy, not the estimator, so the reading is this project's:

1. Zero-DM level of time sample t: the mean over channels of I[f, t], rounded
   half up in exact integer arithmetic, z_t = floor((2 * sum_f I[f, t] +
   nchan) / (2 * nchan)).
2. Output: O[f, t] = min(255, max(0, I[f, t] - z_t + offset)) with the
   caller's integer offset in [0, 255] (the level the filtered data sit at).

Narrowband interference raises the power of a few channels. Reading for that
half of the strategy:

3. Per channel f over the chunk: mu_f = lower median of I[f, :] and sigma_f =
   lower median of |I[f, t] - mu_f| (rank floor((n-1)/2) of the sorted values).
4. Across channels: M = lower median of sigma_f and S = lower median of
   |sigma_f - M|; channel f is flagged iff sigma_f > M + k * S for the caller's
   integer k >= 0.
5. A flagged channel is replaced by its median: O[f, t] = mu_f for every t;
   the other channels are unchanged.
"""
from __future__ import annotations

import numpy as np


def zero_dm_level(fil: np.ndarray) -> np.ndarray:
    """Reading 1: int64 z_t for every time sample of a uint8 [nchan][nsamp] filterbank."""
    fil = np.asarray(fil)
    if fil.dtype != np.uint8 or fil.ndim != 2:
        raise ValueError("filterbank must be uint8 [nchan][nsamp]")
    nchan = fil.shape[0]
    s = fil.astype(np.int64).sum(axis=0)
    return (2 * s + nchan) // (2 * nchan)


def zero_dm(fil: np.ndarray, offset: int) -> np.ndarray:
    """Reading 2: the filtered uint8 filterbank."""
    if not 0 <= int(offset) <= 255:
        raise ValueError("offset must lie in [0, 255]")
    z = zero_dm_level(fil)
    out = fil.astype(np.int64) - z[None, :] + int(offset)
    return np.clip(out, 0, 255).astype(np.uint8)


def _lower_median(v: np.ndarray) -> int:
    v = np.asarray(v, dtype=np.int64)
    r = (v.size - 1) // 2
    return int(np.partition(v, r)[r])


def channel_stats(fil: np.ndarray):
    """Reading 3: int64 arrays (mu_f, sigma_f) over the channels of a uint8 [nchan][nsamp] filterbank."""
    fil = np.asarray(fil)
    if fil.dtype != np.uint8 or fil.ndim != 2:
        raise ValueError("filterbank must be uint8 [nchan][nsamp]")
    mu = np.array([_lower_median(row) for row in fil], dtype=np.int64)
    sg = np.array([_lower_median(np.abs(row.astype(np.int64) - m)) for row, m in zip(fil, mu)], dtype=np.int64)
    return mu, sg


def channel_flags(sigma: np.ndarray, k: int) -> np.ndarray:
    """Reading 4: bool flags from the channels' MADs."""
    if int(k) < 0:
        raise ValueError("k must be >= 0")
    M = _lower_median(sigma)
    S = _lower_median(np.abs(np.asarray(sigma, dtype=np.int64) - M))
    return np.asarray(sigma) > M + int(k) * S


def channel_mask(fil: np.ndarray, k: int):
    """Readings 3-5: (filtered uint8 filterbank, mu, sigma, flags)."""
    mu, sg = channel_stats(fil)
    fl = channel_flags(sg, k)
    out = np.array(fil, dtype=np.uint8, copy=True)
    out[fl] = mu[fl, None].astype(np.uint8)
    return out, mu, sg, fl
