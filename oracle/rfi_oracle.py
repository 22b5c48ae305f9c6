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
