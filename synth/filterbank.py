"""Seeded synthetic 8-bit filterbanks (input generation only).

Holds none of the dedispersion arithmetic: a dispersed pulse is placed along
a per-channel track of sample offsets that the caller supplies.

Model: noise ``clip(round(N(mean, sigma^2)), 0, 255)`` from numpy's PCG64
seeded by ``seed``, channel-major ``[nchan][nsamp]`` uint8; each pulse adds
``amp`` (saturating at 255) to ``width`` samples starting at
``t0 + track[f]`` in every channel f.
"""
from __future__ import annotations

from typing import Optional, Sequence, Tuple

import numpy as np


def filterbank(nchan: int, nsamp: int, seed: int, mean: float = 64.0, sigma: float = 6.0,
               pulses: Sequence[Tuple[int, int, int]] = (), tracks: Optional[np.ndarray] = None) -> np.ndarray:
    """uint8 [nchan][nsamp]; pulses are (t0, width, amp), one track row each."""
    rng = np.random.default_rng(seed)
    out = np.empty((nchan, nsamp), dtype=np.uint8)
    for f in range(nchan):
        v = np.rint(rng.normal(mean, sigma, size=nsamp))
        out[f] = np.clip(v, 0, 255).astype(np.uint8)
    if pulses:
        tr = np.asarray(tracks, dtype=np.int64)
        for k, (t0, width, amp) in enumerate(pulses):
            for f in range(nchan):
                s = t0 + int(tr[k, f])
                e = min(nsamp, s + width)
                if s < 0 or s >= nsamp:
                    continue
                seg = out[f, s:e].astype(np.int64) + amp
                out[f, s:e] = np.minimum(seg, 255).astype(np.uint8)
    return out


def band(nchan: int, f_lo_mhz: float = 1050.0, f_hi_mhz: float = 1450.0) -> Tuple[np.ndarray, float]:
    """Channel centre frequencies (MHz, highest first) of a band split into
    nchan equal channels, and the band top used as the reference."""
    bw = (f_hi_mhz - f_lo_mhz) / nchan
    return f_hi_mhz - bw * (np.arange(nchan) + 0.5), f_hi_mhz
