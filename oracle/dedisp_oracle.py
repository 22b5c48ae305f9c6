"""CPU oracle for incoherent dedispersion (test infrastructure).

TEST INFRASTRUCTURE ONLY. Only the test suite and the benchmark may import
this module; the HIP library and its binding never do, and nothing here is
shared with them.

What is computed (Heimdall++, Section II-B "Incoherent Dedispersion", with
the dispersion measure of Eq. 1, and the dedispersion step of Algorithm 1):
for every trial DM the channels of a filterbank are shifted in time by their
dispersion delay and summed. The paper names the stage and the library it
uses, not the delay law or its rounding, so the reading is this project's:

1. Delay of channel f (centre frequency nu_f, MHz) at trial DM D, in samples
   of tsamp seconds, relative to the reference frequency nu_ref (the top of
   the band): ``k_DM * D * (nu_f^-2 - nu_ref^-2) / tsamp`` with the
   cold-plasma dispersion constant ``k_DM = 4.148808e3 MHz^2 pc^-1 cm^3 s``,
   evaluated in double precision in that order and rounded half up to an
   integer (``floor(v + 0.5)``). Channels above nu_ref are not allowed.
2. Dedispersed series of trial d: ``out[d, t] = sum_f I[f, t + delay[d, f]]``
   for ``0 <= t < nsamp_in - max(delay)``, with I the 8-bit filterbank in
   channel-major order ``[nchan][nsamp_in]``. The sums are exact integers.
"""
from __future__ import annotations

import numpy as np

K_DM = 4.148808e3  # MHz^2 pc^-1 cm^3 s


def delays(freqs_mhz, f_ref_mhz: float, tsamp_s: float, dms) -> np.ndarray:
    """Reading 1: int64 table [ndm][nchan] of per-channel delays in samples."""
    f = np.asarray(freqs_mhz, dtype=np.float64)
    d = np.asarray(dms, dtype=np.float32).astype(np.float64)
    if np.any(f > f_ref_mhz) or np.any(f <= 0) or np.any(d < 0) or not tsamp_s > 0:
        raise ValueError("channels must lie at or below the reference frequency; DMs >= 0; tsamp > 0")
    out = np.empty((d.size, f.size), dtype=np.int64)
    for i in range(d.size):
        for j in range(f.size):
            v = K_DM * d[i] * (1.0 / (f[j] * f[j]) - 1.0 / (f_ref_mhz * f_ref_mhz)) / tsamp_s
            out[i, j] = int(np.floor(v + 0.5))
    return out


def dedisperse(fil: np.ndarray, delay: np.ndarray) -> np.ndarray:
    """Reading 2: int64 [ndm][nsamp_out] channel sums along each trial's delays."""
    fil = np.asarray(fil)
    if fil.dtype != np.uint8 or fil.ndim != 2:
        raise ValueError("filterbank must be uint8 [nchan][nsamp_in]")
    nchan, nin = fil.shape
    delay = np.asarray(delay, dtype=np.int64)
    nout = nin - int(delay.max()) if delay.size else nin
    if nout <= 0:
        raise ValueError("delays exceed the input")
    out = np.zeros((delay.shape[0], nout), dtype=np.int64)
    for d in range(delay.shape[0]):
        for f in range(nchan):
            s = int(delay[d, f])
            out[d] += fil[f, s:s + nout]
    return out
