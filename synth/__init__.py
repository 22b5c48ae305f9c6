"""Seeded synthetic dedispersed blocks (input generation only).

This module holds none of the search's arithmetic. It writes the arrays that
both the CPU oracle and the HIP path consume, so the two sides see the same
bits. It imports neither of them.

Model (stand-in for the telescope data the paper measures on, which is not
available here):

* noise: integer Gaussian ``round(N(mu, sigma^2))`` drawn by inverse CDF from
  Philox4x64-10 words keyed by ``(seed, stream)`` with counter
  ``(t >> 2, row, purpose, 0)``, so every sample depends only on its
  coordinates (``synth.c``);
* drift: ``round(a * sigma * sin(2 pi t / P))`` on the global sample index;
* pulses: boxcars of width ``w`` (log-uniform integer) and target S/N ``s``
  (uniform); amplitude ``round(s * sigma / sqrt(w))`` over ``pulse_rows``
  adjacent DM rows; pulses never overlap in (row, time);
* zero-DM RFI: an impulse at ``t_r`` that incoherent dedispersion smears over
  ``1 + round(dt_d / tsamp)`` samples in row ``d`` (``dt_d`` = the cold-plasma
  delay across the band at that row's DM), amplitude ``round(F / width)``
  with ``F`` giving S/N ``rfi_snr`` at DM 0.

All values are exact integers stored in FP32 (|x| < 2^24).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field, replace
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None

PURPOSE_PULSE = 0x50554C5345  # "PULSE"
PURPOSE_RFI = 0x524649  # "RFI"
PURPOSE_SHAPE = 0x5348415045  # "SHAPE"
K_DM_S_GHZ2 = 4.148808e-3  # dispersion delay constant, seconds * GHz^2 per (pc cm^-3)


def build(force: bool = False) -> str:
    """Compile ``libsynth.so`` with gcc (host code only)."""
    src = os.path.join(_HERE, "synth.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", src, "-o", tmp,
                               "-lm", "-lpthread"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _FillArgs(ctypes.Structure):
    _fields_ = [
        ("out", ctypes.c_void_p),
        ("nrow", ctypes.c_int64), ("nsamp", ctypes.c_int64), ("ld", ctypes.c_int64),
        ("row0", ctypes.c_int64), ("t0", ctypes.c_int64),
        ("seed", ctypes.c_uint64), ("stream", ctypes.c_uint64),
        ("mu", ctypes.c_double), ("sigma", ctypes.c_double),
        ("drift_amp", ctypes.c_double), ("drift_period", ctypes.c_int64),
    ]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.synth_philox_blocks.argtypes = [ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64),
                                            ctypes.c_int64, ctypes.POINTER(ctypes.c_uint64)]
        lib.synth_philox_blocks.restype = None
        lib.synth_fill_noise.argtypes = [ctypes.POINTER(_FillArgs), ctypes.c_int]
        lib.synth_fill_noise.restype = ctypes.c_int
        lib.synth_int_gauss.argtypes = [ctypes.c_double, ctypes.POINTER(ctypes.c_uint64), ctypes.c_int64,
                                        ctypes.POINTER(ctypes.c_int32)]
        lib.synth_int_gauss.restype = ctypes.c_int
        _lib = lib
    return _lib


def philox(ctr: Sequence[int], key: Sequence[int], nblocks: int = 1) -> np.ndarray:
    """Philox4x64-10 blocks for counters ctr, ctr+1, ... (word 0 incremented)."""
    lib = _load()
    c = (ctypes.c_uint64 * 4)(*[int(v) & 0xFFFFFFFFFFFFFFFF for v in ctr])
    k = (ctypes.c_uint64 * 2)(*[int(v) & 0xFFFFFFFFFFFFFFFF for v in key])
    out = np.empty(4 * nblocks, dtype=np.uint64)
    lib.synth_philox_blocks(c, k, nblocks, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    return out


def int_gauss(sigma: float, u: np.ndarray) -> np.ndarray:
    """Inverse-CDF integer Gaussian offsets for uniform 64-bit words ``u``."""
    lib = _load()
    u = np.ascontiguousarray(u, dtype=np.uint64)
    out = np.empty(u.shape, dtype=np.int32)
    rc = lib.synth_int_gauss(float(sigma), u.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), u.size,
                             out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if rc:
        raise RuntimeError("synth_int_gauss failed")
    return out


def _unit(u: int) -> float:
    """Map a 64-bit word to [0, 1)."""
    return (int(u) >> 11) * (1.0 / 9007199254740992.0)


def _round_half_up(v: float) -> int:
    return int(math.floor(v + 0.5))


@dataclass(frozen=True)
class Pulse:
    row: int          # first DM row
    nrows: int        # rows row .. row+nrows-1
    t0: int           # first sample (global index)
    width: int
    snr: float        # target S/N
    amp: int          # integer amplitude added to each sample


@dataclass(frozen=True)
class Block:
    """One dedispersed block (a file, or a beam's observation) and its search plan."""
    ndm: int
    nsamp: int                     # total samples of the observation
    max_width: int
    baseline_len: int
    snr_thresh: float = 6.0
    seed: int = 20251200
    stream: int = 0                # file / beam id (Philox key word 1)
    mu: float = 32768.0
    sigma: float = 1024.0
    drift_amp_sigma: float = 2.0   # drift amplitude in units of sigma (0 = none)
    drift_period: int = 8192
    n_pulses: int = 0
    pulse_width: Tuple[int, int] = (1, 32)
    pulse_snr: Tuple[float, float] = (6.0, 20.0)
    pulse_rows: int = 3
    straddle_period: int = 0       # >0: every other pulse straddles a multiple of this
    n_rfi: int = 0
    rfi_snr: float = 50.0
    dm_max: float = 2000.0
    tsamp: float = 64e-6
    f_lo_ghz: float = 1.0
    f_hi_ghz: float = 1.5

    def with_(self, **kw) -> "Block":
        return replace(self, **kw)


def pulses(b: Block) -> List[Pulse]:
    """Deterministic, non-overlapping pulse list for block ``b``."""
    out: List[Pulse] = []
    if b.n_pulses <= 0 or b.ndm <= 0 or b.nsamp <= 0:
        return out
    rows = max(1, min(b.pulse_rows, b.ndm))
    wmin, wmax = b.pulse_width
    wmax = max(wmin, min(wmax, b.nsamp))
    for p in range(b.n_pulses):
        for attempt in range(100000):
            u = philox((p, attempt, PURPOSE_PULSE, 0), (b.seed, b.stream))
            lw = math.log(wmin) + _unit(u[1]) * (math.log(wmax + 1) - math.log(wmin))
            w = min(wmax, max(wmin, int(math.floor(math.exp(lw)))))
            s = b.pulse_snr[0] + _unit(u[2]) * (b.pulse_snr[1] - b.pulse_snr[0])
            d0 = int(u[0] % np.uint64(b.ndm - rows + 1))
            nper = b.nsamp // b.straddle_period if b.straddle_period > 0 else 0
            if b.straddle_period > 0 and p % 2 == 0 and w >= 2 and nper >= 2:
                edge = b.straddle_period * (1 + int(u[3] % np.uint64(nper - 1)))
                t0 = edge - 1 - int((u[3] >> np.uint64(32)) % np.uint64(w - 1))
            else:
                t0 = int(u[3] % np.uint64(b.nsamp - w + 1))
            if t0 < 0 or t0 + w > b.nsamp:
                continue
            clash = any(not (d0 + rows <= q.row or q.row + q.nrows <= d0 or t0 + w <= q.t0 or q.t0 + q.width <= t0)
                        for q in out)
            if clash:
                continue
            amp = _round_half_up(s * b.sigma / math.sqrt(w))
            out.append(Pulse(d0, rows, t0, w, s, amp))
            break
        else:
            raise RuntimeError("could not place pulse %d" % p)
    return out


def rfi_times(b: Block) -> List[int]:
    return [int(philox((r, 0, PURPOSE_RFI, 0), (b.seed, b.stream))[0] % np.uint64(b.nsamp))
            for r in range(b.n_rfi)]


def rfi_profile(b: Block) -> Tuple[np.ndarray, np.ndarray]:
    """Per-row smear width and amplitude of one zero-DM impulse."""
    d = np.arange(b.ndm, dtype=np.float64)
    dm = b.dm_max * d / (b.ndm - 1) if b.ndm > 1 else np.zeros(1)
    delay = K_DM_S_GHZ2 * dm * (b.f_lo_ghz ** -2 - b.f_hi_ghz ** -2)
    width = 1 + np.floor(delay / b.tsamp + 0.5).astype(np.int64)
    amp = np.floor(b.rfi_snr * b.sigma / width + 0.5).astype(np.int64)
    return width, amp


def generate(b: Block, t0: int = 0, nsamp: Optional[int] = None, rows: Optional[Sequence[int]] = None,
             nthreads: Optional[int] = None, out: Optional[np.ndarray] = None) -> np.ndarray:
    """Samples ``[t0, t0+nsamp)`` of rows ``rows`` (default all) as FP32 ``[nrow][nsamp]``."""
    if nsamp is None:
        nsamp = b.nsamp - t0
    if t0 < 0 or nsamp < 0 or t0 + nsamp > b.nsamp:
        raise ValueError("slice outside the observation")
    row_list = list(range(b.ndm)) if rows is None else [int(r) for r in rows]
    nrow = len(row_list)
    if out is None:
        out = np.empty((nrow, nsamp), dtype=np.float32)
    if out.shape != (nrow, nsamp) or out.dtype != np.float32 or not out.flags.c_contiguous:
        raise ValueError("out must be C-contiguous float32 [nrow][nsamp]")
    if nthreads is None:
        nthreads = min(16, os.cpu_count() or 1)
    lib = _load()
    contiguous = rows is None or row_list == list(range(row_list[0], row_list[0] + nrow)) if nrow else True
    groups = [(row_list[0] if nrow else 0, 0, nrow)] if contiguous else [(r, i, 1) for i, r in enumerate(row_list)]
    for row0, i0, cnt in groups:
        if cnt == 0 or nsamp == 0:
            continue
        view = out[i0:i0 + cnt]
        a = _FillArgs(view.ctypes.data, cnt, nsamp, nsamp, row0, t0, b.seed, b.stream, b.mu, b.sigma,
                      b.drift_amp_sigma * b.sigma, b.drift_period)
        if lib.synth_fill_noise(ctypes.byref(a), int(nthreads)):
            raise RuntimeError("synth_fill_noise failed")
    t1 = t0 + nsamp
    pos = {r: i for i, r in enumerate(row_list)}
    for p in pulses(b):
        lo, hi = max(p.t0, t0), min(p.t0 + p.width, t1)
        if lo >= hi:
            continue
        for r in range(p.row, p.row + p.nrows):
            if r in pos:
                out[pos[r], lo - t0:hi - t0] += np.float32(p.amp)
    if b.n_rfi:
        width, amp = rfi_profile(b)
        for tr in rfi_times(b):
            for i, r in enumerate(row_list):
                if amp[r] == 0:
                    continue
                lo, hi = max(tr, t0), min(tr + int(width[r]), t1)
                if lo < hi:
                    out[i, lo - t0:hi - t0] += np.float32(amp[r])
    return out


# ---------------------------------------------------------------------------
# The workloads measured and tested (sizes follow the paper's data shapes:
# thousands of DM trials, 2^16..2^20-sample chunks, 64 us sampling).

BASE_SEED = 20251200


def config(i: int) -> dict:
    """Workload ``i`` (1..5) as a dict with key ``blocks`` (list of Block) and extras."""
    seed = BASE_SEED + (i - 1)
    if i == 1:
        b = Block(ndm=64, nsamp=16384, max_width=64, baseline_len=4096, snr_thresh=6.0, seed=seed,
                  n_pulses=5, pulse_width=(1, 32), pulse_snr=(6.0, 20.0))
        return {"name": "c1_small_64x16384", "blocks": [b]}
    if i == 2:
        b = Block(ndm=1024, nsamp=1 << 20, max_width=4096, baseline_len=16384, snr_thresh=6.0, seed=seed,
                  n_pulses=200, pulse_width=(1, 1024), pulse_snr=(6.0, 50.0), n_rfi=50, dm_max=2000.0)
        return {"name": "c2_large_1024x2^20", "blocks": [b]}
    if i == 3:
        gulp = 1 << 18
        b = Block(ndm=4096, nsamp=8 * gulp, max_width=4096, baseline_len=16384, snr_thresh=6.0, seed=seed,
                  n_pulses=500, pulse_width=(1, 1024), pulse_snr=(6.0, 50.0), straddle_period=gulp)
        return {"name": "c3_stream_4096x8x2^18", "blocks": [b], "gulp": gulp, "ngulps": 8}
    if i == 4:
        blocks = []
        for f in range(32):
            u = philox((f, 0, PURPOSE_SHAPE, 0), (seed, 0))
            ndm = (256, 512, 1024, 2048)[int(u[0] % np.uint64(4))]
            nsamp = 1 << (16 + int(u[1] % np.uint64(5)))
            blocks.append(Block(ndm=ndm, nsamp=nsamp, max_width=4096, baseline_len=16384, snr_thresh=6.0,
                                seed=seed, stream=f, n_pulses=20, pulse_width=(1, 1024),
                                pulse_snr=(6.0, 50.0)))
        return {"name": "c4_batch_32_files", "blocks": blocks}
    if i == 5:
        blocks = []
        for bm in range(16):
            u = philox((bm, 0, PURPOSE_SHAPE, 1), (seed, 0))
            ndm = 512 + int(u[0] % np.uint64(2048 - 512 + 1))
            nsamp = 1 << (16 + int(u[1] % np.uint64(3)))
            blocks.append(Block(ndm=ndm, nsamp=nsamp, max_width=4096, baseline_len=16384, snr_thresh=6.0,
                                seed=seed, stream=bm, n_pulses=20, pulse_width=(1, 1024),
                                pulse_snr=(6.0, 50.0), n_rfi=5))
        return {"name": "c5_serve_16_beams", "blocks": blocks, "arrival_rate_x_realtime": 1.5,
                "hbm_budget_bytes": 200 * 10 ** 9}
    raise ValueError("config index must be 1..5")
