"""Python binding of libsps (ctypes; argument marshalling only).

Every step of the search runs in the HIP library. PyTorch provides device
memory and streams. If the library is not built this module raises: there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsps.so")

SPS_OK = 0
SPS_ERR_INVALID_ARG = -1
SPS_ERR_OOM = -2
SPS_ERR_HIP = -3
SPS_ERR_OVERFLOW = -4
SPS_ERR_DOMAIN = -5
SPS_ERR_SCRATCH = -6
NOALLOC_SCRATCH_BYTES = 64 << 20

ATTR_MAX_CANDS = 1
ATTR_STATS_SEG = 2
ATTR_DETECT_SEG = 3
ATTR_HIST_BINS = 4
ATTR_TIMING = 5
ATTR_VALIDATE = 6
ATTR_WINDOW = 7  # 0 trailing baseline window (default), 1 centred on its block
ATTR_NORM = 8  # 0 per-block MAD scale (default), 1 one MAD per DM row, 2 one MAD per (DM row, width)
ATTR_FUSED = 9  # batches: 1 (default) statistics and detection in one persistent launch, 0 one per stage
NSTAGES = 4
STAGES = ("block_stats", "detect", "fixup", "plain")
ATTR_NBLOCKS = 16
ATTR_NWIDTHS = 17
ATTR_BLOCK_STRIDE = 18

BLOCK_STRIDE = 64
CAND_DTYPE = np.dtype([("sample", "<i4"), ("dm_idx", "<u4"), ("width", "<u4"), ("snr", "<f4")])
# sps_cluster_rec (40 bytes)
CLUSTER_DTYPE = np.dtype([("sample", "<i4"), ("dm_idx", "<u4"), ("width", "<u4"), ("snr", "<f4"),
                          ("members", "<u4"), ("sample_lo", "<i4"), ("sample_hi", "<i4"), ("dm_lo", "<u4"),
                          ("dm_hi", "<u4"), ("reserved", "<u4")])

# (name, restype, argtypes) of every exported entry point declared in include/sps.h
_P = ctypes.c_void_p
EXPORTS = [
    ("sps_plan_create", _P, [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_float]),
    ("sps_plan_destroy", None, [_P]),
    ("sps_search", ctypes.c_int, [_P, _P, _P, _P, _P]),
    ("sps_search_noalloc", ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_float, _P, _P, _P, _P, ctypes.c_int64]),
    ("sps_block_stats", ctypes.c_int, [_P, _P, _P, _P, _P]),
    ("sps_width_stats", ctypes.c_int, [_P, _P, _P, _P, _P]),
    ("sps_search_plain", ctypes.c_int, [_P, _P, _P, _P, _P]),
    ("sps_plan_set", ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int64]),
    ("sps_plan_get", ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_int64)]),
    ("sps_timing_read", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
    ("sps_stream_create", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_void_p)]),
    ("sps_stream_push", ctypes.c_int, [_P, _P, _P, _P, _P, ctypes.POINTER(ctypes.c_int64)]),
    ("sps_stream_push_graph", ctypes.c_int, [_P, _P, _P, _P, _P, ctypes.POINTER(ctypes.c_int64)]),
    ("sps_stream_flush", ctypes.c_int, [_P, _P, _P, _P, ctypes.POINTER(ctypes.c_int64)]),
    ("sps_stream_state_size", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_uint64)]),
    ("sps_stream_save", ctypes.c_int, [_P, _P, _P, ctypes.c_uint64]),
    ("sps_stream_restore", ctypes.c_int, [_P, _P, _P, ctypes.c_uint64]),
    ("sps_stream_destroy", None, [_P]),
    ("sps_domain_bound", ctypes.c_int64, [ctypes.c_int32]),
    ("sps_footprint", ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_uint64)]),
    ("sps_batch_create", ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p)]),
    ("sps_batch_set", ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int64]),
    ("sps_batch_search", ctypes.c_int, [_P, _P, ctypes.c_int32, _P]),
    ("sps_batch_push", ctypes.c_int, [_P, _P, _P, ctypes.c_int32, _P, _P, _P, _P]),
    ("sps_batch_destroy", None, [_P]),
    ("sps_cluster_create", _P, [ctypes.c_uint32]),
    ("sps_cluster_run", ctypes.c_int, [_P, _P, ctypes.c_uint32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, _P,
                                       _P]),
    ("sps_cluster_destroy", None, [_P]),
    ("sps_dedisp_delays", ctypes.c_int, [ctypes.c_int32, _P, ctypes.c_double, ctypes.c_double, ctypes.c_int32, _P, _P]),
    ("sps_dedisp_create", _P, [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, _P]),
    ("sps_dedisp_nsamp_out", ctypes.c_int64, [_P]),
    ("sps_dedisp_run", ctypes.c_int, [_P, _P, _P, _P]),
    ("sps_dedisp_destroy", None, [_P]),
    ("sps_zero_dm", ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, _P, _P]),
    ("sps_chan_mask", ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, _P, _P, _P]),
    ("sps_last_error", ctypes.c_int, []),
    ("sps_error_string", ctypes.c_char_p, [ctypes.c_int]),
]

_lib = None


class SpsError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__("%s failed: %s (%d)" % (what, error_string(code), code))


def load() -> ctypes.CDLL:
    """Load the in-tree libsps.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libsps.so is not built (run `python -m paper_2512_00398_amd.build`)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, res, args in EXPORTS:
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def error_string(code: int) -> str:
    return load().sps_error_string(int(code)).decode()


def _stream_handle(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _check_series(x, ndm: int, nsamp: int):
    import torch
    if not isinstance(x, torch.Tensor) or not x.is_cuda or x.dtype != torch.float32:
        raise TypeError("series must be a float32 tensor on the GPU")
    if tuple(x.shape) != (ndm, nsamp) or not x.is_contiguous():
        raise ValueError("series must be contiguous [%d][%d]" % (ndm, nsamp))


class Plan:
    """A search plan for blocks of ndm x nsamp samples (see include/sps.h)."""

    def __init__(self, ndm: int, nsamp: int, max_width: int, baseline_len: int, snr_thresh: float):
        lib = load()
        self._h = lib.sps_plan_create(int(ndm), int(nsamp), int(max_width), int(baseline_len),
                                      float(snr_thresh))
        if not self._h:
            raise SpsError(lib.sps_last_error(), "sps_plan_create")
        self.ndm, self.nsamp = int(ndm), int(nsamp)
        self.max_width, self.baseline_len, self.snr_thresh = int(max_width), int(baseline_len), float(snr_thresh)

    # -- attributes
    def set(self, attr: int, value: int) -> None:
        rc = load().sps_plan_set(self._h, int(attr), int(value))
        if rc:
            raise SpsError(rc, "sps_plan_set")

    def get(self, attr: int) -> int:
        v = ctypes.c_int64()
        rc = load().sps_plan_get(self._h, int(attr), ctypes.byref(v))
        if rc:
            raise SpsError(rc, "sps_plan_get")
        return int(v.value)

    @property
    def nblocks(self) -> int:
        return self.get(ATTR_NBLOCKS)

    @property
    def max_cands(self) -> int:
        return self.get(ATTR_MAX_CANDS)

    # -- buffers
    def alloc_cands(self, capacity: Optional[int] = None):
        import torch
        cap = self.max_cands if capacity is None else int(capacity)
        if capacity is not None and cap != self.max_cands:
            self.set(ATTR_MAX_CANDS, cap)
        cands = torch.empty((max(cap, 1), 4), dtype=torch.int32, device="cuda")
        ncand = torch.zeros(1, dtype=torch.int32, device="cuda")
        return cands, ncand

    # -- entry points
    def search(self, series, cands=None, ncand=None, stream=None, plain: bool = False):
        """Enqueue a search; returns the (cands, ncand) device tensors."""
        _check_series(series, self.ndm, self.nsamp)
        if cands is None or ncand is None:
            cands, ncand = self.alloc_cands()
        if cands.shape[0] < self.max_cands:
            raise ValueError("candidate buffer smaller than the plan's capacity")
        fn = load().sps_search_plain if plain else load().sps_search
        rc = fn(self._h, series.data_ptr(), _stream_handle(stream), cands.data_ptr(), ncand.data_ptr())
        if rc:
            raise SpsError(rc, "sps_search_plain" if plain else "sps_search")
        return cands, ncand

    def block_stats(self, series, med=None, mad=None, stream=None):
        import torch
        _check_series(series, self.ndm, self.nsamp)
        nb = self.nblocks
        if med is None:
            med = torch.empty((self.ndm, nb), dtype=torch.int32, device="cuda")
        if mad is None:
            mad = torch.empty((self.ndm, nb), dtype=torch.int32, device="cuda")
        rc = load().sps_block_stats(self._h, series.data_ptr(), _stream_handle(stream), med.data_ptr(),
                                    mad.data_ptr())
        if rc:
            raise SpsError(rc, "sps_block_stats")
        return med, mad

    def width_stats(self, series, center=None, mad=None, stream=None):
        """Per-width statistics (sps_width_stats): int32 [ndm][nwidths] medians c_w and MADs of
        the boxcar-filtered series."""
        import torch
        _check_series(series, self.ndm, self.nsamp)
        nw = self.get(ATTR_NWIDTHS)
        if center is None:
            center = torch.empty((self.ndm, nw), dtype=torch.int32, device="cuda")
        if mad is None:
            mad = torch.empty((self.ndm, nw), dtype=torch.int32, device="cuda")
        rc = load().sps_width_stats(self._h, series.data_ptr(), _stream_handle(stream), center.data_ptr(),
                                    mad.data_ptr())
        if rc:
            raise SpsError(rc, "sps_width_stats")
        return center, mad

    def timing_read(self):
        """Summed ms per stage since the last read, and the number of searches (waits for the events)."""
        ms = (ctypes.c_double * NSTAGES)()
        n = ctypes.c_int64()
        rc = load().sps_timing_read(self._h, ms, ctypes.byref(n))
        if rc:
            raise SpsError(rc, "sps_timing_read")
        return dict(zip(STAGES, list(ms))), int(n.value)

    def close(self) -> None:
        if getattr(self, "_h", None):
            load().sps_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Stream:
    """Gulp-by-gulp search of one observation (see include/sps.h)."""

    def __init__(self, plan: Plan):
        self.plan = plan
        h = ctypes.c_void_p()
        rc = load().sps_stream_create(plan._h, ctypes.byref(h))
        if rc:
            raise SpsError(rc, "sps_stream_create")
        self._h = h.value

    def push(self, gulp, cands, ncand, stream=None, graph: bool = False) -> int:
        """Enqueue one gulp; returns the global index of its first sample.

        graph=True replays a captured HIP graph of the gulp step (pass the
        same gulp/cands/ncand buffers each time)."""
        _check_series(gulp, self.plan.ndm, self.plan.nsamp)
        off = ctypes.c_int64()
        fn = load().sps_stream_push_graph if graph else load().sps_stream_push
        rc = fn(self._h, gulp.data_ptr(), _stream_handle(stream), cands.data_ptr(), ncand.data_ptr(),
                ctypes.byref(off))
        if rc:
            raise SpsError(rc, "sps_stream_push_graph" if graph else "sps_stream_push")
        return int(off.value)

    def flush(self, cands, ncand, stream=None) -> int:
        """Emit the runs still open; returns the number of samples pushed."""
        off = ctypes.c_int64()
        rc = load().sps_stream_flush(self._h, _stream_handle(stream), cands.data_ptr(), ncand.data_ptr(),
                                     ctypes.byref(off))
        if rc:
            raise SpsError(rc, "sps_stream_flush")
        return int(off.value)

    def save(self, stream=None) -> bytes:
        n = ctypes.c_uint64()
        rc = load().sps_stream_state_size(self._h, ctypes.byref(n))
        if rc:
            raise SpsError(rc, "sps_stream_state_size")
        buf = ctypes.create_string_buffer(int(n.value))
        rc = load().sps_stream_save(self._h, _stream_handle(stream), buf, n.value)
        if rc:
            raise SpsError(rc, "sps_stream_save")
        return buf.raw

    def restore(self, state: bytes, stream=None) -> None:
        buf = ctypes.create_string_buffer(state, len(state))
        rc = load().sps_stream_restore(self._h, _stream_handle(stream), buf, len(state))
        if rc:
            raise SpsError(rc, "sps_stream_restore")

    def close(self) -> None:
        if getattr(self, "_h", None):
            load().sps_stream_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def domain_bound(max_width: int) -> int:
    """Largest |sample| the search accepts for this max_width (include/sps.h)."""
    return int(load().sps_domain_bound(int(max_width)))


def footprint(ndm: int, nsamp: int, max_width: int, baseline_len: int, streaming: bool = False) -> int:
    """Device bytes a plan (and a stream on it) of this shape holds; no device needed."""
    v = ctypes.c_uint64()
    rc = load().sps_footprint(int(ndm), int(nsamp), int(max_width), int(baseline_len), int(bool(streaming)),
                              ctypes.byref(v))
    if rc:
        raise SpsError(rc, "sps_footprint")
    return int(v.value)


class BatchItem(ctypes.Structure):
    """sps_batch_item (include/sps.h)."""
    _fields_ = [("d_series", ctypes.c_void_p), ("ndm", ctypes.c_int32), ("max_width", ctypes.c_int32),
                ("nsamp", ctypes.c_int64), ("baseline_len", ctypes.c_int32), ("snr_thresh", ctypes.c_float),
                ("d_cands", ctypes.c_void_p), ("d_ncand", ctypes.c_void_p), ("max_cands", ctypes.c_int64)]


assert ctypes.sizeof(BatchItem) == 56


class Batch:
    """Many independent blocks searched by one persistent launch per stage (see include/sps.h)."""

    def __init__(self):
        h = ctypes.c_void_p()
        rc = load().sps_batch_create(ctypes.byref(h))
        if rc:
            raise SpsError(rc, "sps_batch_create")
        self._h = h.value

    def set(self, attr: int, value: int) -> None:
        rc = load().sps_batch_set(self._h, int(attr), int(value))
        if rc:
            raise SpsError(rc, "sps_batch_set")

    def search(self, items, stream=None) -> None:
        """items: sequence of (series, max_width, baseline_len, snr_thresh, cands, ncand).

        series is a contiguous float32 [ndm][nsamp] GPU tensor; cands an
        int32 [capacity][4] GPU tensor (capacity = its first dimension);
        ncand an int32 GPU tensor of one element."""
        arr = (BatchItem * max(1, len(items)))()
        for k, (x, w, L, th, cands, ncand) in enumerate(items):
            ndm, nsamp = x.shape
            _check_series(x, ndm, nsamp)
            arr[k] = BatchItem(x.data_ptr(), int(ndm), int(w), int(nsamp), int(L), float(th),
                               cands.data_ptr(), ncand.data_ptr(), int(cands.shape[0]))
        rc = load().sps_batch_search(self._h, ctypes.cast(arr, ctypes.c_void_p), len(items), _stream_handle(stream))
        if rc:
            raise SpsError(rc, "sps_batch_search")

    def push(self, streams, gulps, cands, ncands, stream=None):
        """One gulp of each of several distinct Streams in one persistent launch
        per stage (sps_batch_push); returns each gulp's global first-sample index.
        gulps: float32 GPU tensors of each stream's gulp shape; cands / ncands:
        each stream's candidate buffers (int32 [capacity][4], int32 [1])."""
        n = len(streams)
        if not (len(gulps) == len(cands) == len(ncands) == n):
            raise ValueError("one gulp and one candidate buffer pair per stream")
        for st, g in zip(streams, gulps):
            _check_series(g, st.plan.ndm, st.plan.nsamp)
        P = ctypes.c_void_p * max(1, n)
        hs = P(*[st._h for st in streams])
        gs = P(*[g.data_ptr() for g in gulps])
        cs = P(*[c.data_ptr() for c in cands])
        ns = P(*[c.data_ptr() for c in ncands])
        offs = (ctypes.c_int64 * max(1, n))()
        rc = load().sps_batch_push(self._h, hs, gs, n, _stream_handle(stream), cs, ns, offs)
        if rc:
            raise SpsError(rc, "sps_batch_push")
        return [int(offs[i]) for i in range(n)]

    def close(self) -> None:
        if getattr(self, "_h", None):
            load().sps_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def cands_to_numpy(cands, ncand, capacity: Optional[int] = None) -> np.ndarray:
    """Copy the first ncand records to a structured array sorted (dm, width, sample).

    Raises SpsError(SPS_ERR_OVERFLOW) if the true count exceeds the capacity.
    """
    n = int(ncand.item()) & 0xFFFFFFFF
    cap = cands.shape[0] if capacity is None else int(capacity)
    if n > cap:
        raise SpsError(SPS_ERR_OVERFLOW, "search (%d candidates, capacity %d)" % (n, cap))
    a = cands[:n].cpu().numpy().view(CAND_DTYPE).reshape(-1)
    if a.size:
        a = a[np.lexsort((a["sample"], a["width"], a["dm_idx"]))]
    return a


def search(series, max_width: int, baseline_len: int, snr_thresh: float, capacity: Optional[int] = None,
           plain: bool = False) -> np.ndarray:
    """One-shot convenience: plan, search on the current stream, return sorted candidates."""
    import torch
    ndm, nsamp = series.shape
    with Plan(ndm, nsamp, max_width, baseline_len, snr_thresh) as p:
        if capacity is not None:
            p.set(ATTR_MAX_CANDS, capacity)
        cands, ncand = p.alloc_cands()
        p.search(series, cands, ncand, plain=plain)
        torch.cuda.synchronize()
        return cands_to_numpy(cands, ncand, p.max_cands)


def search_noalloc(series, max_width: int, baseline_len: int, snr_thresh: float, cands, ncand, stream=None):
    """The search without a plan and without allocating device memory
    (sps_search_noalloc): scratch from the library's fixed per-GPU array.
    cands is an int32 [capacity][4] GPU tensor, ncand an int32 [1] GPU tensor."""
    ndm, nsamp = series.shape
    _check_series(series, ndm, nsamp)
    rc = load().sps_search_noalloc(int(ndm), int(nsamp), int(max_width), int(baseline_len), float(snr_thresh),
                                   series.data_ptr(), _stream_handle(stream), cands.data_ptr(), ncand.data_ptr(),
                                   int(cands.shape[0]))
    if rc:
        raise SpsError(rc, "sps_search_noalloc")
    return cands, ncand


class Clusterer:
    """Candidate merging and clustering on the GPU (see include/sps.h)."""

    def __init__(self, max_cands: int):
        lib = load()
        self.max_cands = int(max_cands)
        self._h = lib.sps_cluster_create(self.max_cands)
        if not self._h:
            raise SpsError(lib.sps_last_error(), "sps_cluster_create")

    def alloc_out(self, n: Optional[int] = None):
        """Output records (int32 [n][10] GPU tensor) and their count (int32 [1])."""
        import torch
        n = self.max_cands if n is None else int(n)
        return (torch.empty((max(1, n), 10), dtype=torch.int32, device="cuda"),
                torch.zeros((1,), dtype=torch.int32, device="cuda"))

    def run(self, cands, n: int, time_tol: int, dm_tol: int, width_tol: int, out, nout, stream=None) -> None:
        """Cluster the first n records of cands (int32 [capacity][4] GPU tensor) into out / nout."""
        if int(n) > cands.shape[0] or int(n) > out.shape[0]:
            raise ValueError("n exceeds the candidate or output capacity")
        rc = load().sps_cluster_run(self._h, cands.data_ptr(), int(n), int(time_tol), int(dm_tol), int(width_tol),
                                    _stream_handle(stream), out.data_ptr(), nout.data_ptr())
        if rc:
            raise SpsError(rc, "sps_cluster_run")

    def close(self) -> None:
        if getattr(self, "_h", None):
            load().sps_cluster_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def dedisp_delays(freqs_mhz, f_ref_mhz: float, tsamp_s: float, dms) -> np.ndarray:
    """Per-channel dispersion delays in samples, int32 [ndm][nchan] (sps_dedisp_delays)."""
    f = np.ascontiguousarray(freqs_mhz, dtype=np.float64)
    d = np.ascontiguousarray(dms, dtype=np.float32)
    out = np.empty((d.size, f.size), dtype=np.int32)
    rc = load().sps_dedisp_delays(f.size, f.ctypes.data, float(f_ref_mhz), float(tsamp_s), d.size, d.ctypes.data,
                                  out.ctypes.data)
    if rc:
        raise SpsError(rc, "sps_dedisp_delays")
    return out


def zero_dm(fil, offset: int, out=None, stream=None):
    """Broadband (zero-DM) RFI excision of a uint8 GPU filterbank [nchan][nsamp]
    (sps_zero_dm); out may be fil itself (in place) or a new tensor."""
    import torch
    if fil.dtype != torch.uint8 or fil.dim() != 2 or not fil.is_contiguous():
        raise ValueError("filterbank must be a contiguous uint8 GPU tensor [nchan][nsamp]")
    if out is None:
        out = torch.empty_like(fil)
    if out.dtype != torch.uint8 or out.shape != fil.shape or not out.is_contiguous():
        raise ValueError("out must match the filterbank")
    rc = load().sps_zero_dm(fil.data_ptr(), fil.shape[0], fil.shape[1], int(offset), _stream_handle(stream),
                            out.data_ptr())
    if rc:
        raise SpsError(rc, "sps_zero_dm")
    return out


def chan_mask(fil, k: int, out=None, stats=None, stream=None):
    """Narrowband RFI excision of a uint8 GPU filterbank [nchan][nsamp]
    (sps_chan_mask); returns (out, stats) with stats uint8 [nchan][3] =
    (median, MAD, flag) per channel. out may be fil itself (in place)."""
    import torch
    if fil.dtype != torch.uint8 or fil.dim() != 2 or not fil.is_contiguous():
        raise ValueError("filterbank must be a contiguous uint8 GPU tensor [nchan][nsamp]")
    if out is None:
        out = torch.empty_like(fil)
    if out.dtype != torch.uint8 or out.shape != fil.shape or not out.is_contiguous():
        raise ValueError("out must match the filterbank")
    if stats is None:
        stats = torch.empty((fil.shape[0], 3), dtype=torch.uint8, device=fil.device)
    rc = load().sps_chan_mask(fil.data_ptr(), fil.shape[0], fil.shape[1], int(k), _stream_handle(stream),
                              out.data_ptr(), stats.data_ptr())
    if rc:
        raise SpsError(rc, "sps_chan_mask")
    return out, stats


class Dedisperser:
    """Incoherent dedispersion on the GPU (see include/sps.h): an 8-bit
    channel-major filterbank [nchan][nsamp_in] to FP32 [ndm][nsamp_out]."""

    def __init__(self, nchan: int, nsamp_in: int, delays):
        lib = load()
        tab = np.ascontiguousarray(delays, dtype=np.int32)
        if tab.ndim != 2 or tab.shape[1] != nchan:
            raise ValueError("delays must be int32 [ndm][nchan]")
        self.nchan, self.nsamp_in, self.ndm = int(nchan), int(nsamp_in), int(tab.shape[0])
        self._h = lib.sps_dedisp_create(self.nchan, self.nsamp_in, self.ndm, tab.ctypes.data)
        if not self._h:
            raise SpsError(lib.sps_last_error(), "sps_dedisp_create")
        self.nsamp_out = int(lib.sps_dedisp_nsamp_out(self._h))

    def alloc_out(self):
        import torch
        return torch.empty((self.ndm, self.nsamp_out), dtype=torch.float32, device="cuda")

    def run(self, fil, out=None, stream=None):
        """Dedisperse fil (uint8 GPU tensor [nchan][nsamp_in]) into out (FP32 [ndm][nsamp_out])."""
        import torch
        if fil.dtype != torch.uint8 or tuple(fil.shape) != (self.nchan, self.nsamp_in) or not fil.is_contiguous():
            raise ValueError("filterbank must be a contiguous uint8 GPU tensor [nchan][nsamp_in]")
        if out is None:
            out = self.alloc_out()
        if out.dtype != torch.float32 or tuple(out.shape) != (self.ndm, self.nsamp_out) or not out.is_contiguous():
            raise ValueError("out must be a contiguous float32 GPU tensor [ndm][nsamp_out]")
        rc = load().sps_dedisp_run(self._h, fil.data_ptr(), _stream_handle(stream), out.data_ptr())
        if rc:
            raise SpsError(rc, "sps_dedisp_run")
        return out

    def close(self) -> None:
        if getattr(self, "_h", None):
            load().sps_dedisp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def clusters_to_numpy(out, nout) -> np.ndarray:
    """Copy the cluster records to a structured array sorted (dm, width, sample) of their best member."""
    n = int(nout.item()) & 0xFFFFFFFF
    a = out[:n].cpu().numpy().view(CLUSTER_DTYPE).reshape(-1)
    if a.size:
        a = a[np.lexsort((a["sample"], a["width"], a["dm_idx"]))]
    return a
