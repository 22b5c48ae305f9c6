"""Autotuner for the speed-only attributes of a search plan.

The tuned attributes are the baseline kernel's chain length
(ATTR_STATS_SEG, in blocks), the detection segment length (ATTR_DETECT_SEG, in
samples) and the histogram span of the baseline kernel (ATTR_HIST_BINS). None
of them changes a result: before a configuration is recorded the tuner checks
that its candidate set is the one the default configuration returns (count
and an order-independent 64-bit digest of the records), and it raises if not.

Results are kept in a JSON file keyed by GPU architecture and shape class
(ndm and nsamp rounded up to powers of two, max_width, baseline_len). The file
is SPS_AUTOTUNE_CACHE if set, else ~/.cache/sps/autotune.json.

A batch of blocks (sps_batch_search) is tuned the same way as a whole: the
same three attributes, and whether statistics and detection share one
persistent launch, apply to every item; every configuration must return
every item's candidate set unchanged, and the result is cached under the
multiset of the items' shape classes. The fused kernels evaluate every width
in one pass over the samples, so there is no widths-per-pass attribute.
"""
from __future__ import annotations

import json
import os
import tempfile
import time
from typing import Dict, List, Optional

import numpy as np

from . import sps

CACHE_ENV = "SPS_AUTOTUNE_CACHE"
ATTRS = {"stats_seg": sps.ATTR_STATS_SEG, "detect_seg": sps.ATTR_DETECT_SEG, "hist_bins": sps.ATTR_HIST_BINS,
         "fused": sps.ATTR_FUSED}
DEFAULT = {"stats_seg": 0, "detect_seg": 0, "hist_bins": 4096}
BATCH_DEFAULT = {"stats_seg": 0, "detect_seg": 0, "hist_bins": 4096, "fused": 1}


def _pow2ceil(v: int) -> int:
    v = max(1, int(v))
    return 1 << (v - 1).bit_length()


def shape_key(arch: str, ndm: int, nsamp: int, max_width: int, baseline_len: int) -> str:
    return "%s|ndm%d|n%d|w%d|L%d" % (arch, _pow2ceil(ndm), _pow2ceil(nsamp), int(max_width), int(baseline_len))


def cache_path(path: Optional[str] = None) -> str:
    if path:
        return path
    env = os.environ.get(CACHE_ENV)
    if env:
        return env
    return os.path.join(os.path.expanduser("~"), ".cache", "sps", "autotune.json")


def load_cache(path: Optional[str] = None) -> Dict[str, dict]:
    p = cache_path(path)
    if not os.path.exists(p):
        return {}
    with open(p) as f:
        data = json.load(f)
    if not isinstance(data, dict):
        raise ValueError("autotune cache %s is not a JSON object" % p)
    return data


def save_cache(data: Dict[str, dict], path: Optional[str] = None) -> str:
    """Write the cache atomically (temporary file + rename)."""
    p = cache_path(path)
    os.makedirs(os.path.dirname(p) or ".", exist_ok=True)
    fd, tmp = tempfile.mkstemp(prefix=".autotune.", dir=os.path.dirname(p) or ".")
    with os.fdopen(fd, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, p)
    return p


def candidate_configs(ndm: int, nsamp: int, max_width: int, baseline_len: int) -> Dict[str, List[int]]:
    """Values tried per attribute (0 = the library's own choice)."""
    nblocks = (nsamp + sps.BLOCK_STRIDE - 1) // sps.BLOCK_STRIDE
    min_chain = max(64, (4 * baseline_len + 63) // 64)
    stats = [0] + [s for s in (256, 512, 1024, 2048, 4096, 8192, 16384) if min_chain // 2 <= s < nblocks]
    npos = (nsamp + 1023) // 1024 * 1024
    detect = [0] + [s for s in (16384, 32768, 65536, 131072, 262144, 524288)
                    if s >= 4 * max_width and s < npos]
    return {"stats_seg": stats, "detect_seg": detect, "hist_bins": [4096, 16384]}


def digest(cands: np.ndarray) -> int:
    """Order-independent 64-bit digest of candidate records (sum of mixed words)."""
    if cands.size == 0:
        return 0
    w = np.ascontiguousarray(cands).view(np.uint32).reshape(-1, 4).astype(np.uint64)
    with np.errstate(over="ignore"):
        h = (w[:, 0] * np.uint64(0x9E3779B97F4A7C15) ^ w[:, 1] * np.uint64(0xC2B2AE3D27D4EB4F)
             ^ w[:, 2] * np.uint64(0x165667B19E3779F9) ^ w[:, 3] * np.uint64(0xD6E8FEB86659FD93))
        h ^= h >> np.uint64(29)
        h *= np.uint64(0xBF58476D1CE4E5B9)
        h ^= h >> np.uint64(32)
        return int(h.sum(dtype=np.uint64))


def gpu_arch() -> str:
    import torch
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    return str(getattr(props, "gcnArchName", props.name)).split(":")[0]


def _apply(plan: sps.Plan, cfg: dict) -> None:
    for k, v in cfg.items():
        plan.set(ATTRS[k], int(v))


def _measure(plan: sps.Plan, series, cands, ncand, stream, steps: int):
    import torch
    plan.search(series, cands, ncand, stream=stream)
    torch.cuda.synchronize()
    n = int(ncand.item()) & 0xFFFFFFFF
    if n > plan.max_cands:
        raise sps.SpsError(sps.SPS_ERR_OVERFLOW, "autotune search")
    d = digest(cands[:n].cpu().numpy())
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        plan.search(series, cands, ncand, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps, (n, d)


def tune(plan: sps.Plan, series, stream=None, steps: int = 3, path: Optional[str] = None,
         arch: Optional[str] = None, log=None) -> dict:
    """Coordinate search over the tuning attributes on `series`; records and applies the best.

    Returns {"config": {...}, "ms": best, "default_ms": ..., "key": ...}."""
    import torch
    stream = torch.cuda.current_stream() if stream is None else stream
    arch = arch or gpu_arch()
    key = shape_key(arch, plan.ndm, plan.nsamp, plan.max_width, plan.baseline_len)
    cands, ncand = plan.alloc_cands()
    best = dict(DEFAULT)
    _apply(plan, best)
    best_ms, ref = _measure(plan, series, cands, ncand, stream, steps)
    default_ms = best_ms
    tried = 1
    for attr, values in candidate_configs(plan.ndm, plan.nsamp, plan.max_width, plan.baseline_len).items():
        for v in values:
            if v == best[attr]:
                continue
            cfg = dict(best)
            cfg[attr] = v
            _apply(plan, cfg)
            ms, res = _measure(plan, series, cands, ncand, stream, steps)
            tried += 1
            if res != ref:
                raise RuntimeError("tuning %s changed the result (%s vs %s)" % (cfg, res, ref))
            if log:
                log("autotune %s: %.3f ms" % (cfg, ms))
            if ms < best_ms:
                best_ms, best = ms, cfg
    _apply(plan, best)
    data = load_cache(path)
    data[key] = {"config": best, "ms": best_ms, "default_ms": default_ms, "tried": tried,
                 "when": time.strftime("%Y-%m-%dT%H:%M:%S")}
    save_cache(data, path)
    return {"key": key, "config": best, "ms": best_ms, "default_ms": default_ms, "tried": tried}


def lookup(ndm: int, nsamp: int, max_width: int, baseline_len: int, arch: str,
           path: Optional[str] = None) -> Optional[dict]:
    ent = load_cache(path).get(shape_key(arch, ndm, nsamp, max_width, baseline_len))
    if not ent:
        return None
    cfg = ent.get("config", {})
    if set(cfg) - set(ATTRS):
        raise ValueError("autotune cache entry has unknown attributes: %s" % sorted(cfg))
    return cfg


def apply(plan: sps.Plan, path: Optional[str] = None, arch: Optional[str] = None) -> Optional[dict]:
    """Set the cached configuration for this plan's shape class, if any; returns it."""
    cfg = lookup(plan.ndm, plan.nsamp, plan.max_width, plan.baseline_len, arch or gpu_arch(), path)
    if cfg:
        _apply(plan, cfg)
    return cfg


def batch_key(arch: str, shapes) -> str:
    """Cache key of a batch: the sorted multiset of its items' shape classes.
    shapes: (ndm, nsamp, max_width, baseline_len) per item."""
    classes = {}
    for ndm, nsamp, w, L in shapes:
        k = shape_key(arch, ndm, nsamp, w, L).split("|", 1)[1]
        classes[k] = classes.get(k, 0) + 1
    return "%s|batch|%s" % (arch, ";".join("%dx%s" % (classes[k], k) for k in sorted(classes)))


def batch_candidate_configs(shapes) -> Dict[str, List[int]]:
    """Values tried for a batch: chain lengths and detection segments that fit its items."""
    nb_max = max((n + sps.BLOCK_STRIDE - 1) // sps.BLOCK_STRIDE for _, n, _, _ in shapes)
    min_chain = max(max(64, (4 * L + 63) // 64) for _, _, _, L in shapes)
    stats = [0] + [s for s in (256, 512, 1024, 2048, 4096, 8192) if min_chain // 2 <= s < nb_max]
    wmax = max(w for _, _, w, _ in shapes)
    nmax = max(n for _, n, _, _ in shapes)
    detect = [0] + [s for s in (16384, 32768, 65536, 131072, 262144) if s >= 4 * wmax and s < nmax]
    return {"stats_seg": stats, "detect_seg": detect, "hist_bins": [4096, 16384], "fused": [1, 0]}


def _batch_apply(batch: sps.Batch, cfg: dict) -> None:
    for k, v in cfg.items():
        batch.set(ATTRS[k], int(v))


def _batch_measure(batch: sps.Batch, items, stream, steps: int):
    import torch
    batch.search(items, stream=stream)
    torch.cuda.synchronize()
    res = []
    for (x, w, L, th, cands, ncand) in items:
        n = int(ncand.item()) & 0xFFFFFFFF
        if n > cands.shape[0]:
            raise sps.SpsError(sps.SPS_ERR_OVERFLOW, "autotune batch")
        res.append((n, digest(cands[:n].cpu().numpy())))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        batch.search(items, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps, tuple(res)


def tune_batch(batch: sps.Batch, items, stream=None, steps: int = 2, path: Optional[str] = None,
               arch: Optional[str] = None, log=None) -> dict:
    """Coordinate search over the batch's tuning attributes on `items` (the
    sps.Batch.search item tuples); records and applies the best. Every
    configuration must return each item's candidates unchanged."""
    import torch
    stream = torch.cuda.current_stream() if stream is None else stream
    arch = arch or gpu_arch()
    shapes = [(int(x.shape[0]), int(x.shape[1]), int(w), int(L)) for (x, w, L, _, _, _) in items]
    key = batch_key(arch, shapes)
    best = dict(BATCH_DEFAULT)
    _batch_apply(batch, best)
    best_ms, ref = _batch_measure(batch, items, stream, steps)
    default_ms = best_ms
    tried = 1
    for attr, values in batch_candidate_configs(shapes).items():
        for v in values:
            if v == best[attr]:
                continue
            cfg = dict(best)
            cfg[attr] = v
            _batch_apply(batch, cfg)
            ms, res = _batch_measure(batch, items, stream, steps)
            tried += 1
            if res != ref:
                raise RuntimeError("tuning %s changed a batch result" % cfg)
            if log:
                log("autotune batch %s: %.3f ms" % (cfg, ms))
            if ms < best_ms:
                best_ms, best = ms, cfg
    _batch_apply(batch, best)
    data = load_cache(path)
    data[key] = {"config": best, "ms": best_ms, "default_ms": default_ms, "tried": tried,
                 "when": time.strftime("%Y-%m-%dT%H:%M:%S")}
    save_cache(data, path)
    return {"key": key, "config": best, "ms": best_ms, "default_ms": default_ms, "tried": tried}


def apply_batch(batch: sps.Batch, shapes, path: Optional[str] = None, arch: Optional[str] = None) -> Optional[dict]:
    """Set the cached configuration for this batch's multiset of shape classes, if any; returns it."""
    ent = load_cache(path).get(batch_key(arch or gpu_arch(), shapes))
    if not ent:
        return None
    cfg = ent.get("config", {})
    if set(cfg) - set(ATTRS):
        raise ValueError("autotune cache entry has unknown attributes: %s" % sorted(cfg))
    _batch_apply(batch, cfg)
    return cfg
