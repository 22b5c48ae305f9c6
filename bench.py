"""Throughput of the per-DM-trial single-pulse search on one MI355X.

A step is one full search (baseline + MAD normalisation + boxcar matched
filter at every width + threshold + run-based peak detection + candidate
compaction) of the single-large-file workload: 1024 DM trials x 2^20 samples,
widths 1..4096, baseline window 16384, threshold 6. Inputs are synthetic
(seeded, integer-valued noise + drift + pulses + zero-DM RFI) and resident in
HBM before the timed region. Prints one JSON line.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 1|2]
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
# 32-bit integer vector adds: 256 CUs x 64 lanes per clock x 2.4 GHz
ALU_INT32_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# the dedispersion kernel adds packed pairs of 16-bit sums: one 32-bit add
# retires two sample additions, so its attainable rate is twice the int32 rate
ALU_PAIR_ADD_PEAK_TOPS = 2 * ALU_INT32_PEAK_TOPS

# HBM bytes per launch on the default workload, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (KiB per dispatch) scaled by what the same counters read for a
# 1 GiB device copy (fetch x 2.000, write x 1.000); the command lines and raw
# figures are in profiles/. A figure is reported only while the code it was
# measured on is unchanged (hash of the files below without their comments),
# else null.
_CSRC = "paper_2512_00398_amd/csrc/"
KERNEL_SOURCES = {
    "detect": [_CSRC + "sps_detect.hip", _CSRC + "sps_detect_body.h", _CSRC + "sps_runs.h", _CSRC + "sps_wave.h",
               _CSRC + "sps_internal.h", _CSRC + "sps_api.hip", "include/sps.h"],
    "block_stats": [_CSRC + "sps_stats.hip", _CSRC + "sps_chain.h", _CSRC + "sps_wave.h", _CSRC + "sps_internal.h",
                    _CSRC + "sps_api.hip", "include/sps.h"],
    "dedisp": [_CSRC + "sps_dedisp.hip", _CSRC + "sps_internal.h", _CSRC + "sps_api.hip", "include/sps.h"],
}
MEASURED_TRAFFIC = {
    # kernel: (sources hash, bytes per launch); profiles/kernels_c2_1024x2p20.md,
    # profiles/dedisp_1024ch_1024dm_2p18.md
    "detect": ("28cb64f53eaf4840", (2237782 * 2 + 170188) * 1024),
    "block_stats": ("83db0f9652526326", (4349769 * 2 + 137136) * 1024),
    "dedisp": ("ba24418b892897af", (3431724 * 2 + 1048576) * 1024),
}


# VALU wave-instructions per launch on the default workload, from rocprofv3
# SQ_INSTS_VALU (profiles/); reported only while the sources are unchanged.
VALU_ISSUE_PER_S = 256 * 2.4e9
MEASURED_VALU = {
    # kernel: (sources hash, SQ_INSTS_VALU per launch); profiles/kernels_c2_1024x2p20.md
    "detect": ("28cb64f53eaf4840", 3.311e9),
    "block_stats": ("83db0f9652526326", 1.875e9),
}


def measured_issue(kernel: str):
    ent = MEASURED_VALU.get(kernel)
    if not ent or ent[0] != sources_hash(kernel):
        return None
    return ent[1]


def sources_hash(kernel: str) -> str:
    """Hash of the kernel's sources with comments and whitespace removed (a
    comment cannot change the code the counters were taken on)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, f), "r", encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    ent = MEASURED_TRAFFIC.get(kernel)
    if not ent or ent[0] != sources_hash(kernel):
        return None
    return ent[1]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _oracle_row(args):
    """CPU-baseline worker: the oracle on one row of the workload (timed inside)."""
    cfg_index, row, centred, row_norm, width_norm = args
    import numpy as np  # noqa: F401
    import oracle
    import synth
    b = synth.config(cfg_index)["blocks"][0]
    x = synth.generate(b, rows=[row], nthreads=1)
    t0 = time.time()
    c = oracle.search(x, b.max_width, b.baseline_len, b.snr_thresh, centered=centred, row_norm=row_norm,
                      width_norm=width_norm)
    t1 = time.time()
    return t0, t1, int(c.size), b.nsamp


def host_cores() -> int:
    """Cores this process may run on (the affinity mask, not the machine's count)."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def cpu_baseline(cfg_index: int, nrows: int, centred: bool = False, row_norm: bool = False,
                 width_norm: bool = False):
    """The oracle on a bounded sample of whole DM rows, one process per core
    (at most 16, the host share of one GPU), timed as wall clock over the
    sample; the rate is samples of the sampled rows per second."""
    cores = host_cores()
    procs = max(1, min(16, cores, nrows))
    ndm = __import__("synth").config(cfg_index)["blocks"][0].ndm
    rows = [int(r * (ndm - 1) / max(1, nrows - 1)) for r in range(nrows)]
    ctx = mp.get_context("spawn")
    with ctx.Pool(procs) as pool:
        res = pool.map(_oracle_row, [(cfg_index, r, centred, row_norm, width_norm) for r in rows])
    span = max(r[1] for r in res) - min(r[0] for r in res)
    samples = sum(r[3] for r in res)
    return {"value": samples / span, "unit": "DM-trial-samples/s", "cores": procs, "host_cores": cores,
            "kind": "oracle",
            "sample": "%d of %d DM rows (whole 2^%d-sample rows), numpy oracle, one process per row on %d of the "
                      "%d host cores; rate over the sampled rows (the full block scales linearly in rows)" %
                      (nrows, ndm, (res[0][3]).bit_length() - 1, procs, cores),
            "cpu_seconds": round(sum(r[1] - r[0] for r in res), 2), "seconds": round(span, 3)}


def bench_stream(args):
    """Streaming workload: 4096 DM trials, gulps of 2^18 samples pushed one by
    one (history, block statistics and open runs carried on the device), each
    gulp step replayed from a captured HIP graph; eager pushes timed beside."""
    import torch
    import synth
    from paper_2512_00398_amd import sps

    cfg = synth.config(3)
    b = cfg["blocks"][0]
    gulp, ng = cfg["gulp"], cfg["ngulps"]
    gulps = []
    for k in range(ng):
        x = synth.generate(b, t0=k * gulp, nsamp=gulp)
        gulps.append(torch.from_numpy(x).cuda())
        del x
    log("generated %d gulps of %d x %d" % (ng, b.ndm, gulp))
    stream = torch.cuda.current_stream()
    plan = sps.Plan(b.ndm, gulp, b.max_width, b.baseline_len, b.snr_thresh)
    cb = [plan.alloc_cands() for _ in range(2)]

    def one_pass(st, graph):
        n = 0
        for k in range(ng):
            c, nc = cb[k % 2]
            st.push(gulps[k], c, nc, stream=stream, graph=graph)
            if k % 2 == 1:
                n += int(cb[0][1].item()) + int(cb[1][1].item())  # both slots are complete here
        return n

    res = {}
    for graph in (True, False):
        st = sps.Stream(plan)
        for _ in range(max(1, args.warmup)):
            one_pass(st, graph)  # captures the graphs on the first pass
        torch.cuda.synchronize()
        if not graph:
            plan.set(sps.ATTR_TIMING, 1)
            plan.timing_read()
        passes = max(1, args.steps // ng)
        t0 = time.perf_counter()
        ncand = 0
        for _ in range(passes):
            ncand += one_pass(st, graph)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if not graph:
            stages, nsearch = plan.timing_read()
            plan.set(sps.ATTR_TIMING, 0)
            res["stages_ms"] = {k: round(v / max(1, nsearch), 4) for k, v in stages.items() if k != "plain"}
        res["graph" if graph else "eager"] = {"ms_per_gulp": dt * 1e3 / (passes * ng), "gulps": passes * ng,
                                             "candidates": ncand}
        st.close()
        log("%s: %.3f ms per gulp" % ("graph" if graph else "eager", dt * 1e3 / (passes * ng)))
    if res["graph"]["candidates"] != res["eager"]["candidates"]:
        raise SystemExit("graph and eager candidate counts differ")
    samples = b.ndm * gulp
    ms = res["graph"]["ms_per_gulp"]
    st_ms = res["stages_ms"]
    dom = "block_stats" if st_ms["block_stats"] >= st_ms["detect"] else "detect"
    achieved = 4.0 * samples / (st_ms[dom] * 1e-3) / 1e9
    out = {
        "metric": "DM-trial-samples/s", "value": samples / (ms * 1e-3), "unit": "DM-trial-samples/s", "n_gpus": 1,
        "steps": res["graph"]["gulps"], "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "i32", "data": "synthetic",
        "config": {"workload": "%s: ndm=%d, gulps of %d samples, widths=1..4096, baseline=%d, theta=%g, "
                               "captured HIP graph per gulp step" % (cfg["name"], b.ndm, gulp, b.baseline_len,
                                                                     b.snr_thresh),
                   "step": "one gulp"},
        "roofline": {"bound": "hbm", "kernel": dom + " (eager pass timing)", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None},
        "eager_ms_per_gulp": res["eager"]["ms_per_gulp"],
        "stages_ms": st_ms,
        "candidates_per_gulp": res["graph"]["candidates"] / res["graph"]["gulps"],
        "cpu_baseline": None,
    }
    plan.close()
    print(json.dumps(out))


def bench_dedisp(args):
    """Incoherent dedispersion on the device, the producer of the search's
    input: a seeded 8-bit filterbank of 1024 channels over 1050-1450 MHz at
    49.152 us (FAST-like L band), 1024 trial DMs over 0-1000 pc cm^-3, output
    chunks of 2^18 samples (the paper's 256K-sample chunks), channel-major and
    HBM-resident before the timed region. Also times the zero-DM excision of
    the filterbank, and excision, dedispersion and the search of its output
    in sequence (the device-resident pipeline)."""
    import numpy as np
    import torch
    from synth import filterbank as fb
    from paper_2512_00398_amd import sps

    nchan, ndm, nout, tsamp = 1024, 1024, 1 << 18, 49.152e-6
    f, fref = fb.band(nchan)
    dms = np.linspace(0, 1000, ndm).astype(np.float32)
    tab = sps.dedisp_delays(f, fref, tsamp, dms)
    nin = nout + int(tab.max())
    log("generate filterbank %d x %d" % (nchan, nin))
    rng = np.random.default_rng(77)
    picks = rng.integers(0, ndm, size=24)
    pulses = [(int(rng.integers(0, nout - 4096)), int(2 ** rng.integers(0, 9)), int(rng.integers(3, 30)))
              for _ in picks]
    fil = fb.filterbank(nchan, nin, seed=77, pulses=pulses, tracks=tab[picks])
    fd = torch.from_numpy(fil).cuda()
    stream = torch.cuda.current_stream()
    k = sps.Dedisperser(nchan, nin, tab)
    out = k.alloc_out()
    for _ in range(args.warmup):
        k.run(fd, out, stream=stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        k.run(fd, out, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kms = e0.elapsed_time(e1) / args.steps
    ms = (t1 - t0) * 1e3 / args.steps
    # broadband (zero-DM) RFI excision of the same filterbank into a second buffer
    fz = torch.empty_like(fd)
    sps.zero_dm(fd, 64, out=fz, stream=stream)
    torch.cuda.synchronize()
    ez0, ez1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ez0.record(stream)
    for _ in range(args.steps):
        sps.zero_dm(fd, 64, out=fz, stream=stream)
    ez1.record(stream)
    torch.cuda.synchronize()
    zms = ez0.elapsed_time(ez1) / args.steps
    # narrowband excision (channel statistics, flags, replacement) into the same second buffer
    st = torch.empty((nchan, 3), dtype=torch.uint8, device="cuda")
    sps.chan_mask(fd, 4, out=fz, stats=st, stream=stream)
    torch.cuda.synchronize()
    ez0.record(stream)
    for _ in range(args.steps):
        sps.chan_mask(fd, 4, out=fz, stats=st, stream=stream)
    ez1.record(stream)
    torch.cuda.synchronize()
    mms = ez0.elapsed_time(ez1) / args.steps
    # the pipeline: zero-DM excision, dedispersion, then the search of its output
    plan = sps.Plan(ndm, nout, 4096, 16384, 6.0)
    cands, ncand = plan.alloc_cands()
    sps.zero_dm(fd, 64, out=fz, stream=stream)
    k.run(fz, out, stream=stream)
    plan.search(out, cands, ncand, stream=stream)
    torch.cuda.synchronize()
    tp0 = time.perf_counter()
    for _ in range(args.steps):
        sps.zero_dm(fd, 64, out=fz, stream=stream)
        k.run(fz, out, stream=stream)
        plan.search(out, cands, ncand, stream=stream)
    torch.cuda.synchronize()
    pipe_ms = (time.perf_counter() - tp0) * 1e3 / args.steps
    n = int(ncand.item())
    plan.close()
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import dedisp_oracle as dd
        rows = 8
        c0 = time.perf_counter()
        dd.dedisperse(fil, tab[:: ndm // rows][:rows].astype(np.int64))
        cs = time.perf_counter() - c0
        cpu = {"value": rows * nout / cs, "unit": "DM-trial-samples/s", "cores": 1, "kind": "oracle",
               "sample": "%d of %d trial DMs, full %d-channel rows of %d samples, one process" % (rows, ndm, nchan, nout),
               "seconds": round(cs, 3)}
    k.close()
    adds = float(ndm) * nchan * nout
    achieved = adds / (kms * 1e-3) / 1e12
    peak = ALU_PAIR_ADD_PEAK_TOPS
    print(json.dumps({
        "metric": "DM-trial-samples/s", "value": ndm * nout / (ms * 1e-3), "unit": "DM-trial-samples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8->i32", "data": "synthetic",
        "config": {"workload": "dedisp: 1024 channels 1050-1450 MHz, tsamp 49.152 us, 1024 trial DMs 0-1000, "
                               "%d output samples (%d input)" % (nout, nin)},
        "roofline": {"bound": "alu", "kernel": "dedisp", "achieved": achieved, "peak": peak, "unit": "TOP/s",
                     "peak_note": "sample additions per second: 32-bit adds of packed 16-bit pairs (2 per lane per "
                                  "clock, 256 CUs x 64 lanes x 2.4 GHz)",
                     "frac": achieved / peak, "traffic": measured_traffic("dedisp"),
                     "algorithmic_ops": adds, "algorithmic_bytes": float(nchan) * nin + 4.0 * ndm * nout},
        "kernel_ms": kms,
        "zero_dm": {"ms": zms, "algorithmic_GBps": 2.0 * nchan * nin / (zms * 1e-3) / 1e9,
                    "note": "filterbank read once and written once (algorithmic bytes; the kernel's own reads "
                            "and writes are the same here: one pass, words held in registers)"},
        "chan_mask": {"ms": mms, "k": 4, "flagged": int(st[:, 2].sum().item())},
        "pipeline": "zero-DM excision + dedispersion + search", "pipeline_ms_per_chunk": pipe_ms,
        "pipeline_candidates": n, "cpu_baseline": cpu}))


def bench_batch(args):
    """Many-file workload: one batched search (persistent launch per stage)
    against a loop of single-block searches over the same resident files."""
    import torch
    import synth
    from paper_2512_00398_amd import sps

    cfg = synth.config(4)
    blocks = cfg["blocks"]
    xs, outs, items, plans = [], [], [], []
    for k, b in enumerate(blocks):
        x = synth.generate(b)
        xs.append(torch.from_numpy(x).cuda())
        del x
        # room for the drift flood (about 0.8% of the samples become candidates)
        cap = min((1 << 32) - 1, int(0.012 * b.ndm * b.nsamp) + (1 << 16))
        cands = torch.empty((cap, 4), dtype=torch.int32, device="cuda")
        ncand = torch.zeros((1,), dtype=torch.int32, device="cuda")
        outs.append((cands, ncand))
        items.append((xs[-1], b.max_width, b.baseline_len, b.snr_thresh, cands, ncand))
        plans.append(sps.Plan(b.ndm, b.nsamp, b.max_width, b.baseline_len, b.snr_thresh))
        plans[-1].set(sps.ATTR_MAX_CANDS, cap)
    log("generated %d files, %.3g samples" % (len(blocks), sum(b.ndm * b.nsamp for b in blocks)))
    stream = torch.cuda.current_stream()
    batch = sps.Batch()
    # the batch runs on the autotuner's configuration for its shape classes
    # (tuned now, untimed, if the cache has none); every configuration tried
    # must return every file's candidates unchanged
    from paper_2512_00398_amd import autotune
    shapes = [(b.ndm, b.nsamp, b.max_width, b.baseline_len) for b in blocks]
    tuned = autotune.apply_batch(batch, shapes)
    tuned_from = "cache"
    if tuned is None:
        res = autotune.tune_batch(batch, items, stream=stream, steps=1, log=log)
        tuned, tuned_from = res["config"], "tuned now (default %.1f ms, tuned %.1f ms)" % (res["default_ms"], res["ms"])
    log("batch tuning: %s (%s)" % (tuned, tuned_from))
    for p, b in zip(plans, blocks):
        autotune.apply(p)  # per-file plans take their own cached configuration, if any

    def run_batch():
        batch.search(items, stream=stream)

    def run_loop():
        for p, it in zip(plans, items):
            p.search(it[0], it[4], it[5], stream=stream)

    def timed(fn, steps):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps, e0.elapsed_time(e1) / steps

    ms_batch, dev_batch = timed(run_batch, args.steps)
    n_batch = [int(n.item()) & 0xFFFFFFFF for _, n in outs]
    for (c, _), nb in zip(outs, n_batch):
        if nb > c.shape[0]:
            raise SystemExit("candidate buffer overflow in the batch (%d > %d)" % (nb, c.shape[0]))
    log("batch: %.3f ms/step" % ms_batch)
    ms_loop, dev_loop = timed(run_loop, args.steps)
    n_loop = [int(n.item()) & 0xFFFFFFFF for _, n in outs]
    log("per-file loop: %.3f ms/step" % ms_loop)
    if n_batch != n_loop:
        raise SystemExit("batch and per-file candidate counts differ")
    samples = sum(b.ndm * b.nsamp for b in blocks)
    value = samples / (ms_batch * 1e-3)
    achieved = 4.0 * samples / (dev_batch * 1e-3) / 1e9
    out = {
        "metric": "DM-trial-samples/s", "value": value, "unit": "DM-trial-samples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_batch, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "i32", "data": "synthetic",
        "config": {"workload": "%s: %d files, ndm 256..2048, nsamp 2^16..2^20, widths=1..4096, baseline=16384, "
                               "theta=6, %d samples" % (cfg["name"], len(blocks), samples),
                   "input": "f32 integer-valued, HBM-resident"},
        "roofline": {"bound": "hbm", "kernel": "whole batch (all stages)", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None},
        "per_file_loop_ms_per_step": ms_loop,
        "batch_vs_loop": ms_loop / ms_batch,
        "tuning": {"config": tuned, "source": tuned_from,
                   "attributes": "chain length (blocks), detection segment (samples), histogram span; every width "
                                 "is evaluated in one pass, so there is no widths-per-pass attribute"},
        "candidates": sum(n_batch),
        "cpu_baseline": None,
    }
    batch.close()
    for p in plans:
        p.close()
    print(json.dumps(out))


def bench_serve(args):
    """Serving workload: 16 beams, Poisson gulp arrivals at 1.5x real time,
    admission against the memory budget; gulp latency percentiles at the
    literal rate and over a time-compressed sweep up to saturation."""
    import torch
    import synth
    from paper_2512_00398_amd import serve

    cfg = synth.config(5)
    blocks = cfg["blocks"]
    G = 2  # distinct gulps held per beam, replayed in turn
    pools = []
    for b in blocks:
        x = synth.generate(b.with_(nsamp=G * b.nsamp))
        pools.append(torch.from_numpy(x.reshape(b.ndm, G, b.nsamp).transpose(1, 0, 2).copy()).cuda())
        del x
    specs = [serve.BeamSpec(ndm=b.ndm, nsamp=b.nsamp, max_width=b.max_width, baseline_len=b.baseline_len,
                            snr_thresh=b.snr_thresh) for b in blocks]
    log("serving %d beams, %.3g samples per round of gulps" % (len(specs), sum(s.ndm * s.nsamp for s in specs)))

    def source(beam, k):
        return pools[beam][k % G]

    rate = cfg["arrival_rate_x_realtime"]
    budget = cfg["hbm_budget_bytes"]
    seed = synth.BASE_SEED + 4

    def run(compress, batch=True, **kw):
        arr = serve.poisson_arrivals(specs, rate, seed, **kw)
        ex = serve.GpuExecutor(source, nstreams=4, cand_cap=1 << 23, batch=batch)
        rep = serve.serve(specs, arr, ex, budget, compress=compress, slots=args.serve_slots,
                          min_group=args.serve_min_group if batch else 1)
        s = rep.summary()
        s["compress"] = "inf" if compress == float("inf") else compress
        s["executor"] = "batched (sps_batch_push)" if batch else "one device stream per beam"
        if batch:
            s["gulps_per_launch_max"] = max(ex.batch_sizes) if ex.batch_sizes else 0
            s["gulps_per_launch_mean"] = (sum(ex.batch_sizes) / len(ex.batch_sizes)) if ex.batch_sizes else 0.0
        s["offered_samples_per_s"] = (sum(specs[a.beam].ndm * specs[a.beam].nsamp for a in arr) /
                                      (max(a.t for a in arr) / compress) if compress != float("inf") else None)
        s["ncand_total"] = int(sum(r.ncand for r in rep.records))
        log("serve x%s: %s" % (s["compress"], {k: s[k] for k in ("gulps", "p50_ms", "p99_ms", "samples_per_s")}))
        return s

    for _ in range(max(1, args.warmup)):
        run(float("inf"), gulps_per_beam=2)
    literal = run(1.0, horizon=args.serve_horizon)
    sweep = [run(c, gulps_per_beam=6) for c in (10.0, 30.0, 60.0, 120.0, float("inf"))]
    per_beam = run(float("inf"), batch=False, gulps_per_beam=6)
    if len({s["ncand_total"] for s in sweep + [per_beam]}) != 1:
        raise SystemExit("candidate totals differ between serving runs of the same gulps: %s" %
                         [s["ncand_total"] for s in sweep + [per_beam]])
    sat = sweep[-1]
    out = {
        "metric": "DM-trial-samples/s", "value": sat["samples_per_s"], "unit": "DM-trial-samples/s", "n_gpus": 1,
        "steps": sat["gulps"], "warmup": args.warmup, "ms_per_step": sat["wall_s"] * 1e3 / sat["gulps"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "i32", "data": "synthetic",
        "config": {"workload": "%s: 16 beams, ndm 512..2048, gulps 2^16..2^18, widths=1..4096, baseline=16384, "
                               "theta=6, Poisson arrivals at %.1fx real time, budget %d B, %d gulps in flight" %
                               (cfg["name"], rate, budget, args.serve_slots),
                   "value_is": "saturation throughput (all arrivals at once), gulp = step",
                   "executor": "continuous batching: gulps ready together share one launch per stage; under "
                               "load ready gulps wait for %d free slots" % args.serve_min_group},
        "latency_literal_rate": literal,
        "latency_sweep": sweep,
        "saturation_per_beam_streams": per_beam,
        "cpu_baseline": None,
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2, choices=[1, 2, 3, 4, 5, 6],
                    help="1 small block, 2 single large block (default), 3 streaming 8 gulps through captured "
                         "HIP graphs, 4 batch of 32 files, "
                         "5 serving 16 beams (literal arrival rate, then a time-compressed sweep), "
                         "6 incoherent dedispersion of a 1024-channel filterbank (and the search of its output)")
    ap.add_argument("--serve-horizon", type=float, default=20.0,
                    help="seconds of literal-rate arrivals served in --config 5")
    ap.add_argument("--serve-slots", type=int, default=8, help="gulps in flight at most in --config 5")
    ap.add_argument("--serve-min-group", type=int, default=4,
                    help="--config 5, batched executor: under load, ready gulps wait for this many free slots")
    ap.add_argument("--cpu-rows", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip timing the plain per-stage path")
    ap.add_argument("--no-cluster", action="store_true", help="skip timing the clustering of the candidates")
    ap.add_argument("--cluster-tol", type=int, nargs=3, default=[32, 3, 2], metavar=("TIME", "DM", "WIDTH"),
                    help="clustering tolerances: samples, DM trials, log2 widths")
    ap.add_argument("--per-dm-rows", type=int, default=32,
                    help="rows timed for the per-DM-trial loop of the plain path (0: skip)")
    ap.add_argument("--autotune", action="store_true",
                    help="tune the plan's speed-only attributes on the input first (untimed; cached as JSON)")
    ap.add_argument("--window", default="trailing", choices=["trailing", "centred"],
                    help="baseline window placement (SPS_ATTR_WINDOW)")
    ap.add_argument("--norm", default="block", choices=["block", "row", "width"],
                    help="noise scale: per-block MAD, one MAD per DM row, or one MAD per (DM row, width) "
                         "(SPS_ATTR_NORM 0, 1, 2)")
    ap.add_argument("--mode", default="search", choices=["search", "copy"],
                    help="copy: time a plain device-to-device copy of 1 GiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only (got --gpus %d): the search shards by DM rows, files or "
              "beams with no exchange, so one GPU's share is the unit of measurement" % args.gpus, file=sys.stderr)
        sys.exit(2)

    if args.mode == "copy":
        import torch
        n = 1 << 28  # 2^28 float32 = 1 GiB read + 1 GiB written per copy
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        print(json.dumps({"mode": "copy", "bytes_read": 4 * n, "bytes_written": 4 * n, "ms": dt * 1e3,
                          "GBps_read_plus_write": 8 * n / dt / 1e9}))
        return

    if args.config == 3:
        return bench_stream(args)
    if args.config == 4:
        return bench_batch(args)
    if args.config == 5:
        return bench_serve(args)
    if args.config == 6:
        return bench_dedisp(args)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on %d rows" % args.cpu_rows)
        cpu = cpu_baseline(args.config, args.cpu_rows, args.window == "centred", args.norm == "row",
                           args.norm == "width")
        log("cpu baseline: %.3g samples/s on %d cores" % (cpu["value"], cpu["cores"]))

    import numpy as np
    import torch
    import synth
    from paper_2512_00398_amd import sps

    cfg = synth.config(args.config)
    b = cfg["blocks"][0]
    log("generate %s (%d x %d)" % (cfg["name"], b.ndm, b.nsamp))
    x = synth.generate(b)
    xd = torch.from_numpy(x).cuda()
    del x
    stream = torch.cuda.current_stream()
    plan = sps.Plan(b.ndm, b.nsamp, b.max_width, b.baseline_len, b.snr_thresh)
    variant = {sps.ATTR_WINDOW: int(args.window == "centred"), sps.ATTR_NORM: {"block": 0, "row": 1, "width": 2}[args.norm]}
    for attr, v in variant.items():
        plan.set(attr, v)
    default_variant = not any(variant.values())
    tuned = None
    if args.autotune:
        from paper_2512_00398_amd import autotune
        tuned = autotune.tune(plan, xd, stream=stream, steps=2, log=log)
        log("autotune: %s (%.3f ms, default %.3f ms)" % (tuned["config"], tuned["ms"], tuned["default_ms"]))
    cands, ncand = plan.alloc_cands()
    for i in range(args.warmup):
        plan.search(xd, cands, ncand, stream=stream)
    torch.cuda.synchronize()
    log("warmup done")
    plan.set(sps.ATTR_TIMING, 1)
    plan.timing_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        plan.search(xd, cands, ncand, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stages, nsearch = plan.timing_read()
    n = int(ncand.item())
    log("timed %d steps: %.3f ms/step, %d candidates" % (args.steps, (t1 - t0) * 1e3 / args.steps, n))

    # the plain per-stage path on the same input (comparison only, not the metric)
    plain_ms = None
    if args.norm == "width":
        args.no_plain = True  # the per-stage path keeps per-block or per-row scales only
    if not args.no_plain:
        plan.search(xd, cands, ncand, stream=stream, plain=True)
        torch.cuda.synchronize()
        n_plain = int(ncand.item())
        plan.timing_read()
        tp0 = time.perf_counter()
        for i in range(max(1, args.steps // 2)):
            plan.search(xd, cands, ncand, stream=stream, plain=True)
        torch.cuda.synchronize()
        plain_ms = (time.perf_counter() - tp0) * 1e3 / max(1, args.steps // 2)
        pst, pn = plan.timing_read()
        log("plain per-stage path: %.3f ms/step (%d candidates)" % (plain_ms, n_plain))
        if n_plain != n:
            raise SystemExit("plain and fused candidate counts differ: %d vs %d" % (n_plain, n))

    # the plain path as a per-DM-trial loop (one row per call, the shape of the
    # staged per-trial loop), timed on a sample of rows and scaled to ndm rows
    per_dm_ms = None
    if not args.no_plain and args.per_dm_rows > 0:
        rows = min(args.per_dm_rows, b.ndm)
        p1 = sps.Plan(1, b.nsamp, b.max_width, b.baseline_len, b.snr_thresh)
        for attr, v in variant.items():
            p1.set(attr, v)
        c1, n1 = p1.alloc_cands()
        p1.search(xd[0:1], c1, n1, stream=stream, plain=True)
        torch.cuda.synchronize()
        tq0 = time.perf_counter()
        for r in range(rows):
            p1.search(xd[r:r + 1], c1, n1, stream=stream, plain=True)
        torch.cuda.synchronize()
        per_dm_ms = (time.perf_counter() - tq0) * 1e3 / rows * b.ndm
        p1.close()
        log("plain per-DM loop: %.1f ms per %d rows (from %d rows)" % (per_dm_ms, b.ndm, rows))

    # candidate merging and clustering of this search's candidates (reported beside the metric)
    cluster = None
    if not args.no_cluster and n > 0:
        plan.search(xd, cands, ncand, stream=stream)
        k = sps.Clusterer(n)
        out_c, nout = k.alloc_out(n)
        tt, dt, wt = args.cluster_tol
        k.run(cands, n, tt, dt, wt, out_c, nout, stream=stream)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(3):
            k.run(cands, n, tt, dt, wt, out_c, nout, stream=stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        cms = ev0.elapsed_time(ev1) / 3
        cluster = {"tolerances": {"samples": tt, "dm_trials": dt, "log2_width": wt}, "ms": cms, "candidates": n,
                   "clusters": int(nout.item()), "candidates_per_s": n / (cms * 1e-3)}
        k.close()
        log("clustering: %.3f ms for %d candidates -> %d clusters" % (cms, n, cluster["clusters"]))

    samples = b.ndm * b.nsamp
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = samples * args.steps / (t1 - t0)
    avg = {k: v / max(1, nsearch) for k, v in stages.items()}
    # Algorithmic bytes: 4 B per DM-trial-sample (the FP32 block read once)
    # plus 16 B per candidate written; the medians and MADs that pass from the
    # statistics kernel to the detection kernel are not algorithmic traffic.
    alg_bytes = 4.0 * samples + 16.0 * n
    dom = "block_stats" if avg["block_stats"] >= avg["detect"] else "detect"
    dom_bytes = 4.0 * samples + (16.0 * n if dom == "detect" else 0.0)
    achieved = dom_bytes / (avg[dom] * 1e-3) / 1e9
    issue = measured_issue(dom) if args.config == 2 and default_variant else None
    if issue:
        issue = {"valu_wave_instructions_per_launch": issue, "valu_issue_ms": issue / VALU_ISSUE_PER_S * 1e3,
                 "valu_issue_frac_of_kernel_time": issue / VALU_ISSUE_PER_S / (avg[dom] * 1e-3),
                 "peak_note": "one VALU wave-instruction per CU per clock: 256 CUs x 2.4 GHz"}
    out = {
        "metric": "DM-trial-samples/s",
        "value": value,
        "unit": "DM-trial-samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i32",
        "data": "synthetic",
        "config": {"workload": "%s: ndm=%d nsamp=%d widths=1..%d baseline=%d theta=%g%s" %
                               (cfg["name"], b.ndm, b.nsamp, b.max_width, b.baseline_len, b.snr_thresh,
                                "" if default_variant else " window=%s norm=%s" % (args.window, args.norm)),
                   "input": "f32 integer-valued, HBM-resident", "snr": "f64 decision, f32 output"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(dom) if args.config == 2 and default_variant else None,
                     "algorithmic_bytes": dom_bytes, "issue": issue},
        "path_roofline": {"achieved": alg_bytes / (ms_per_step * 1e-3) / 1e9, "unit": "GB/s",
                          "frac": alg_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
                          "algorithmic_bytes": alg_bytes, "note": "whole search (every kernel) per step"},
        "stages_ms": {k: round(v, 4) for k, v in avg.items() if k != "plain"},
        "plain_ms_per_step": plain_ms,
        "fused_vs_plain": (plain_ms / ms_per_step) if plain_ms else None,
        "plain_per_dm_loop_ms_per_step": per_dm_ms,
        "fused_vs_per_dm_loop": (per_dm_ms / ms_per_step) if per_dm_ms else None,
        "candidates": n,
        "cluster": cluster,
        "tuning": tuned["config"] if tuned else "library defaults",
        "cpu_baseline": cpu,
    }
    plan.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
