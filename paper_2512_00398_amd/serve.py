"""Serving loop: many beams streamed concurrently on one GPU.

Each beam is one long observation arriving gulp by gulp (the paper's
real-time setting: chunks of a continuous stream searched as they arrive,
Sections III-B and V-C). A beam owns a plan and a device-resident stream
(history, block statistics and open runs are carried between its gulps), so a
beam's results are those of searching its whole observation at once.

The scheduler is plain host logic and runs against any executor:

- Admission: a beam is admitted when its device footprint (plan + stream +
  input and candidate buffers) fits in what is left of the memory budget;
  otherwise it waits, first come first served, until admitted beams finish.
- Dispatch: every arriving gulp of an admitted beam is enqueued as soon as
  one of `slots` in-flight places is free (continuous: nothing waits for a
  batch to fill; arrivals beyond the slots wait first come first served).
  Gulps that become ready together are handed over together: a batching
  executor searches gulps of different beams in one launch per stage while
  earlier launches are still on the device. A beam's gulps stay in order.
- Latency of a gulp: from its arrival to the completion of its search on the
  device (candidates in device memory).

GpuExecutor does the device work through the HIP library; a test may pass any
object with the same methods.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import sps


@dataclasses.dataclass(frozen=True)
class BeamSpec:
    ndm: int
    nsamp: int                # samples per gulp (multiple of 64)
    max_width: int = 4096
    baseline_len: int = 16384
    snr_thresh: float = 6.0
    tsamp: float = 64e-6      # seconds per sample (sets the real-time gulp period)

    @property
    def gulp_seconds(self) -> float:
        return self.nsamp * self.tsamp


@dataclasses.dataclass(frozen=True)
class Arrival:
    t: float                  # seconds after the start of the run (before time compression)
    beam: int
    k: int                    # gulp index within the beam


def poisson_arrivals(specs: Sequence[BeamSpec], rate_x_realtime: float, seed: int,
                     gulps_per_beam: Optional[int] = None, horizon: Optional[float] = None) -> List[Arrival]:
    """Poisson arrivals per beam, mean inter-arrival = gulp duration / rate.

    Stops each beam after `gulps_per_beam` gulps and/or at time `horizon`."""
    if gulps_per_beam is None and horizon is None:
        raise ValueError("give gulps_per_beam or horizon")
    out: List[Arrival] = []
    for b, s in enumerate(specs):
        rng = np.random.default_rng([seed, b])
        mean = s.gulp_seconds / rate_x_realtime
        t, k = 0.0, 0
        while True:
            t += float(rng.exponential(mean))
            if (gulps_per_beam is not None and k >= gulps_per_beam) or (horizon is not None and t > horizon):
                break
            out.append(Arrival(t, b, k))
            k += 1
    out.sort(key=lambda a: (a.t, a.beam, a.k))
    return out


class Admission:
    """First-come-first-served admission against a byte budget."""

    def __init__(self, budget: int):
        self.budget = int(budget)
        self.used = 0
        self.admitted: Dict[int, int] = {}
        self.waiting: "collections.OrderedDict[int, int]" = collections.OrderedDict()

    def enqueue(self, beam: int, nbytes: int) -> None:
        if beam in self.admitted or beam in self.waiting:
            return
        if nbytes > self.budget:
            raise ValueError("beam %d needs %d bytes, more than the whole budget %d" % (beam, nbytes, self.budget))
        self.waiting[beam] = int(nbytes)

    def drain(self) -> List[int]:
        """Admit from the head of the waiting line while it fits; returns the beams admitted."""
        got = []
        while self.waiting:
            beam, nbytes = next(iter(self.waiting.items()))
            if self.used + nbytes > self.budget:
                break
            self.waiting.popitem(last=False)
            self.admitted[beam] = nbytes
            self.used += nbytes
            got.append(beam)
        return got

    def release(self, beam: int) -> List[int]:
        self.used -= self.admitted.pop(beam)
        return self.drain()


@dataclasses.dataclass
class GulpRecord:
    beam: int
    k: int
    arrival: float            # seconds (compressed clock)
    submitted: float          # host seconds when enqueued
    done: Optional[float] = None
    ncand: Optional[int] = None
    started: Optional[float] = None   # the device reached the gulp (its stream's event)
    noticed: Optional[float] = None   # the host saw the completion (poll)

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclasses.dataclass
class Report:
    records: List[GulpRecord]
    wall: float
    samples: int
    max_concurrent_bytes: int
    max_inflight: int = 0

    def latencies(self) -> np.ndarray:
        return np.array([r.latency for r in self.records], dtype=np.float64)

    def breakdown(self) -> Optional[dict]:
        """p50/p99 (ms) of each part of a gulp's life, where the executor timed it:
        host_wait (arrival to submission: admission, free slot, scheduling loop),
        device_queue (submission to its stream reaching it), search (on the
        device), notice (completion to the host seeing it, the polling delay;
        after the latency's end, but a slot stays busy until then)."""
        recs = [r for r in self.records if r.started is not None and r.noticed is not None]
        if not recs:
            return None
        parts = {"host_wait": [r.submitted - r.arrival for r in recs],
                 "device_queue": [max(0.0, r.started - r.submitted) for r in recs],
                 "search": [r.done - r.started for r in recs],
                 "notice": [max(0.0, r.noticed - r.done) for r in recs]}
        return {k: {"p50_ms": float(np.percentile(v, 50) * 1e3), "p99_ms": float(np.percentile(v, 99) * 1e3)}
                for k, v in parts.items()}

    def summary(self) -> dict:
        lat = self.latencies()
        out = {"gulps": len(self.records), "p50_ms": float(np.percentile(lat, 50) * 1e3) if lat.size else None,
               "p99_ms": float(np.percentile(lat, 99) * 1e3) if lat.size else None,
               "max_ms": float(lat.max() * 1e3) if lat.size else None, "wall_s": self.wall,
               "samples_per_s": self.samples / self.wall if self.wall > 0 else None,
               "max_admitted_bytes": self.max_concurrent_bytes, "max_inflight": self.max_inflight}
        bd = self.breakdown()
        if bd is not None:
            out["breakdown"] = bd
        return out


def serve(specs: Sequence[BeamSpec], arrivals: Sequence[Arrival], executor, budget: int, compress: float = 1.0,
          clock: Callable[[], float] = time.perf_counter, sleep: Callable[[float], None] = time.sleep,
          slots: Optional[int] = None, min_group: int = 1) -> Report:
    """Run the arrivals through the executor; compress > 1 speeds the arrival clock up
    (float('inf'): everything arrives at once); slots caps the gulps in flight.
    min_group > 1: while gulps are on the device, ready gulps wait until
    min(min_group, ready) of them can go together (larger shared launches
    under load; an idle device takes whatever is ready at once)."""
    left = collections.Counter(a.beam for a in arrivals)
    adm = Admission(budget)
    backlog: Dict[int, collections.deque] = collections.defaultdict(collections.deque)
    records: List[GulpRecord] = []
    inflight: Dict[int, GulpRecord] = {}
    pending = collections.deque(sorted(arrivals, key=lambda a: (a.t, a.beam, a.k)))
    ready: collections.deque = collections.deque()  # admitted, waiting for a slot
    state = {"max_used": 0, "samples": 0, "max_inflight": 0}
    t0 = clock()
    executor.start(t0)

    def now() -> float:
        return clock() - t0

    def due(a: Arrival) -> float:
        return 0.0 if compress == float("inf") else a.t / compress

    many = getattr(executor, "submit_many", None)

    def dispatch() -> None:
        # every ready gulp that has a slot goes to the device now; an executor
        # that batches takes them together (gulps of different beams share a launch)
        if min_group > 1 and inflight and ready:
            free = len(ready) if slots is None else slots - len(inflight)
            if free < min(min_group, len(ready)):
                return
        group = []
        while ready and (slots is None or len(inflight) < slots):
            a, arrived = ready.popleft()
            rec = GulpRecord(a.beam, a.k, arrived, now())
            inflight[id(rec)] = rec
            state["samples"] += specs[a.beam].ndm * specs[a.beam].nsamp
            group.append((rec, specs[a.beam]))
        if not group:
            return
        if many is not None:
            many(group)
        else:
            for rec, spec in group:
                executor.submit(rec, spec)
        state["max_inflight"] = max(state["max_inflight"], len(inflight))

    def admit(beams: List[int]) -> None:
        for b in beams:
            executor.open(b, specs[b])
            state["max_used"] = max(state["max_used"], adm.used)
            while backlog[b]:
                ready.append(backlog[b].popleft())

    while pending or inflight or ready:
        tn = now()
        while pending and due(pending[0]) <= tn:
            a = pending.popleft()
            if a.beam in adm.admitted:
                ready.append((a, due(a)))
            else:
                backlog[a.beam].append((a, due(a)))
                adm.enqueue(a.beam, executor.footprint(specs[a.beam]))
                admit(adm.drain())
        dispatch()
        for rec in executor.poll():
            del inflight[id(rec)]
            records.append(rec)
            left[rec.beam] -= 1
            if left[rec.beam] == 0:
                executor.close(rec.beam)
                admit(adm.release(rec.beam))
        dispatch()
        if pending and not inflight and not ready:
            sleep(max(0.0, min(due(pending[0]) - now(), 1e-3)))
        elif inflight:
            sleep(5e-5)
    if any(backlog.values()) or adm.waiting:
        raise RuntimeError("serving ended with gulps that were never admitted")
    wall = now()
    executor.stop()
    records.sort(key=lambda r: (r.beam, r.k))
    rep = Report(records, wall, state["samples"], state["max_used"])
    rep.max_inflight = state["max_inflight"]
    return rep


class GpuExecutor:
    """Device work of the serving loop: one plan + stream per admitted beam.

    gulp_source(beam, k) returns the device tensor [ndm][nsamp] of gulp k of
    the beam, produced on the caller's current stream. The search of a gulp
    is ordered after that stream's work and the tensor is kept alive until
    the search has finished with it. Nothing here waits for the device while
    gulps are submitted: each gulp's completion is seen through its events.
    With keep=True every gulp gets its own candidate buffer, copied to the
    host once the gulp has completed (global sample indices kept for
    inspection); otherwise the beam's buffers are reused in turn and only the
    counts are kept."""

    def __init__(self, gulp_source: Callable[[int, int], "object"], nstreams: int = 4, cand_cap: int = 1 << 22,
                 cand_slots: int = 2, keep: bool = False, batch: bool = False):
        import torch
        self.torch = torch
        self.src = gulp_source
        self.streams = [torch.cuda.Stream() for _ in range(nstreams)]
        self.copy_stream = torch.cuda.Stream()
        # batch=True: gulps submitted together go through one persistent launch
        # per stage (sps_batch_push), one round per set of distinct beams; the
        # rounds rotate over the device streams (a context per stream), and a
        # beam's gulp waits for the event of its previous gulp when that ran on
        # another stream. Otherwise each beam pushes on its own device stream.
        self.batches = [sps.Batch() for _ in self.streams] if batch else None
        self.batch = self.batches
        self.round = 0
        self.last_event: Dict[int, Tuple[object, object]] = {}  # beam -> (device stream, event of its last gulp)
        self.batch_sizes: List[int] = []
        self.cap = int(cand_cap)
        self.slots = int(cand_slots)
        self.keep = keep
        self.beams: Dict[int, dict] = {}
        self.waiting: List[tuple] = []
        self.kept: Dict[int, list] = collections.defaultdict(list)
        self.intervals: List[Tuple[int, float, float]] = []  # (beam, device start, device end) per gulp
        self.ref = None

    def footprint(self, s: BeamSpec) -> int:
        return sps.footprint(s.ndm, s.nsamp, s.max_width, s.baseline_len, True) + self.slots * (16 * self.cap + 4)

    def start(self, t0: float) -> None:
        """t0: the scheduler's clock origin in time.perf_counter seconds."""
        torch = self.torch
        self.t0 = t0
        self.ref = torch.cuda.Event(enable_timing=True)
        self.ref.record(self.streams[0])
        self.ref.synchronize()
        self.t_ref = time.perf_counter()

    def open(self, beam: int, s: BeamSpec) -> None:
        torch = self.torch
        plan = sps.Plan(s.ndm, s.nsamp, s.max_width, s.baseline_len, s.snr_thresh)
        plan.set(sps.ATTR_MAX_CANDS, self.cap)
        st = sps.Stream(plan)
        bufs = [(torch.empty((self.cap, 4), dtype=torch.int32, device="cuda"),
                 torch.zeros((1,), dtype=torch.int32, device="cuda")) for _ in range(self.slots)]
        self.beams[beam] = {"plan": plan, "stream": st, "bufs": bufs, "hs": self.streams[beam % len(self.streams)],
                            "n": 0, "spec": s}

    def _clock(self, ev) -> float:
        """Scheduler-clock seconds of a completed timing event."""
        return self.t_ref - self.t0 + self.ref.elapsed_time(ev) * 1e-3

    def _prepare(self, rec: GulpRecord, hs=None):
        """The gulp's tensor, ordered on device stream hs (default: the beam's), and its candidate buffers."""
        torch = self.torch
        b = self.beams[rec.beam]
        hs = b["hs"] if hs is None else hs
        x = self.src(rec.beam, rec.k)
        # the gulp was written on the caller's stream: the search waits for it,
        # and the allocator keeps its memory until hs is past the search
        hs.wait_stream(torch.cuda.current_stream())
        x.record_stream(hs)
        if self.keep:
            with torch.cuda.stream(hs):
                cands = torch.empty((self.cap, 4), dtype=torch.int32, device="cuda")
                ncand = torch.empty((1,), dtype=torch.int32, device="cuda")
        else:
            cands, ncand = b["bufs"][b["n"] % self.slots]
        b["n"] += 1
        return b, hs, x, cands, ncand

    def _track(self, hs, recs, began, ev, xs, cands, ncands, offs) -> None:
        """Count copies and completion events of gulps just enqueued on hs."""
        torch = self.torch
        for rec, x, c, n, off in zip(recs, xs, cands, ncands, offs):
            host_n = torch.empty((1,), dtype=torch.int32, pin_memory=True)
            with torch.cuda.stream(hs):
                host_n.copy_(n, non_blocking=True)
            copied = torch.cuda.Event()               # count readable on the host
            copied.record(hs)
            self.waiting.append((rec, began, ev, copied, host_n, x, c, n, off))

    def submit(self, rec: GulpRecord, s: BeamSpec) -> None:
        if self.batch is not None:
            return self.submit_many([(rec, s)])
        torch = self.torch
        b, hs, x, cands, ncand = self._prepare(rec)
        began = torch.cuda.Event(enable_timing=True)  # the beam's stream reached this gulp
        began.record(hs)
        off = b["stream"].push(x, cands, ncand, stream=hs)
        ev = torch.cuda.Event(enable_timing=True)     # search done: candidates in device memory
        ev.record(hs)
        self._track(hs, [rec], began, ev, [x], [cands], [ncand], [off])

    def submit_many(self, group) -> None:
        """Gulps (rec, spec) that became ready together. With batching, each
        round of distinct beams is one sps_batch_push; a beam's next gulp goes
        to the next round (it needs this one's carry)."""
        if self.batch is None:
            for rec, s in group:
                self.submit(rec, s)
            return
        torch = self.torch
        pending = list(group)
        while pending:
            seen, now_, later = set(), [], []
            for rec, s in pending:
                (later if rec.beam in seen else now_).append((rec, s))
                seen.add(rec.beam)
            pending = later
            k = self.round % len(self.streams)
            self.round += 1
            hs = self.streams[k]
            for rec, _ in now_:
                prev = self.last_event.get(rec.beam)
                if prev is not None and prev[0] is not hs:
                    hs.wait_event(prev[1])  # the beam's previous gulp (and its carry) first
            prep = [self._prepare(rec, hs) for rec, _ in now_]
            began = torch.cuda.Event(enable_timing=True)
            began.record(hs)
            offs = self.batches[k].push([p[0]["stream"] for p in prep], [p[2] for p in prep], [p[3] for p in prep],
                                        [p[4] for p in prep], stream=hs)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(hs)
            for rec, _ in now_:
                self.last_event[rec.beam] = (hs, ev)
            self.batch_sizes.append(len(now_))
            self._track(hs, [rec for rec, _ in now_], began, ev, [p[2] for p in prep], [p[3] for p in prep],
                        [p[4] for p in prep], offs)

    def poll(self) -> List[GulpRecord]:
        done = []
        still = []
        for item in self.waiting:
            rec, began, ev, copied, host_n, x, cands, ncand, off = item
            if copied.query():
                rec.noticed = time.perf_counter() - self.t0
                rec.done = self._clock(ev)
                rec.started = self._clock(began)
                self.intervals.append((rec.beam, rec.started, rec.done))
                rec.ncand = int(host_n.item()) & 0xFFFFFFFF
                if rec.ncand > self.cap:
                    raise sps.SpsError(sps.SPS_ERR_OVERFLOW, "gulp %d of beam %d" % (rec.k, rec.beam))
                if self.keep:
                    # the gulp is complete; copy on a stream of its own so that
                    # the beam's later gulps are not waited for
                    with self.torch.cuda.stream(self.copy_stream):
                        got = sps.cands_to_numpy(cands, ncand, self.cap)
                    self.kept[rec.beam].append((got, off))
                done.append(rec)
            else:
                still.append(item)
        self.waiting = still
        return done

    def device_overlap(self) -> Tuple[int, int]:
        """Most gulps, and most distinct beams, whose device intervals (from the
        beam's stream reaching the gulp to its search's end) share an instant."""
        marks = sorted([(t0, 1, b) for b, t0, _ in self.intervals] + [(t1, -1, b) for b, _, t1 in self.intervals],
                       key=lambda m: (m[0], m[1]))
        live: collections.Counter = collections.Counter()
        best_g = best_b = 0
        for _, d, b in marks:
            live[b] += d
            if live[b] == 0:
                del live[b]
            best_g = max(best_g, sum(live.values()))
            best_b = max(best_b, len(live))
        return best_g, best_b

    def close(self, beam: int) -> None:
        b = self.beams.pop(beam)
        cands, ncand = b["bufs"][b["n"] % self.slots]
        prev = self.last_event.pop(beam, None)
        if prev is not None and prev[0] is not b["hs"]:
            b["hs"].wait_event(prev[1])
        end = b["stream"].flush(cands, ncand, stream=b["hs"])
        if self.keep:
            b["hs"].synchronize()
            self.kept[beam].append((sps.cands_to_numpy(cands, ncand, self.cap), end))
        b["stream"].close()  # waits for this beam's own last push only
        b["plan"].close()

    def stop(self) -> None:
        self.torch.cuda.synchronize()
        if self.batches is not None:
            for bt in self.batches:
                bt.close()
