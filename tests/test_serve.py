"""Serving loop: scheduler logic on the CPU (simulated device and clock), and on
the GPU that a beam served in a mix of beams gets exactly its results alone."""
import collections

import numpy as np
import pytest

from paper_2512_00398_amd import serve


class FakeClock:
    def __init__(self):
        self.t = 100.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class SimExecutor:
    """One FIFO device: service time = samples / rate, started when submitted."""

    def __init__(self, clock, rate=1e9, foot=100):
        self.clock, self.rate, self.foot = clock, rate, foot
        self.free_at = 0.0
        self.q = []
        self.open_beams = set()
        self.events = []
        self.order = collections.defaultdict(list)

    def footprint(self, spec):
        return self.foot * spec.ndm

    def start(self, t0):
        self.t0 = t0

    def open(self, beam, spec):
        assert beam not in self.open_beams
        self.open_beams.add(beam)
        self.events.append(("open", beam))

    def submit(self, rec, spec):
        assert rec.beam in self.open_beams
        now = self.clock() - self.t0
        start = max(now, self.free_at)
        rec.started = start
        self.free_at = start + spec.ndm * spec.nsamp / self.rate
        self.q.append((self.free_at, rec))
        self.order[rec.beam].append(rec.k)

    def poll(self):
        now = self.clock() - self.t0
        done = [r for t, r in self.q if t <= now]
        for t, r in self.q:
            if t <= now:
                r.done = t
                r.noticed = now
                r.ncand = 0
        self.q = [(t, r) for t, r in self.q if t > now]
        return done

    def close(self, beam):
        self.open_beams.remove(beam)
        self.events.append(("close", beam))

    def stop(self):
        pass


def specs4():
    return [serve.BeamSpec(ndm=512, nsamp=1 << 16), serve.BeamSpec(ndm=1024, nsamp=1 << 17),
            serve.BeamSpec(ndm=2048, nsamp=1 << 16), serve.BeamSpec(ndm=700, nsamp=1 << 18)]


def test_poisson_arrivals_rate_and_order():
    sp = [serve.BeamSpec(ndm=512, nsamp=1 << 16)]
    arr = serve.poisson_arrivals(sp, rate_x_realtime=1.5, seed=3, gulps_per_beam=4000)
    t = np.array([a.t for a in arr])
    mean = sp[0].gulp_seconds / 1.5
    gaps = np.diff(np.concatenate([[0.0], t]))
    # mean of 4000 exponential gaps within 5 standard errors
    assert abs(gaps.mean() - mean) < 5 * mean / np.sqrt(4000)
    assert [a.k for a in arr] == list(range(4000))
    h = serve.poisson_arrivals(specs4(), 1.5, 3, horizon=30.0)
    assert all(a.t <= 30.0 for a in h) and h == sorted(h, key=lambda a: (a.t, a.beam, a.k))
    assert h == serve.poisson_arrivals(specs4(), 1.5, 3, horizon=30.0)


def test_admission_fcfs_budget():
    a = serve.Admission(1000)
    for b, n in ((0, 600), (1, 300), (2, 500), (3, 100)):
        a.enqueue(b, n)
    assert a.drain() == [0, 1]          # 2 does not fit; 3 waits behind it (strict FCFS)
    assert a.used == 900
    assert a.release(0) == [2, 3]
    assert a.used == 900
    with pytest.raises(ValueError):
        a.enqueue(9, 2000)


def test_serve_all_gulps_in_order_within_budget():
    clk = FakeClock()
    sp = specs4()
    ex = SimExecutor(clk, rate=2e10, foot=100)
    arr = serve.poisson_arrivals(sp, 10.0, seed=11, gulps_per_beam=6)
    budget = 100 * 2048 + 100 * 1024  # never all four beams at once
    rep = serve.serve(sp, arr, ex, budget, compress=1.0, clock=clk, sleep=clk.sleep)
    assert len(rep.records) == len(arr)
    for b in range(len(sp)):
        assert ex.order[b] == list(range(6))
    assert rep.max_concurrent_bytes <= budget
    assert (rep.latencies() > 0).all()
    opened = [b for e, b in ex.events if e == "open"]
    assert sorted(opened) == [0, 1, 2, 3]
    s = rep.summary()
    assert s["gulps"] == 24 and s["p99_ms"] >= s["p50_ms"] > 0


def test_latency_breakdown_adds_up():
    # host wait + device queue + search is the latency; notice (the host
    # seeing a completion) comes after it
    clk = FakeClock()
    specs = specs4()
    arr = serve.poisson_arrivals(specs, 40.0, seed=5, gulps_per_beam=3)
    ex = SimExecutor(clk, rate=2e9)
    rep = serve.serve(specs, arr, ex, 1 << 40, compress=8.0, clock=clk, sleep=clk.sleep, slots=3)
    for r in rep.records:
        parts = (r.submitted - r.arrival) + (r.started - r.submitted) + (r.done - r.started)
        assert abs(parts - r.latency) < 1e-9
        assert r.submitted >= r.arrival and r.started >= r.submitted and r.noticed >= r.done
    bd = rep.summary()["breakdown"]
    assert set(bd) == {"host_wait", "device_queue", "search", "notice"}
    for v in bd.values():
        assert 0.0 <= v["p50_ms"] <= v["p99_ms"]
    # a record the executor did not time leaves the breakdown out
    rep.records[0].started = None
    rep.records = rep.records[:1]
    assert "breakdown" not in rep.summary()


def test_min_group_holds_gulps_for_shared_launches():
    # under load, ready gulps wait for min_group free slots and then go
    # together; with nothing on the device they go at once
    class GroupExecutor(SimExecutor):
        def __init__(self, *a, **kw):
            super().__init__(*a, **kw)
            self.groups = []

        def submit_many(self, group):
            self.groups.append(len(group))
            for rec, spec in group:
                self.submit(rec, spec)

    clk = FakeClock()
    sp = specs4()
    arr = serve.poisson_arrivals(sp, 10.0, seed=3, gulps_per_beam=8)
    out = {}
    for mg in (1, 4):
        ex = GroupExecutor(clk, rate=2e9)
        rep = serve.serve(sp, arr, ex, 1 << 40, compress=float("inf"), clock=clk, sleep=clk.sleep, slots=8,
                          min_group=mg)
        assert len(rep.records) == len(arr) and rep.max_inflight <= 8
        for b in range(len(sp)):
            assert ex.order[b] == list(range(8))
        out[mg] = ex.groups
    assert max(out[1][1:]) < 4  # one slot frees at a time
    assert min(out[4][:-1]) >= 4 and len(out[4]) < len(out[1])


def test_serve_saturation_latency_grows():
    # Offered load above the device rate: the backlog, hence p99, grows with compression.
    sp = specs4()
    arr = serve.poisson_arrivals(sp, 1.5, seed=5, gulps_per_beam=10)
    out = []
    for compress in (1.0, float("inf")):
        clk = FakeClock()
        ex = SimExecutor(clk, rate=1e9, foot=1)
        rep = serve.serve(sp, arr, ex, 10 ** 9, compress=compress, clock=clk, sleep=clk.sleep)
        out.append(rep.summary())
    assert out[1]["p99_ms"] > out[0]["p99_ms"]


@pytest.mark.gpu
def test_beam_in_mix_equals_alone_and_oracle():
    import torch
    import oracle
    import synth
    from parity import exact_equal
    from paper_2512_00398_amd import sps
    gulp = 4096
    blocks = [synth.Block(ndm=6, nsamp=6 * gulp, max_width=512, baseline_len=3000, seed=71, n_pulses=8,
                          pulse_width=(1, 256), pulse_snr=(6.0, 25.0), straddle_period=gulp),
              synth.Block(ndm=3, nsamp=6 * gulp, max_width=4096, baseline_len=5000, seed=72, n_pulses=8,
                          pulse_width=(1, 1024), pulse_snr=(6.0, 25.0), straddle_period=gulp),
              synth.Block(ndm=9, nsamp=6 * gulp, max_width=64, baseline_len=700, seed=73, n_pulses=8,
                          pulse_width=(1, 64), pulse_snr=(6.0, 25.0), straddle_period=gulp)]
    xs = [synth.generate(b) for b in blocks]
    dev = [torch.from_numpy(x).cuda() for x in xs]
    sp = [serve.BeamSpec(ndm=b.ndm, nsamp=gulp, max_width=b.max_width, baseline_len=b.baseline_len,
                         snr_thresh=5.0) for b in blocks]

    def source(beam, k):
        return dev[beam][:, k * gulp:(k + 1) * gulp].contiguous()

    def collect(kept):
        parts = []
        for c, off in kept:
            a = np.empty(c.size, dtype=oracle.CAND_DTYPE)
            a["sample"] = c["sample"].astype(np.int64) + off
            a["dm_idx"], a["width"], a["snr"] = c["dm_idx"], c["width"], c["snr"]
            parts.append(a)
        return oracle.sort_cands(np.concatenate(parts))

    arr = serve.poisson_arrivals(sp, 1.5, seed=9, gulps_per_beam=6)
    print("serve mix", [(s.ndm, s.nsamp, s.max_width) for s in sp], flush=True)
    ex = serve.GpuExecutor(source, nstreams=3, cand_cap=1 << 18, keep=True)
    rep = serve.serve(sp, arr, ex, budget=1 << 40, compress=float("inf"))
    assert len(rep.records) == 18
    # the gulps really were on the device together: submission never waits,
    # and the device intervals of gulps of all three beams overlap
    gulps, beams = ex.device_overlap()
    print("in flight at once: %d (scheduler), %d gulps of %d beams (device)" % (rep.max_inflight, gulps, beams),
          flush=True)
    assert rep.max_inflight >= 3
    assert beams >= 3
    bd = rep.summary()["breakdown"]  # every part timed on the device and the host
    print("latency parts", bd, flush=True)
    assert bd["search"]["p50_ms"] > 0 and all(v["p50_ms"] >= 0 for v in bd.values())
    for b in range(3):
        print("beam %d alone" % b, flush=True)
        alone_ex = serve.GpuExecutor(source, nstreams=1, cand_cap=1 << 18, keep=True)
        serve.serve(sp, [serve.Arrival(float(k), b, k) for k in range(6)], alone_ex, budget=1 << 40,
                    compress=float("inf"))
        mix = collect(ex.kept[b])
        alone = collect(alone_ex.kept[b])
        assert exact_equal(mix, alone), b
        ref = oracle.search(xs[b], blocks[b].max_width, blocks[b].baseline_len, 5.0)
        assert exact_equal(mix, ref), b


def test_serve_slots_cap_inflight_and_keep_order():
    clk = FakeClock()
    sp = specs4()
    ex = SimExecutor(clk, rate=1e9, foot=1)
    arr = serve.poisson_arrivals(sp, 1.5, seed=21, gulps_per_beam=8)
    rep = serve.serve(sp, arr, ex, 10 ** 9, compress=float("inf"), clock=clk, sleep=clk.sleep, slots=3)
    assert len(rep.records) == len(arr)
    assert rep.max_inflight == 3
    for b in range(len(sp)):
        assert ex.order[b] == list(range(8))


@pytest.mark.gpu
def test_batched_serving_equals_alone_and_oracle():
    # Continuous batching: gulps of four beams that are ready together go
    # through one launch per stage (sps_batch_push); each beam's candidates
    # equal the beam served alone (its own pushes) and the oracle.
    import torch
    import oracle
    import synth
    from parity import exact_equal
    gulp = 4096
    specs_ = [(6, 512, 3000, 91), (3, 4096, 5000, 92), (9, 64, 700, 93), (4, 1024, 2000, 94)]
    blocks = [synth.Block(ndm=nd, nsamp=5 * gulp, max_width=w, baseline_len=L, seed=sd, n_pulses=6,
                          pulse_width=(1, min(w, 256)), pulse_snr=(6.0, 25.0), straddle_period=gulp)
              for nd, w, L, sd in specs_]
    xs = [synth.generate(b) for b in blocks]
    dev = [torch.from_numpy(x).cuda() for x in xs]
    sp = [serve.BeamSpec(ndm=b.ndm, nsamp=gulp, max_width=b.max_width, baseline_len=b.baseline_len,
                         snr_thresh=5.0) for b in blocks]

    def source(beam, k):
        return dev[beam][:, k * gulp:(k + 1) * gulp].contiguous()

    def collect(kept):
        parts = []
        for c, off in kept:
            a = np.empty(c.size, dtype=oracle.CAND_DTYPE)
            a["sample"] = c["sample"].astype(np.int64) + off
            a["dm_idx"], a["width"], a["snr"] = c["dm_idx"], c["width"], c["snr"]
            parts.append(a)
        return oracle.sort_cands(np.concatenate(parts))

    arr = serve.poisson_arrivals(sp, 1.5, seed=19, gulps_per_beam=5)
    print("batched serve", [(s.ndm, s.nsamp, s.max_width) for s in sp], flush=True)
    ex = serve.GpuExecutor(source, cand_cap=1 << 18, keep=True, batch=True)
    rep = serve.serve(sp, arr, ex, budget=1 << 40, compress=float("inf"))
    assert len(rep.records) == 20
    print("launch sizes", ex.batch_sizes, flush=True)
    assert max(ex.batch_sizes) >= 3  # gulps of at least three beams shared one launch
    for b in range(len(sp)):
        alone_ex = serve.GpuExecutor(source, nstreams=1, cand_cap=1 << 18, keep=True)
        serve.serve(sp, [serve.Arrival(float(k), b, k) for k in range(5)], alone_ex, budget=1 << 40,
                    compress=float("inf"))
        mix, alone = collect(ex.kept[b]), collect(alone_ex.kept[b])
        assert exact_equal(mix, alone), b
        ref = oracle.search(xs[b], blocks[b].max_width, blocks[b].baseline_len, 5.0)
        assert exact_equal(mix, ref), b
