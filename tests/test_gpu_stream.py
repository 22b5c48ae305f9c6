"""GPU streaming: gulp-by-gulp search equals the one-shot oracle on the concatenation.

Candidates from every push (sample + gulp offset) and from the final flush
(sample + end offset) must equal the oracle's candidates for the whole
observation; checkpoint/restore mid-stream must not change anything.
"""
import numpy as np
import pytest

import oracle
import synth
from parity import compare_cands, exact_equal

pytestmark = pytest.mark.gpu


def sps():
    from paper_2512_00398_amd import sps as m
    return m


def run_stream(x, gulp, max_width, L, theta, restore_after=None, detect_seg=0, stats_seg=0, norm=0, graph=False):
    import torch
    m = sps()
    ndm, total = x.shape
    assert total % gulp == 0
    print("stream case ndm=%d total=%d gulp=%d w=%d L=%d restore=%s norm=%d graph=%s" % (
        ndm, total, gulp, max_width, L, restore_after, norm, graph), flush=True)
    parts = []
    with m.Plan(ndm, gulp, max_width, L, theta) as plan:
        if detect_seg:
            plan.set(m.ATTR_DETECT_SEG, detect_seg)
        if stats_seg:
            plan.set(m.ATTR_STATS_SEG, stats_seg)
        if norm:
            plan.set(m.ATTR_NORM, norm)
        cands, ncand = plan.alloc_cands()
        st = m.Stream(plan)
        buf = torch.empty((ndm, gulp), dtype=torch.float32, device="cuda")
        for g in range(total // gulp):
            xd = torch.from_numpy(np.ascontiguousarray(x[:, g * gulp:(g + 1) * gulp])).cuda()
            if graph:  # replays read one fixed buffer
                buf.copy_(xd)
                xd = buf
            off = st.push(xd, cands, ncand, graph=graph)
            torch.cuda.synchronize()
            assert off == g * gulp
            c = m.cands_to_numpy(cands, ncand, plan.max_cands)
            parts.append((c, off))
            if restore_after is not None and g == restore_after:
                state = st.save()
                st.close()
                st = m.Stream(plan)
                st.restore(state)
        end = st.flush(cands, ncand)
        torch.cuda.synchronize()
        assert end == total
        parts.append((m.cands_to_numpy(cands, ncand, plan.max_cands), end))
        st.close()
    out = []
    for c, off in parts:
        a = np.empty(c.size, dtype=oracle.CAND_DTYPE)
        a["sample"] = c["sample"].astype(np.int64) + off
        a["dm_idx"], a["width"], a["snr"] = c["dm_idx"], c["width"], c["snr"]
        out.append(a)
    return oracle.sort_cands(np.concatenate(out))


CASES = [
    # gulp shorter than the baseline window (history shifts within itself)
    dict(name="short-gulps", ndm=6, total=16384, gulp=2048, w=64, L=4096, theta=5.0),
    # gulp shorter than the widest boxcar
    dict(name="gulp<maxw", ndm=4, total=8192, gulp=1024, w=2048, L=700, theta=4.0),
    # minimal gulp of one block
    dict(name="gulp=64", ndm=3, total=4096, gulp=64, w=128, L=200, theta=3.5),
    # long gulps, every width, pulses across gulp edges
    dict(name="long-gulps", ndm=8, total=8 * 8192, gulp=8192, w=4096, L=4096, theta=5.0),
]


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_stream_equals_one_shot(case):
    b = synth.Block(ndm=case["ndm"], nsamp=case["total"], max_width=case["w"], baseline_len=case["L"],
                    seed=99, n_pulses=12, pulse_width=(1, min(512, case["w"])), pulse_snr=(6.0, 30.0),
                    straddle_period=case["gulp"])
    x = synth.generate(b)
    got = run_stream(x, case["gulp"], case["w"], case["L"], case["theta"])
    ref = oracle.search(x, case["w"], case["L"], case["theta"])
    assert compare_cands(got, ref, case["theta"], case["name"]) == 0
    assert exact_equal(got, ref)
    assert ref.size > 0


def test_stream_checkpoint_restore_and_tilings():
    b = synth.Block(ndm=5, nsamp=6 * 4096, max_width=1024, baseline_len=3000, seed=7, n_pulses=10,
                    pulse_width=(1, 512), pulse_snr=(6.0, 25.0), straddle_period=4096)
    x = synth.generate(b)
    ref = oracle.search(x, 1024, 3000, 5.0)
    plain = run_stream(x, 4096, 1024, 3000, 5.0)
    restored = run_stream(x, 4096, 1024, 3000, 5.0, restore_after=2)
    tiled = run_stream(x, 4096, 1024, 3000, 5.0, detect_seg=1024, stats_seg=64)
    assert exact_equal(plain, ref)
    assert exact_equal(restored, ref)
    assert exact_equal(tiled, ref)


def test_stream_workload_rows_full_length():
    # The streaming workload's gulp shape (2^18 samples, 13 widths, window
    # 16384, pulses straddling gulp edges) on a subset of its rows.
    cfg = synth.config(3)
    b = cfg["blocks"][0].with_(ndm=32)
    gulp = cfg["gulp"]
    x = synth.generate(b)
    got = run_stream(x, gulp, b.max_width, b.baseline_len, b.snr_thresh)
    rows = [0, 13, 31]
    ref = oracle.search(x, b.max_width, b.baseline_len, b.snr_thresh, rows=rows)
    sel = np.isin(got["dm_idx"], rows)
    assert compare_cands(got[sel], ref, b.snr_thresh, "c3-rows") == 0
    assert exact_equal(got[sel], ref)


def gulp_scaled_block(seed, ndm, gulp, ngulps, w, L, factors):
    # every gulp's samples multiplied by its own integer factor: the noise
    # level changes from gulp to gulp, so one scale per gulp differs from
    # the block scale and from one scale for the whole row
    b = synth.Block(ndm=ndm, nsamp=gulp * ngulps, max_width=w, baseline_len=L, seed=seed, n_pulses=10,
                    pulse_width=(1, min(w, 256)), pulse_snr=(8.0, 30.0), straddle_period=gulp)
    x = synth.generate(b).astype(np.float64)
    for g in range(ngulps):
        x[:, g * gulp:(g + 1) * gulp] *= factors[g % len(factors)]
    return x.astype(np.float32)


ROW_SCALE_CASES = [
    dict(name="short-gulps", ndm=5, gulp=2048, ngulps=6, w=256, L=3000, theta=5.0, factors=(1, 3, 2)),
    dict(name="gulp=64", ndm=3, gulp=64, ngulps=40, w=128, L=200, theta=4.0, factors=(1, 2)),
    dict(name="long-gulps", ndm=6, gulp=16384, ngulps=4, w=4096, L=4096, theta=5.5, factors=(2, 1, 4, 1)),
]


@pytest.mark.parametrize("case", ROW_SCALE_CASES, ids=[c["name"] for c in ROW_SCALE_CASES])
def test_stream_row_scale_per_gulp(case):
    # SPS_ATTR_NORM = 1 in a stream: one row scale per gulp (the oracle's
    # reading 10 with the gulp as the chunk), eager, after a checkpoint and
    # from captured graphs
    x = gulp_scaled_block(1200 + len(case["name"]), case["ndm"], case["gulp"], case["ngulps"], case["w"], case["L"],
                          case["factors"])
    g = case["gulp"]
    gulps = [x[:, k * g:(k + 1) * g] for k in range(case["ngulps"])]
    ref = oracle.search_stream(gulps, case["w"], case["L"], case["theta"], row_norm=True)
    got = run_stream(x, g, case["w"], case["L"], case["theta"], norm=1)
    assert compare_cands(got, ref, case["theta"], case["name"]) == 0
    assert exact_equal(got, ref)
    assert ref.size > 0
    assert not exact_equal(ref, oracle.search(x, case["w"], case["L"], case["theta"], row_norm=True))
    restored = run_stream(x, g, case["w"], case["L"], case["theta"], norm=1, restore_after=case["ngulps"] // 2)
    assert exact_equal(restored, ref)
    graphed = run_stream(x, g, case["w"], case["L"], case["theta"], norm=1, graph=True)
    assert exact_equal(graphed, ref)


def test_stream_scale_attribute_checked_at_push():
    import torch
    m = sps()
    with m.Plan(2, 4096, 64, 1000, 5.0) as p:
        p.set(m.ATTR_NORM, 1)
        st = m.Stream(p)
        c, n = p.alloc_cands()
        x = torch.zeros((2, 4096), dtype=torch.float32, device="cuda")
        st.push(x, c, n)
        p.set(m.ATTR_NORM, 2)  # the per-width scale needs the whole filtered series
        with pytest.raises(m.SpsError):
            st.push(x, c, n)
        with pytest.raises(m.SpsError):
            st.push(x, c, n, graph=True)
        p.set(m.ATTR_NORM, 0)
        st.push(x, c, n)
        torch.cuda.synchronize()
        st.close()


def test_graph_gulp_step_matches_eager_every_replay():
    # The captured gulp step is replayed once per gulp from a fixed input
    # buffer refilled by eager copies; every replay must equal the eager push.
    import torch
    m = sps()
    b = synth.Block(ndm=6, nsamp=10 * 2048, max_width=512, baseline_len=3000, seed=31, n_pulses=10,
                    pulse_width=(1, 256), pulse_snr=(6.0, 25.0), straddle_period=2048)
    x = synth.generate(b)
    gulp = 2048
    ref = oracle.search(x, 512, 3000, 5.0)
    with m.Plan(6, gulp, 512, 3000, 5.0) as pe, m.Plan(6, gulp, 512, 3000, 5.0) as pg:
        ce, ne = pe.alloc_cands()
        cg, ng = pg.alloc_cands()
        se, sg = m.Stream(pe), m.Stream(pg)
        buf = torch.empty((6, gulp), dtype=torch.float32, device="cuda")
        out = []
        for g in range(x.shape[1] // gulp):
            print("graph replay %d" % g, flush=True)
            buf.copy_(torch.from_numpy(np.ascontiguousarray(x[:, g * gulp:(g + 1) * gulp])))
            off_g = sg.push(buf, cg, ng, graph=True)
            torch.cuda.synchronize()
            got_g = m.cands_to_numpy(cg, ng, pg.max_cands)
            off_e = se.push(buf, ce, ne)
            torch.cuda.synchronize()
            got_e = m.cands_to_numpy(ce, ne, pe.max_cands)
            assert off_g == off_e == g * gulp
            assert exact_equal(got_g, got_e), "replay %d differs from the eager push" % g
            a = np.empty(got_g.size, dtype=oracle.CAND_DTYPE)
            a["sample"] = got_g["sample"].astype(np.int64) + off_g
            a["dm_idx"], a["width"], a["snr"] = got_g["dm_idx"], got_g["width"], got_g["snr"]
            out.append(a)
        end = sg.flush(cg, ng)
        torch.cuda.synchronize()
        last = m.cands_to_numpy(cg, ng, pg.max_cands)
        a = np.empty(last.size, dtype=oracle.CAND_DTYPE)
        a["sample"] = last["sample"].astype(np.int64) + end
        a["dm_idx"], a["width"], a["snr"] = last["dm_idx"], last["width"], last["snr"]
        out.append(a)
        se.close()
        sg.close()
    got = oracle.sort_cands(np.concatenate(out))
    assert exact_equal(got, ref)


def test_graph_rotating_buffers_equal_one_shot():
    # Three input buffers and two candidate buffers in rotation: six buffer
    # triples, each captured once and replayed; more triples than the cache
    # holds once a fourth input buffer joins for the last gulps.
    import torch
    m = sps()
    gulp, ng = 2048, 14
    b = synth.Block(ndm=5, nsamp=ng * gulp, max_width=1024, baseline_len=2500, seed=57, n_pulses=12,
                    pulse_width=(1, 512), pulse_snr=(6.0, 25.0), straddle_period=gulp)
    x = synth.generate(b)
    ref = oracle.search(x, 1024, 2500, 5.0)
    out = []
    with m.Plan(5, gulp, 1024, 2500, 5.0) as p:
        bufs = [torch.empty((5, gulp), dtype=torch.float32, device="cuda") for _ in range(4)]
        cb = [p.alloc_cands() for _ in range(3)]
        st = m.Stream(p)
        for g in range(ng):
            xb = bufs[g % 3] if g < 10 else bufs[3 if g % 2 else g % 3]
            c, n = cb[g % 2] if g < 12 else cb[2]
            print("rotating graph push %d" % g, flush=True)
            xb.copy_(torch.from_numpy(np.ascontiguousarray(x[:, g * gulp:(g + 1) * gulp])))
            off = st.push(xb, c, n, graph=True)
            torch.cuda.synchronize()
            got = m.cands_to_numpy(c, n, p.max_cands)
            a = np.empty(got.size, dtype=oracle.CAND_DTYPE)
            a["sample"] = got["sample"].astype(np.int64) + off
            a["dm_idx"], a["width"], a["snr"] = got["dm_idx"], got["width"], got["snr"]
            out.append(a)
        c, n = cb[0]
        end = st.flush(c, n)
        torch.cuda.synchronize()
        last = m.cands_to_numpy(c, n, p.max_cands)
        a = np.empty(last.size, dtype=oracle.CAND_DTYPE)
        a["sample"] = last["sample"].astype(np.int64) + end
        a["dm_idx"], a["width"], a["snr"] = last["dm_idx"], last["width"], last["snr"]
        out.append(a)
        st.close()
    assert exact_equal(oracle.sort_cands(np.concatenate(out)), ref)


def test_stream_validation_rejects_bad_gulp():
    import torch
    m = sps()
    x = np.zeros((2, 1024), dtype=np.float32)
    with m.Plan(2, 1024, 64, 300, 5.0) as p:
        p.set(m.ATTR_VALIDATE, 1)
        c, n = p.alloc_cands()
        st = m.Stream(p)
        assert st.push(torch.from_numpy(x).cuda(), c, n) == 0
        x[1, 5] = 0.25
        with pytest.raises(m.SpsError) as e:
            st.push(torch.from_numpy(x).cuda(), c, n)
        assert e.value.code == m.SPS_ERR_DOMAIN
        with pytest.raises(m.SpsError):
            st.push(torch.from_numpy(x).cuda(), c, n, graph=True)
        # the rejected gulp was not pushed: the next one continues at 1024
        x[1, 5] = 0.0
        assert st.push(torch.from_numpy(x).cuda(), c, n) == 1024
        torch.cuda.synchronize()
        st.close()


def _globalise(c, off):
    a = np.empty(c.size, dtype=oracle.CAND_DTYPE)
    a["sample"] = c["sample"].astype(np.int64) + off
    a["dm_idx"], a["width"], a["snr"] = c["dm_idx"], c["width"], c["snr"]
    return a


def test_batch_push_equals_stream_push_and_oracle():
    # Gulps of three streams of different shapes and parameters pushed
    # together (one persistent launch per stage per round, sps_batch_push):
    # each stream's candidates and offsets equal its own pushes and the oracle
    # on its concatenated observation.
    import torch
    m = sps()
    shapes = [(6, 4096, 512, 3000, 5.0, 3), (3, 8192, 4096, 5000, 5.5, 3), (9, 2048, 64, 700, 4.5, 3),
              (4, 2048, 256, 1500, 5.0, 3)]
    norms = [0, 0, 0, 1]  # the last stream takes one row scale per gulp
    blocks = [synth.Block(ndm=nd, nsamp=g * ng, max_width=w, baseline_len=L, snr_thresh=th, seed=810 + k, n_pulses=6,
                          pulse_width=(1, min(w, 256)), pulse_snr=(6.0, 25.0), straddle_period=g)
              for k, (nd, g, w, L, th, ng) in enumerate(shapes)]
    xs = [synth.generate(b) for b in blocks]
    xs[3] = gulp_scaled_block(833, 4, 2048, 3, 256, 1500, (1, 3, 2))
    plans = [m.Plan(nd, g, w, L, th) for (nd, g, w, L, th, _) in shapes]
    for p, nrm in zip(plans, norms):
        p.set(m.ATTR_NORM, nrm)
    streams = [m.Stream(p) for p in plans]
    bufs = [p.alloc_cands() for p in plans]
    parts = [[] for _ in shapes]
    print("batch push of %d streams" % len(shapes), flush=True)
    with m.Batch() as b:
        with pytest.raises(m.SpsError):  # one gulp per stream and call
            g0 = torch.from_numpy(np.ascontiguousarray(xs[0][:, :shapes[0][1]])).cuda()
            b.push([streams[0], streams[0]], [g0, g0], [bufs[0][0]] * 2, [bufs[0][1]] * 2)
        for k in range(3):
            gulps = [torch.from_numpy(np.ascontiguousarray(x[:, k * s[1]:(k + 1) * s[1]])).cuda()
                     for x, s in zip(xs, shapes)]
            offs = b.push(streams, gulps, [c for c, _ in bufs], [n for _, n in bufs])
            torch.cuda.synchronize()
            assert offs == [k * s[1] for s in shapes]
            for i, (c, n) in enumerate(bufs):
                parts[i].append(_globalise(m.cands_to_numpy(c, n, plans[i].max_cands), offs[i]))
    for i, (st, (c, n)) in enumerate(zip(streams, bufs)):
        end = st.flush(c, n)
        torch.cuda.synchronize()
        parts[i].append(_globalise(m.cands_to_numpy(c, n, plans[i].max_cands), end))
        got = oracle.sort_cands(np.concatenate(parts[i]))
        nd, g, w, L, th, ng = shapes[i]
        alone = run_stream(xs[i], g, w, L, th, norm=norms[i])
        assert exact_equal(got, alone), i
        ref = oracle.search_stream([xs[i][:, k * g:(k + 1) * g] for k in range(ng)], w, L, th, row_norm=bool(norms[i]))
        assert compare_cands(got, ref, th, "batch push %d" % i) == 0 and exact_equal(got, ref), i
        st.close()
    for p in plans:
        p.close()


def test_streams_on_random_shapes_equal_oracle():
    # Seeded random streams (gulp lengths that are multiples of 64, widths,
    # windows, thresholds, the block scale or one row scale per gulp, noise
    # changing from gulp to gulp): every stream equals the oracle's reading of
    # its concatenated gulps.
    rng = np.random.default_rng(909)
    for trial in range(8):
        gulp = 64 * int(rng.integers(1, 64))
        ng = int(rng.integers(2, 7))
        w = 1 << int(rng.integers(0, 11))
        L = int(rng.integers(1, 6000))
        th = float(rng.uniform(3.5, 6.0))
        norm = int(rng.integers(0, 2))
        ndm = int(rng.integers(1, 6))
        factors = tuple(int(f) for f in rng.integers(1, 4, size=3))
        x = gulp_scaled_block(4000 + trial, ndm, gulp, ng, w, L, factors)
        print("random stream %d: ndm=%d gulp=%d x%d w=%d L=%d norm=%d" % (trial, ndm, gulp, ng, w, L, norm),
              flush=True)
        got = run_stream(x, gulp, w, L, th, norm=norm, graph=bool(trial % 2))
        ref = oracle.search_stream([x[:, k * gulp:(k + 1) * gulp] for k in range(ng)], w, L, th,
                                   row_norm=bool(norm))
        assert compare_cands(got, ref, th, "random stream %d" % trial) == 0
        assert exact_equal(got, ref), trial
