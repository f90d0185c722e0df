"""GPU tests of the resident batch and the serving loops (mp_batch_*,
mp_serve_*), called through the C ABI.

A batched RVE runs the same per-tile arithmetic in the same order as a solo
plan (mp_plan_*), and its step control (convergence test, extrapolation,
commit) runs on the device with the same code, so the bar is bit-for-bit
equality with the solo solve of the same problem: fields, per-step iteration
counts, step records and final status.  The solo FP64 path is itself held to
the oracle (test_gpu_parity); one batched RVE is also compared with the oracle
directly here.  Every graph replay is followed by eager host work (reads,
admissions, releases) before the next one.
"""
import numpy as np
import pytest

from oracle import micropolar as O
from paper_2409_10774_amd import workloads as W
from tests.test_gpu_parity import long_axis_workload, rel, say, small_workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_10774_amd import mp as _mp
    return _mp


FIELDS = ("e", "g", "t", "m", "p", "q")


def solo(mp, wl, precision, **kw):
    plan = mp.Plan(wl.phase_map, wl.phases, tol=wl.tol, precision=precision, **kw)
    st, it = plan.solve(wl.times, wl.E, wl.G, raise_on_error=False)
    n = plan.steps()
    rec = np.array([np.concatenate([plan.response(s), plan.error_parts(s)])
                    for s in range(1, n + 1)]).reshape(n, 47)
    out = dict(status=st, iters=it[:n], rec=rec, fields={k: plan.field(k) for k in FIELDS})
    plan.close()
    return out


def batched(B, rid):
    state, status, steps, iters = B.query(rid)
    rec = B.responses(rid)
    return dict(state=state, status=status, iters=[int(v) for v in rec[:, 41]], rec=rec,
                total=iters, fields={k: B.field(rid, k) for k in FIELDS})


def assert_same(a, b, tag):
    assert a["status"] == b["status"], (tag, a["status"], b["status"])
    assert a["iters"] == b["iters"], (tag, a["iters"], b["iters"])
    for k in FIELDS:
        assert np.array_equal(a["fields"][k], b["fields"][k]), (tag, k, rel(a["fields"][k], b["fields"][k]))
    assert np.array_equal(a["rec"], b["rec"]), (tag, np.abs(a["rec"] - b["rec"]).max())


def mixed_set(tol):
    """RVEs of three shape classes, different materials, paths and step counts."""
    out = []
    # seed 58 puts inclusions into the 24 x 16 x 12 crop (seed 43 leaves it homogeneous)
    for i, (n, steps, seed) in enumerate([((16, 16, 16), 3, 40), ((12, 6, 8), 4, 41),
                                          ((16, 16, 16), 2, 42), ((24, 16, 12), 3, 58),
                                          ((12, 6, 8), 2, 44), ((16, 16, 16), 4, 45)]):
        wl = small_workload(n, seed=seed, contrast=3.0 + 2 * i, steps=steps,
                            G_end=0.0 if i % 2 else 0.002)
        wl.tol = tol
        out.append(wl)
    return out


SHAPES = [(16, 16, 16), (12, 6, 8), (24, 16, 12)]


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-8), ("mixed", 1e-6)])
def test_batch_equals_solo(mp, precision, tol):
    say(f"case: batch of 6 RVEs in 3 shape classes vs solo plans, {precision}")
    wls = mixed_set(tol)
    B = mp.Batch(SHAPES, arena_bytes=256 << 20, precision=precision, max_rves=16,
                 iters_per_launch=8, autotune=True)
    for c in range(len(SHAPES)):
        sch = B.schedule(c)
        say("class", SHAPES[c], sch)
        nh = SHAPES[c][0] // 2
        for p in ("y_fwd", "z_green", "y_inv"):
            assert sch[p]["tx"] >= 1 and nh % sch[p]["tx"] == 0 and sch[p]["grid"] > 0
    ids = [B.admit(w.phase_map, w.phases, w.times, w.E, w.G, tol=w.tol) for w in wls]
    launches = B.drain()
    say("graph launches", launches, B.stats())
    for rid, w in zip(ids, wls):
        b = batched(B, rid)
        assert b["state"] == mp.MP_RVE_DONE
        s = solo(mp, w, precision)
        say(f"  rve {rid} n={w.phase_map.shape} iters {b['iters']} solo {s['iters']}")
        assert_same(b, s, rid)
        assert b["total"] == sum(s["iters"])
    B.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-8), ("mixed", 1e-6)])
def test_batch_long_axis_equals_solo(mp, precision, tol):
    """Classes with 256- and 192-point axes (x passes with one Alg. 1 level
    per block, one-wide z tiles) in one batch: bit for bit the solo plans."""
    shapes = [(256, 6, 4), (4, 6, 256), (192, 4, 6)]
    say(f"case: batch of thin long-axis RVEs {shapes} vs solo plans, {precision}")
    wls = []
    for n in shapes:
        w = long_axis_workload(n, seed=sum(n))
        w.tol = tol
        wls.append(w)
    B = mp.Batch(shapes, arena_bytes=256 << 20, precision=precision, max_rves=8,
                 iters_per_launch=8, autotune=True)
    ids = [B.admit(w.phase_map, w.phases, w.times, w.E, w.G, tol=w.tol) for w in wls]
    launches = B.drain()
    say("graph launches", launches)
    for rid, w in zip(ids, wls):
        b = batched(B, rid)
        assert b["state"] == mp.MP_RVE_DONE
        s = solo(mp, w, precision)
        say(f"  rve {rid} n={w.phase_map.shape} iters {b['iters']} solo {s['iters']}")
        assert_same(b, s, rid)
        assert b["total"] == sum(s["iters"])
    B.close()


def test_batch_rve_against_oracle(mp):
    say("case: one batched FP64 RVE against the oracle")
    wl = small_workload((12, 6, 8), seed=7, steps=3)
    B = mp.Batch([(12, 6, 8)], arena_bytes=64 << 20, precision="fp64", max_rves=4)
    rid = B.admit(wl.phase_map, wl.phases, wl.times, wl.E, wl.G, tol=wl.tol)
    B.drain()
    b = batched(B, rid)
    out = O.Solver(wl.phase_map, wl.phases, h=wl.h, tol=wl.tol).solve(
        wl.times, wl.E, wl.G, fields_at=(len(wl.E),))
    assert b["iters"] == out["iters"], (b["iters"], out["iters"])
    f = out["fields"][len(wl.E)]
    errs = {k: rel(b["fields"][k], f[k]) for k in FIELDS if np.abs(f[k]).max() > 0}
    say("field rel", errs)
    assert max(errs.values()) < 1e-10
    big = np.abs(out["resp"]).max(axis=0) > 1e-12 * np.abs(out["resp"]).max()
    curve = np.abs(b["rec"][:, :40] - out["resp"]).max(axis=0) / np.maximum(
        np.abs(out["resp"]).max(axis=0), 1e-300)
    assert curve[big].max() < 1e-10
    B.close()


def test_batch_alone_vs_mix_with_failures(mp):
    """RVEs that stop early (max_iter reached, divergence) next to normal
    ones: every RVE's result equals its solo solve, statuses included."""
    say("case: alone vs mix, with a not-converging and a diverging RVE")
    sph = W.single_sphere_16()
    sph_short = W.Workload("sph", sph.phase_map, sph.phases, sph.times[:4], sph.E[:3], sph.G[:3],
                           tol=sph.tol)
    normal = small_workload((16, 16, 16), seed=3, steps=3)
    items = [(sph_short, dict(max_iter=3)), (sph_short, dict(ref_mode="volume_mean")), (normal, {}),
             (sph_short, {})]
    B = mp.Batch([(16, 16, 16)], arena_bytes=128 << 20, precision="fp64", max_rves=8)
    ids = [B.admit(w.phase_map, w.phases, w.times, w.E, w.G, tol=w.tol, **kw) for w, kw in items]
    B.drain()
    for rid, (w, kw) in zip(ids, items):
        b = batched(B, rid)
        s = solo(mp, w, "fp64", **kw)
        say(f"  rve {rid} {kw} status {b['status']} solo {s['status']} iters {b['iters']}")
        assert_same(b, s, rid)
    assert batched(B, ids[0])["status"] == mp.MP_E_NOT_CONVERGED
    assert batched(B, ids[1])["status"] == mp.MP_E_DIVERGED
    assert B.query(ids[1])[2] == 0          # the diverged step is not committed
    B.close()


def test_batch_continuous_admission_and_release(mp):
    """Admissions between graph launches, release of finished RVEs and reuse
    of their arena regions; every result equals its solo solve."""
    say("case: continuous admission / release")
    wls = mixed_set(1e-8)
    B = mp.Batch(SHAPES, arena_bytes=256 << 20, precision="fp64", max_rves=16, iters_per_launch=4)
    first = [B.admit(w.phase_map, w.phases, w.times, w.E, w.G, tol=w.tol) for w in wls[:3]]
    for _ in range(3):
        B.run()
    later = [B.admit(w.phase_map, w.phases, w.times, w.E, w.G, tol=w.tol) for w in wls[3:5]]
    B.drain()
    done = dict(zip(first + later, wls[:5]))
    for rid, w in done.items():
        assert_same(batched(B, rid), solo(mp, w, "fp64"), rid)
    used = B.stats()["arena_used"]
    for rid in first:
        B.release(rid)
    assert B.stats()["arena_used"] < used
    again = B.admit(wls[5].phase_map, wls[5].phases, wls[5].times, wls[5].E, wls[5].G, tol=wls[5].tol)
    B.drain()
    assert_same(batched(B, again), solo(mp, wls[5], "fp64"), again)
    for rid in later:
        assert_same(batched(B, rid), solo(mp, done[rid], "fp64"), rid)
    B.close()


def test_batch_admission_by_footprint(mp):
    say("case: admission refused when the arena is full, accepted after a release")
    w = small_workload((16, 16, 16), seed=11, steps=2)
    probe = mp.Batch([(16, 16, 16)], arena_bytes=8 << 20, precision="fp64", max_rves=4)
    need = probe.footprint(w.phase_map, w.phases, len(w.E))
    probe.close()
    head = 1 << 20   # descriptors and lists
    B = mp.Batch([(16, 16, 16)], arena_bytes=head + need + need // 2, precision="fp64", max_rves=4,
                 autotune=False)
    a = B.admit(w.phase_map, w.phases, w.times, w.E, w.G, tol=w.tol)
    rid, st = B.admit(w.phase_map, w.phases, w.times, w.E, w.G, tol=w.tol, raise_on_error=False)
    assert rid is None and st == mp.MP_E_NOMEM
    B.drain()
    B.release(a)
    b = B.admit(w.phase_map, w.phases, w.times, w.E, w.G, tol=w.tol)
    B.drain()
    assert_same(batched(B, b), solo(mp, w, "fp64"), b)
    B.close()


def assert_reply(reqs, i, ref, tag):
    """A served request's reply (step records, final fields) equals the solo
    solve of the same precision bit for bit."""
    rec = reqs.records[i]
    n = len(ref["iters"])
    assert np.array_equal(rec[:n, :47], ref["rec"]), (tag, np.abs(rec[:n, :47] - ref["rec"]).max())
    assert np.isnan(rec[n:]).all()
    for k in FIELDS:
        got = reqs.fields[i][k]
        got = got.cpu().numpy() if hasattr(got, "cpu") else got
        assert np.array_equal(got, ref["fields"][k]), (tag, k)


def test_serving_loops(mp):
    """A short Poisson trace through continuous batching (mixed, fields
    delivered into device memory) and through the sequential FP64 server
    (host memory): every request answered, and every reply (step records and
    final fields) equal to the solo solve of the same precision bit for bit,
    alone against in the mix."""
    say("case: serving loops on a 6-request trace")
    rng = np.random.default_rng(5)
    wls = mixed_set(1e-6)
    arrivals = np.cumsum(rng.exponential(0.02, size=len(wls)))
    import torch
    items = [(a, w.phase_map, w.phases, w.times, w.E, w.G, dict(tol=w.tol)) for a, w in zip(arrivals, wls)]
    B = mp.Batch(SHAPES, arena_bytes=256 << 20, precision="mixed", max_rves=16, iters_per_launch=8)
    reqs = mp.Requests(items, precision="mixed", fields=FIELDS, device="cuda:0")
    ta, td, st, it = mp.serve_batched(B, reqs)
    say("batched admit", np.round(ta, 3), "done", np.round(td, 3), "iters", it)
    assert (st == mp.MP_OK).all()
    assert (ta >= arrivals - 1e-9).all() and (td >= ta).all()
    for i, w in enumerate(wls):
        ref = solo(mp, w, "mixed")
        assert it[i] == sum(ref["iters"])
        assert_reply(reqs, i, ref, ("batched", i))
    assert B.stats()["resident"] == 0
    B.close()
    ws = torch.empty(64 << 20, dtype=torch.uint8, device="cuda:0")
    reqs64 = mp.Requests(items, precision="fp64", fields=FIELDS)
    ts, td2, st2, it2 = mp.serve_sequential(reqs64, ws)
    say("sequential start", np.round(ts, 3), "done", np.round(td2, 3), "iters", it2)
    assert (st2 == mp.MP_OK).all() and (td2 >= ts).all() and (ts >= arrivals - 1e-9).all()
    for i, w in enumerate(wls):
        ref = solo(mp, w, "fp64")
        assert it2[i] == sum(ref["iters"])
        assert_reply(reqs64, i, ref, ("sequential", i))


def test_serving_fp64_reply_against_oracle(mp):
    """The reply of a request served by continuous batching in FP64 (next to
    another request) against the oracle: equal iteration counts, response
    curves and fields within 1e-10."""
    say("case: FP64 served reply against the oracle")
    wls = mixed_set(1e-8)[:2]
    items = [(0.0, w.phase_map, w.phases, w.times, w.E, w.G, dict(tol=w.tol)) for w in wls]
    B = mp.Batch(SHAPES, arena_bytes=128 << 20, precision="fp64", max_rves=4, iters_per_launch=8)
    reqs = mp.Requests(items, precision="fp64", fields=FIELDS)
    ta, td, st, it = mp.serve_batched(B, reqs)
    B.close()
    assert (st == mp.MP_OK).all()
    w = wls[0]
    out = O.Solver(w.phase_map, w.phases, tol=w.tol).solve(w.times, w.E, w.G, fields_at=(len(w.E),))
    rec = reqs.records[0]
    assert [int(v) for v in rec[:, 41]] == out["iters"]
    f = out["fields"][len(w.E)]
    errs = {k: rel(reqs.fields[0][k], f[k]) for k in FIELDS}
    big = np.abs(out["resp"]).max(axis=0) > 1e-12 * np.abs(out["resp"]).max()
    curve = np.abs(rec[:, :40] - out["resp"]).max(axis=0) / np.maximum(np.abs(out["resp"]).max(axis=0), 1e-300)
    say("iterations", out["iters"], "field rel", errs, "curve rel %.2e" % curve[big].max())
    assert max(errs.values()) < 1e-10 and curve[big].max() < 1e-10


def test_batch_cancel_slot_limit_and_empty(mp):
    """Releasing an unfinished RVE cancels it without disturbing the others;
    admission beyond max_rves is refused with MP_E_NOMEM; a batch with
    nothing resident runs and reports zero active RVEs."""
    say("case: cancel, slot limit, empty batch")
    wls = mixed_set(1e-8)[:3]
    B = mp.Batch(SHAPES, arena_bytes=256 << 20, precision="fp64", max_rves=2, iters_per_launch=4)
    assert B.run() == 0 and B.drain() == 1
    a = B.admit(wls[0].phase_map, wls[0].phases, wls[0].times, wls[0].E, wls[0].G, tol=wls[0].tol)
    b = B.admit(wls[1].phase_map, wls[1].phases, wls[1].times, wls[1].E, wls[1].G, tol=wls[1].tol)
    rid, st = B.admit(wls[2].phase_map, wls[2].phases, wls[2].times, wls[2].E, wls[2].G, tol=wls[2].tol,
                      raise_on_error=False)
    assert rid is None and st == mp.MP_E_NOMEM
    B.run()
    assert B.query(a)[0] == mp.MP_RVE_RUNNING
    B.release(a)                        # cancel mid-path
    c = B.admit(wls[2].phase_map, wls[2].phases, wls[2].times, wls[2].E, wls[2].G, tol=wls[2].tol)
    B.drain()
    assert_same(batched(B, b), solo(mp, wls[1], "fp64"), b)
    assert_same(batched(B, c), solo(mp, wls[2], "fp64"), c)
    B.close()


def test_drain_in_bounded_calls_equals_solo(mp):
    """mp_batch_drain queues each graph launch before reading back the state
    after the previous one; with max_launches it stops at that many launches
    (1, then 3), RVEs stay resident and running, and the rest of the drain
    finishes them equal bit for bit to their solo plans."""
    say("case: drain split into bounded calls, mixed, 3 RVEs")
    wls = mixed_set(1e-6)[:3]
    B = mp.Batch(SHAPES, arena_bytes=256 << 20, precision="mixed", max_rves=8, iters_per_launch=4)
    ids = [B.admit(w.phase_map, w.phases, w.times, w.E, w.G, tol=w.tol) for w in wls]
    assert B.drain(1) == 1
    assert any(B.query(i)[0] == mp.MP_RVE_RUNNING for i in ids)
    assert B.drain(3) == 3
    rest = B.drain()
    say("launches after the bounded calls", rest)
    assert rest >= 1
    for rid, w in zip(ids, wls):
        b = batched(B, rid)
        assert b["state"] == mp.MP_RVE_DONE
        assert_same(b, solo(mp, w, "mixed"), rid)
    assert B.drain() == 1   # nothing left: one launch, no work
    B.close()
