"""Full-size parity on the 128^3 and 256^3 cells, in the launch configuration
the benchmark times, through the C ABI.

- 128^3 cell (40 spheres, contrast 10, E11 and Gamma12 ramps, tolerance 1e-8),
  first three load steps converged on their own schedule against the oracle's
  (tests/golden/spheres128_steps3.npz, written by make_spheres128_golden.py
  from the oracle alone): equal iteration counts per step, the 40 averages of
  every step and the final fields at 4352 sampled voxels (random ones, an x
  row and a z column through a sphere) within 1e-10.  This crosses Alg. 2's
  extrapolated first iterates and commits at full size.
- 128^3 cell, three steps of three loop iterations each against the oracle
  run here on the same schedule: every field element by element within 1e-10.
- 256^3 cell in the mixed form, step 1 on a fixed schedule of two iterations,
  against the oracle on the same schedule (tests/golden/spheres256_step1.npz,
  make_spheres256_golden.py): fields at the sampled voxels and the averages
  within 1e-4 of their scale.
- the same 256^3 cell and schedule in FP64 (the largest grid, with 256-point
  x rows on one Alg. 1 level per block and one-wide z tiles), against the same
  expected values: fields and averages within 1e-10.
- many-RVE workload at full size: RVEs of 32^3, 64^3, 96^3 and 128^3 from it
  (contrast up to 20, tolerance 1e-6, mixed) in one batch, each equal bit for
  bit to its solo plan (whose FP64 path the tests above hold to the oracle).
- serving at full size: a 256^3 request beside 32^3 and 64^3 ones through
  continuous batching (mixed), every reply (step records, final fields) equal
  bit for bit to the request solved alone.
"""
import os

import numpy as np
import pytest

from oracle import micropolar as O
from paper_2409_10774_amd import workloads as W
from tests.test_gpu_batch import FIELDS as BFIELDS, assert_reply, assert_same, batched, solo
from tests.test_gpu_parity import rel, say

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
FIELDS = ("e", "g", "t", "m", "p", "q")


@pytest.fixture(scope="module")
def mp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_10774_amd import mp as _mp
    return _mp


def sampled(fields, idx):
    return {k: (v.reshape(9, -1)[:, idx] if k in "egtm" else v.reshape(-1)[idx]) for k, v in fields.items()}


def curve_rel(a, b):
    big = np.abs(b).max(axis=0) > 1e-12 * np.abs(b).max()
    return (np.abs(a - b).max(axis=0)[big] / np.abs(b).max(axis=0)[big]).max()


def test_spheres128_three_converged_steps_vs_oracle(mp):
    gold = np.load(os.path.join(GOLDEN, "spheres128_steps3.npz"))
    wl = W.random_spheres_128(n_steps=3)
    say("case: 128^3 cell, 3 converged load steps vs the oracle's expected values")
    plan = mp.Plan(wl.phase_map, wl.phases, tol=wl.tol)
    it = plan.solve(wl.times, wl.E, wl.G)
    say("iterations", it, "oracle", gold["iters"].tolist())
    resp = plan.responses()[:, :40]
    got = sampled(plan.fields(), gold["idx"])
    plan.close()
    if it != gold["iters"].tolist():
        # compare on the oracle's schedule as well, to tell a count shift
        # from a difference in the fields
        plan = mp.Plan(wl.phase_map, wl.phases, tol=wl.tol)
        for s, k in enumerate(gold["iters"]):
            plan.set_fixed_iterations(int(k))
            plan.solve(wl.times[s: s + 2], wl.E[s: s + 1], wl.G[s: s + 1])
        resp = plan.responses()[:, :40]
        got = sampled(plan.fields(), gold["idx"])
        plan.close()
    errs = {k: rel(got[k], gold[k]) for k in FIELDS}
    c = curve_rel(resp, gold["resp"])
    say("sampled field rel", {k: "%.1e" % v for k, v in errs.items()}, "curve rel %.1e" % c)
    assert it == gold["iters"].tolist()
    assert max(errs.values()) < 1e-10 and c < 1e-10


def test_spheres128_fixed_schedule_vs_oracle(mp):
    wl = W.random_spheres_128(n_steps=3)
    say("case: 128^3 cell, 3 steps x 3 iterations, every field vs the oracle")
    plan = mp.Plan(wl.phase_map, wl.phases, tol=wl.tol)
    plan.set_fixed_iterations(3)
    plan.solve(wl.times, wl.E, wl.G)
    got, resp = plan.fields(), plan.responses()[:, :40]
    plan.close()
    out = O.Solver(wl.phase_map, wl.phases, tol=wl.tol).solve(wl.times, wl.E, wl.G, schedule=[3, 3, 3],
                                                              fields_at=(3,))
    f = out["fields"][3]
    errs = {k: rel(got[k], f[k]) for k in FIELDS}
    c = curve_rel(resp, out["resp"])
    say("field rel", {k: "%.1e" % v for k, v in errs.items()}, "curve rel %.1e" % c)
    assert max(errs.values()) < 1e-10 and c < 1e-10


def test_spheres256_mixed_fixed_schedule_vs_oracle(mp):
    path = os.path.join(GOLDEN, "spheres256_step1.npz")
    if not os.path.exists(path):
        pytest.skip("expected values not written (make_spheres256_golden.py)")
    gold = np.load(path)
    wl = W.random_spheres_256(n_steps=1)
    say("case: 256^3 cell, mixed form, step 1 on 2 fixed iterations vs the oracle")
    plan = mp.Plan(wl.phase_map, wl.phases, tol=wl.tol, precision="mixed")
    plan.set_fixed_iterations(int(gold["iters"][0]))
    plan.solve(wl.times, wl.E, wl.G)
    got = sampled(plan.fields(), gold["idx"])
    resp = plan.responses()[:, :40]
    plan.close()
    errs = {k: rel(got[k], gold[k]) for k in FIELDS}
    scale = np.abs(gold["resp"]).max()
    c = np.abs(resp - gold["resp"]).max() / scale
    say("sampled field rel", {k: "%.1e" % v for k, v in errs.items()}, "averages %.1e of their scale" % c)
    assert max(errs.values()) < 1e-4 and c < 1e-4


def test_spheres256_fp64_fixed_schedule_vs_oracle(mp):
    path = os.path.join(GOLDEN, "spheres256_step1.npz")
    if not os.path.exists(path):
        pytest.skip("expected values not written (make_spheres256_golden.py)")
    gold = np.load(path)
    wl = W.random_spheres_256(n_steps=1)
    say("case: 256^3 cell, FP64, step 1 on 2 fixed iterations vs the oracle")
    plan = mp.Plan(wl.phase_map, wl.phases, tol=wl.tol)
    plan.set_fixed_iterations(int(gold["iters"][0]))
    plan.solve(wl.times, wl.E, wl.G)
    got = sampled(plan.fields(), gold["idx"])
    resp = plan.responses()[:, :40]
    plan.close()
    errs = {k: rel(got[k], gold[k]) for k in FIELDS}
    c = curve_rel(resp, gold["resp"])
    say("sampled field rel", {k: "%.1e" % v for k, v in errs.items()}, "curve rel %.1e" % c)
    assert max(errs.values()) < 1e-10 and c < 1e-10


def test_batch_rves_full_size_equal_solo(mp):
    rves = W.batch_rves(seed=3, count=64, n_steps=2)
    pick = []
    for n in (32, 64, 96, 128):
        pick.append(next(w for w in rves if w.phase_map.shape[0] == n))
    say("case: many-RVE workload at full size, one RVE of each edge in one batch vs solo plans, mixed,",
        [w.name for w in pick])
    shapes = [w.phase_map.shape[::-1] for w in pick]
    B = mp.Batch(shapes, arena_bytes=4 << 30, precision="mixed", max_rves=8, iters_per_launch=8, autotune=True)
    ids = [B.admit(w.phase_map, w.phases, w.times, w.E, w.G, tol=w.tol) for w in pick]
    launches = B.drain()
    say("graph launches", launches)
    for rid, w in zip(ids, pick):
        b = batched(B, rid)
        assert b["state"] == mp.MP_RVE_DONE and b["status"] == mp.MP_OK
        s = solo(mp, w, "mixed")
        say(f"  rve {w.name}: iterations {b['iters']}")
        assert_same(b, s, w.name)
    B.close()


def test_serving_with_256_request_equals_solo(mp):
    wls = [W.random_rve(seed=201, n=256, n_steps=1), W.random_rve(seed=202, n=32, n_steps=3),
           W.random_rve(seed=203, n=64, n_steps=2)]
    say("case: serving a 256^3 request beside 32^3 and 64^3 ones, mixed, replies vs solo plans")
    items = [(0.01 * i, w.phase_map, w.phases, w.times, w.E, w.G, dict(tol=w.tol)) for i, w in enumerate(wls)]
    shapes = sorted({w.phase_map.shape[::-1] for w in wls})
    B = mp.Batch(shapes, arena_bytes=12 << 30, precision="mixed", max_rves=8, iters_per_launch=8)
    reqs = mp.Requests(items, precision="mixed", fields=BFIELDS, device="cuda:0")
    ta, td, st, it = mp.serve_batched(B, reqs)
    B.close()
    say("done", np.round(td, 2), "iterations", it)
    assert (st == mp.MP_OK).all()
    for i, w in enumerate(wls):
        ref = solo(mp, w, "mixed")
        assert it[i] == sum(ref["iters"])
        assert_reply(reqs, i, ref, ("served", w.name))
