"""The stored Green operator (MP_GREEN_STORED: the inverse Fourier symbol of
the reference medium written once per frequency at plan creation, as the
paper precomputes its Green tensors, Sec. 2.4) on the HIP path, through the
C ABI, against the oracle's dense per-frequency inverse:

- the Green operator alone on grids with ragged and long axes, for
  isotropic reference media (with and without a skew couple modulus) and a
  tensor reference, FP64: within 1e-12;
- whole load paths (Alg. 2) on small grids, FP64: equal iteration counts,
  fields and response curves within 1e-10;
- the same in the mixed form, converged against the oracle, within the
  mixed form's bound of 1e-4;
- the 32^3 RVE of the many-RVE workload: stored and computed operators
  give the same iteration counts and fields within 1e-12 (they differ by
  rounding only);
- batches: RVEs with the stored operator beside RVEs with the computed one
  in the same shape classes (the class then solves per tile), FP64 and mixed,
  each equal bit for bit to its solo plan of the same kind, admitted before
  and after the first graph capture.
"""
import numpy as np
import pytest

from oracle import micropolar as O
from paper_2409_10774_amd import workloads as W
from tests.test_gpu_parity import GRIDS, REFS, compare_run, rel, say, small_workload
from tests.test_gpu_batch import assert_same, batched, mixed_set, solo
from tests.test_gpu_refmedium import GREEN_GRIDS, aniso_cell

pytestmark = pytest.mark.gpu

FIELDS = ("e", "g", "t", "m", "p", "q")


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


@pytest.fixture(scope="module")
def mp(torch):
    from paper_2409_10774_amd import mp as _mp
    return _mp


@pytest.mark.parametrize("ref", REFS)
@pytest.mark.parametrize("n,h", GRIDS)
def test_stored_green_apply_isotropic(torch, mp, n, h, ref):
    say(f"case: stored green apply n={n} h={h} ref={ref}")
    rng = np.random.default_rng(2)
    pm = np.zeros(n[::-1], np.uint8)
    plan = mp.Plan(pm, [W.Phase(*ref)], h=h, ref_mode="explicit", ref=ref, green="stored")
    f = rng.standard_normal((18,) + n[::-1])
    out = plan.green_apply(torch.from_numpy(f).to(plan.device)).cpu().numpy()
    plan.close()
    e, g = O.GreenOperator(n, h, ref).apply(f[:9], f[9:])
    errs = rel(out[:9], e), rel(out[9:], g)
    say("rel errors", errs)
    assert max(errs) < 1e-12


@pytest.mark.parametrize("n,h", GREEN_GRIDS)
def test_stored_green_apply_tensor_reference(torch, mp, n, h):
    say(f"case: stored green apply, tensor reference, n={n} h={h}")
    rng = np.random.default_rng(3)
    pm = (rng.random(n[::-1]) < 0.3).astype(np.uint8)
    mat = W.matrix_phase(kappa=0.5, tY=np.inf, mY=np.inf)
    inc = W.anisotropic_phase(7, t_scale=3.0, m_scale=2.0)
    plan = mp.Plan(pm, [mat, inc], h=h, ref_mode="tensor_mean", green="stored")
    f = rng.standard_normal((18,) + n[::-1])
    out = plan.green_apply(torch.from_numpy(f).to(plan.device)).cpu().numpy()
    plan.close()
    e, g = O.GreenOperator(n, h, O.reference_tensors(pm, [mat, inc])).apply(f[:9], f[9:])
    errs = rel(out[:9], e), rel(out[9:], g)
    say("rel errors", errs)
    assert max(errs) < 1e-12


@pytest.mark.parametrize("n", [(8, 8, 8), (12, 6, 8), (24, 16, 12), (6, 48, 4)])
def test_stored_full_path_vs_oracle(torch, mp, n):
    say(f"case: Alg. 2 with the stored Green operator, n={n}")
    wl = small_workload(n, seed=sum(n))
    plan = mp.Plan(wl.phase_map, wl.phases, tol=wl.tol, green="stored")
    compare_run(mp, plan, wl, len(wl.E))
    plan.close()


def test_stored_tensor_reference_full_path_vs_oracle(torch, mp):
    say("case: Eq. 5 inclusion, tensor phase-mean reference, stored Green operator, 12x6x8, FP64")
    w = aniso_cell()
    plan = mp.Plan(w.phase_map, w.phases, tol=w.tol, ref_mode="tensor_phase_mean", green="stored")
    it = plan.solve(w.times, w.E, w.G)
    got = {k: plan.field(k) for k in FIELDS}
    plan.close()
    out = O.Solver(w.phase_map, w.phases, tol=w.tol, ref_mode="tensor_phase_mean").solve(
        w.times, w.E, w.G, fields_at=(len(w.E),))
    f = out["fields"][len(w.E)]
    errs = {k: rel(got[k], f[k]) for k in FIELDS}
    say("iterations", it, "oracle", out["iters"], "field rel", {k: "%.1e" % v for k, v in errs.items()})
    assert it == out["iters"]
    assert max(errs.values()) < 1e-10


@pytest.mark.parametrize("n", [(16, 16, 16), (24, 12, 32)])
def test_stored_mixed_vs_oracle(torch, mp, n):
    say(f"case: mixed form with the stored Green operator vs the oracle, n={n}")
    wl = small_workload(n, seed=sum(n), contrast=10.0, steps=3, G_end=0.0)
    wl.tol = 1e-6
    plan = mp.Plan(wl.phase_map, wl.phases, tol=wl.tol, precision="mixed", green="stored")
    it = plan.solve(wl.times, wl.E, wl.G)
    recs = plan.responses()
    got = {k: plan.field(k) for k in FIELDS}
    plan.close()
    assert (recs[:, 40] <= wl.tol).all()
    ref = O.Solver(wl.phase_map, wl.phases, tol=wl.tol).solve(wl.times, wl.E, wl.G, fields_at=(len(wl.E),))
    f = ref["fields"][len(wl.E)]
    errs = {k: rel(got[k], f[k]) for k in FIELDS}
    say("iterations", it, "oracle", ref["iters"], "field rel", {k: "%.1e" % v for k, v in errs.items()})
    assert max(errs.values()) < 1e-4
    assert all(abs(a - b) <= 2 + 0.1 * b for a, b in zip(it, ref["iters"]))


def test_stored_equals_computed_rve32(torch, mp):
    wl = W.batch_rves(seed=3, count=64, n_steps=3)
    wl = next(w for w in wl if w.phase_map.shape[0] == 32)
    say(f"case: {wl.name}, stored vs computed Green operator, 3 steps, FP64")
    res = {}
    for green in ("computed", "stored"):
        plan = mp.Plan(wl.phase_map, wl.phases, tol=wl.tol, green=green)
        it = plan.solve(wl.times, wl.E, wl.G)
        res[green] = (it, {k: plan.field(k) for k in FIELDS})
        plan.close()
    (ia, fa), (ib, fb) = res["computed"], res["stored"]
    errs = {k: rel(fb[k], fa[k]) for k in FIELDS}
    say("iterations", ia, ib, "rel", {k: "%.1e" % v for k, v in errs.items()})
    assert ia == ib
    assert max(errs.values()) < 1e-12


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-8), ("mixed", 1e-6)])
def test_batch_stored_and_computed_equal_solo(mp, precision, tol):
    say(f"case: batch of stored and computed Green operators in 3 shape classes vs solo plans, {precision}")
    wls = mixed_set(tol)
    shapes = [(16, 16, 16), (12, 6, 8), (24, 16, 12)]
    B = mp.Batch(shapes, arena_bytes=256 << 20, precision=precision, max_rves=16, iters_per_launch=8,
                 autotune=True)
    greens = ["stored" if i % 2 == 0 else "computed" for i in range(len(wls))]
    # half admitted, one launch (graph captured), then the rest: a class takes
    # its first stored RVE after the capture
    ids = []
    for w, gm in zip(wls[:3], greens[:3]):
        ids.append(B.admit(w.phase_map, w.phases, w.times, w.E, w.G, tol=w.tol, green=gm))
    B.run()
    for w, gm in zip(wls[3:], greens[3:]):
        ids.append(B.admit(w.phase_map, w.phases, w.times, w.E, w.G, tol=w.tol, green=gm))
    launches = B.drain()
    say("graph launches", launches)
    for rid, w, gm in zip(ids, wls, greens):
        b = batched(B, rid)
        assert b["state"] == mp.MP_RVE_DONE
        s = solo(mp, w, precision, green=gm)
        say(f"  rve {rid} {gm} n={w.phase_map.shape} iters {b['iters']} solo {s['iters']}")
        assert_same(b, s, rid)
    B.close()
