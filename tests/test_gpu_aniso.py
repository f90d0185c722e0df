"""Phases with the general centrosymmetric elastic tensors of Eq. 5 on the
HIP path (the x pass's Eq. 5 variant), against the oracle:
  - a homogeneous anisotropic cell: t = A:E, m = B:Gamma (index sums
    written out), uniform;
  - an anisotropic inclusion in a plastic matrix on a ragged grid, FP64: equal
    iteration counts, fields and response curves within 1e-10;
  - the same cell in mixed precision on a fixed schedule, against the FP64
    path on that schedule;
  - a resident batch holding Eq. 5 and isotropic RVEs, with isotropic and
    tensor reference media in one shape class, admitted after the first
    graph capture: every RVE equals its solo plan bit for bit (FP64 and
    mixed);
  - the continuous-batching server with Eq. 5 and tensor-reference requests
    arriving mid-run: every request served with the solo iteration counts.
"""
import numpy as np
import pytest

from oracle import micropolar as O
from paper_2409_10774_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def mp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_10774_amd import mp as _mp
    return _mp


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    r = np.abs(b).max()
    return np.abs(a - b).max() / r if r > 0 else np.abs(a - b).max()


def cell(n=(12, 6, 8), steps=3):
    ph, _ = W.random_spheres(max(n), 11, 3, 1.5, 3.0)
    ph = ph[: n[2], : n[1], : n[0]].copy()
    mat = W.matrix_phase(kappa=0.5, length=1.0, tY=0.004)
    mat.beta = 0.8 * mat.gamma
    inc = W.anisotropic_phase(5, t_scale=3.0, m_scale=4.0)
    times, E, G = W.ramp_path(steps, E_end=W.unit((0, 0), 0.01) + W.unit((1, 2), 0.004),
                              G_end=W.unit((0, 1), 0.002), t_end=float(steps))
    return W.Workload("aniso", ph, [mat, inc], times, E, G, tol=1e-8)


def test_homogeneous_anisotropic_cell(mp):
    say("case: homogeneous Eq. 5 cell, 8^3, 2 steps")
    ph = W.anisotropic_phase(4)
    pm = np.zeros((8, 8, 8), np.uint8)
    Ev = np.array([0.3, 0.1, -0.2, 0.05, -0.4, 0.2, 0.1, 0.0, 0.25]) * 1e-2
    Gv = np.array([0.0, 0.2, 0.1, -0.1, 0.05, 0.0, 0.3, -0.2, 0.1]) * 1e-2
    times = np.array([0.0, 1.0, 2.0])
    plan = mp.Plan(pm, [ph], tol=1e-12)
    it = plan.solve(times, times[1:, None] * Ev, times[1:, None] * Gv)
    assert max(it) <= 2, it
    E, G = (2 * Ev).reshape(3, 3), (2 * Gv).reshape(3, 3)
    t_ref = np.einsum("klmn,mn->kl", ph.A, E).reshape(9)
    m_ref = np.einsum("lkmn,mn->kl", ph.B, G).reshape(9)
    t = plan.field("t").reshape(9, -1)
    m = plan.field("m").reshape(9, -1)
    assert np.abs(t - t_ref[:, None]).max() < 1e-14 * np.abs(t_ref).max()
    assert np.abs(m - m_ref[:, None]).max() < 1e-14 * np.abs(m_ref).max()


def test_anisotropic_inclusion_fp64_vs_oracle(mp):
    say("case: Eq. 5 inclusion in a plastic matrix, 12x6x8, 3 steps, FP64")
    w = cell()
    plan = mp.Plan(w.phase_map, w.phases, tol=w.tol)
    it = plan.solve(w.times, w.E, w.G)
    out = O.Solver(w.phase_map, w.phases, tol=w.tol).solve(w.times, w.E, w.G, fields_at=(3,))
    say("iterations gpu", it, "oracle", out["iters"])
    if it != out["iters"]:
        out = O.Solver(w.phase_map, w.phases, tol=w.tol).solve(w.times, w.E, w.G, schedule=it,
                                                               fields_at=(3,))
    f = out["fields"][3]
    assert f["p"].max() > 0
    errs = {k: rel(plan.field(k), f[k]) for k in ("e", "g", "t", "m", "p", "q")}
    say("field rel errors", errs)
    assert max(errs.values()) < TOL
    resp = plan.responses()[:, :40]
    scale = np.abs(out["resp"]).max(axis=0)
    big = scale > 1e-12 * scale.max()
    curve = (np.abs(resp - out["resp"])[:, big].max(axis=0) / scale[big]).max()
    say(f"curves max rel {curve:.2e}")
    assert curve < TOL


def test_anisotropic_inclusion_mixed_vs_fp64(mp):
    say("case: Eq. 5 inclusion, mixed vs FP64 on a fixed schedule of 40 iterations per step")
    w = cell()
    f = {}
    for prec in ("fp64", "mixed"):
        plan = mp.Plan(w.phase_map, w.phases, tol=w.tol, precision=prec)
        plan.set_fixed_iterations(40)
        plan.solve(w.times, w.E, w.G)
        f[prec] = {k: plan.field(k) for k in ("e", "g", "t", "m")}
    errs = {k: rel(f["mixed"][k], f["fp64"][k]) for k in f["fp64"]}
    say("mixed vs fp64 field rel", errs)
    assert max(errs.values()) < 1e-5


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_with_anisotropic_phases_equals_solo(mp, precision):
    say(f"case: batch of Eq. 5 and isotropic RVEs vs solo plans, {precision}")
    from tests.test_gpu_batch import assert_same, batched, solo
    from tests.test_gpu_parity import small_workload
    a1 = cell()
    a2 = cell(steps=2)
    a2.phases = [a2.phases[0], W.anisotropic_phase(9, t_scale=2.5, m_scale=3.0)]
    a2.ref_mode = "tensor_phase_mean"
    iso = small_workload((16, 16, 16), seed=40, contrast=3.0, steps=3, G_end=0.002)
    iso2 = small_workload((16, 16, 16), seed=45, contrast=4.0, steps=2, G_end=0.0)
    iso2.ref_mode = "tensor_phase_mean"
    wls = [a1, iso, a2, iso2]
    for w in wls:
        w.tol = 1e-8 if precision == "fp64" else 1e-6
    B = mp.Batch([(12, 6, 8), (16, 16, 16)], arena_bytes=128 << 20, precision=precision, max_rves=8,
                 iters_per_launch=8, autotune=False)
    # the isotropic RVE runs first (graph captured with the plain x passes);
    # admitting the Eq. 5 RVEs switches their class to the Eq. 5 variant
    ids = [None, B.admit(iso.phase_map, iso.phases, iso.times, iso.E, iso.G, tol=iso.tol), None, None]
    for _ in range(3):
        B.run()
    for k in (0, 2, 3):
        w = wls[k]
        ids[k] = B.admit(w.phase_map, w.phases, w.times, w.E, w.G, tol=w.tol, ref_mode=w.ref_mode)
    B.drain()
    for rid, w in zip(ids, wls):
        b = batched(B, rid)
        assert b["state"] == mp.MP_RVE_DONE
        s = solo(mp, w, precision, ref_mode=w.ref_mode)
        say(f"  rve {rid} n={w.phase_map.shape} iters {b['iters']} solo {s['iters']}")
        assert_same(b, s, rid)
    B.close()


def test_serving_with_anisotropic_requests(mp):
    say("case: serving loop with Eq. 5 and tensor-reference requests arriving mid-run")
    import numpy as np
    from tests.test_gpu_batch import solo
    from tests.test_gpu_parity import small_workload
    iso = small_workload((16, 16, 16), seed=40, contrast=3.0, steps=3, G_end=0.002)
    a1 = cell()
    a2 = cell(steps=2)
    a2.phases = [a2.phases[0], W.anisotropic_phase(9, t_scale=2.5, m_scale=3.0)]
    kw = [dict(), dict(), dict(ref_mode="tensor_phase_mean")]
    wls = [iso, a1, a2]
    for w in wls:
        w.tol = 1e-6
    arrivals = np.array([0.0, 0.01, 0.02])
    items = [(t, w.phase_map, w.phases, w.times, w.E, w.G, dict(tol=w.tol, **k))
             for t, w, k in zip(arrivals, wls, kw)]
    B = mp.Batch([(12, 6, 8), (16, 16, 16)], arena_bytes=128 << 20, precision="mixed", max_rves=8,
                 iters_per_launch=8)
    from tests.test_gpu_batch import FIELDS, assert_reply
    reqs = mp.Requests(items, precision="mixed", fields=FIELDS)
    ta, td, st, it = mp.serve_batched(B, reqs)
    say("admit", np.round(ta, 3), "done", np.round(td, 3), "iters", it)
    assert (st == mp.MP_OK).all()
    for i, (w, k) in enumerate(zip(wls, kw)):
        ref = solo(mp, w, "mixed", **k)
        assert it[i] == sum(ref["iters"]), i
        assert_reply(reqs, i, ref, i)
    B.close()
