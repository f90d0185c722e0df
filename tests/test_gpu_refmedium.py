"""General reference medium (A0 = <A(x)>, B0 = <B(x)> as tensors, Alg. 2
with every phase's own law) on the HIP path, against the oracle:
  - the Green operator alone (z pass with the factored 6x6 Fourier symbol)
    for an anisotropic reference, on grids with ragged and long axes, FP64;
  - isotropic phases with beta = gamma: the tensor-mean paths (general
    symbol, row-matrix polarization) against the closed-form isotropic paths
    of the same means on one fixed schedule (the reference media are equal);
  - an Eq. 5 inclusion in a plastic matrix with the unweighted tensor mean
    (the volume mean diverges there: a stiff phase in a small volume), FP64,
    to convergence: iteration counts and fields against the oracle, and
    fewer iterations than with the isotropic phase-mean reference;
  - the same cell in mixed precision on a fixed schedule against FP64;
  - the 128^3 cell of Eq. 5 spheres (the benchmark's anisotropic workload)
    at full size on a fixed schedule, against the oracle;
  - the paper's manufactured solution (App. D.1) with a tensor reference.
"""
import numpy as np
import pytest

from oracle import micropolar as O
from paper_2409_10774_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-10


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


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    r = np.abs(b).max()
    return np.abs(a - b).max() / r if r > 0 else np.abs(a - b).max()


def aniso_cell(n=(12, 6, 8), steps=3):
    ph, _ = W.random_spheres(max(n), 11, 3, 1.5, 3.0)
    ph = ph[: n[2], : n[1], : n[0]].copy()
    mat = W.matrix_phase(kappa=0.5, length=1.0, tY=0.004)
    mat.beta = 0.8 * mat.gamma
    inc = W.anisotropic_phase(5, t_scale=3.0, m_scale=4.0)
    times, E, G = W.ramp_path(steps, E_end=W.unit((0, 0), 0.01) + W.unit((1, 2), 0.004),
                              G_end=W.unit((0, 1), 0.002), t_end=float(steps))
    return W.Workload("aniso", ph, [mat, inc], times, E, G, tol=1e-8)


GREEN_GRIDS = [((4, 4, 4), 1.0), ((8, 6, 12), 0.5), ((16, 32, 24), 1.0), ((6, 192, 4), 1.0),
               ((64, 64, 64), 1.0), ((16, 8, 128), 1.0), ((8, 4, 256), 0.5)]


@pytest.mark.parametrize("n,h", GREEN_GRIDS)
def test_green_apply_general_reference(torch, mp, n, h):
    say(f"case: general-reference green apply n={n} h={h}")
    rng = np.random.default_rng(3)
    pm = (rng.random(n[::-1]) < 0.3).astype(np.uint8)
    mat = W.matrix_phase(kappa=0.5, tY=np.inf, mY=np.inf)
    inc = W.anisotropic_phase(7, t_scale=3.0, m_scale=2.0)
    plan = mp.Plan(pm, [mat, inc], h=h, ref_mode="tensor_mean")
    f = rng.standard_normal((18,) + n[::-1])
    out = plan.green_apply(torch.from_numpy(f).to(plan.device)).cpu().numpy()
    G = O.GreenOperator(n, h, O.reference_tensors(pm, [mat, inc]))
    e, g = G.apply(f[:9], f[9:])
    errs = rel(out[:9], e), rel(out[9:], g)
    say("rel errors", errs)
    assert max(errs) < 1e-12


@pytest.mark.parametrize("iso,tensor,contrast", [("phase_mean", "tensor_phase_mean", 5.0),
                                                 ("volume_mean", "tensor_mean", 2.0)])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-4)])
def test_tensor_mean_of_isotropic_phases_matches_closed_form(mp, iso, tensor, contrast, precision, tol):
    say(f"case: sphere 16^3 (beta = gamma, contrast {contrast}), {tensor} vs {iso}, {precision}, "
        "3 x 25 iterations")
    wl = W.single_sphere_16(contrast)
    assert all(p.beta == p.gamma for p in wl.phases)
    f = {}
    for mode in (iso, tensor):
        plan = mp.Plan(wl.phase_map, wl.phases, tol=wl.tol, ref_mode=mode, precision=precision)
        plan.set_fixed_iterations(25)
        plan.solve(wl.times[:4], wl.E[:3], wl.G[:3])
        f[mode] = {k: plan.field(k) for k in ("e", "g", "t", "m", "p", "q")}
    assert 0 < f[iso]["p"].max() < 1
    errs = {k: rel(f[tensor][k], f[iso][k]) for k in f[iso]}
    say("tensor vs closed-form rel", errs)
    assert max(errs.values()) < tol


def test_anisotropic_reference_fp64_vs_oracle(mp):
    say("case: Eq. 5 inclusion, tensor phase-mean reference, 12x6x8, 3 steps, FP64")
    w = aniso_cell()
    plan = mp.Plan(w.phase_map, w.phases, tol=w.tol, ref_mode="tensor_phase_mean")
    it = plan.solve(w.times, w.E, w.G)
    solver = lambda: O.Solver(w.phase_map, w.phases, tol=w.tol, ref_mode="tensor_phase_mean")
    out = solver().solve(w.times, w.E, w.G, fields_at=(3,))
    say("iterations gpu", it, "oracle", out["iters"])
    if it != out["iters"]:
        out = solver().solve(w.times, w.E, w.G, schedule=it, fields_at=(3,))
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
    iso = mp.Plan(w.phase_map, w.phases, tol=w.tol)
    it_iso = iso.solve(w.times, w.E, w.G)
    say("iterations with the isotropic reference", it_iso)
    assert sum(it) < sum(it_iso)


def test_anisotropic_reference_mixed_vs_fp64(mp):
    say("case: Eq. 5 inclusion, tensor phase-mean reference, mixed vs FP64, 40 iterations per step")
    w = aniso_cell()
    f = {}
    for prec in ("fp64", "mixed"):
        plan = mp.Plan(w.phase_map, w.phases, tol=w.tol, precision=prec, ref_mode="tensor_phase_mean")
        plan.set_fixed_iterations(40)
        plan.solve(w.times, w.E, w.G)
        f[prec] = {k: plan.field(k) for k in ("e", "g", "t", "m")}
    errs = {k: rel(f["mixed"][k], f["fp64"][k]) for k in f["fp64"]}
    say("mixed vs fp64 field rel", errs)
    assert max(errs.values()) < 1e-5


def test_aniso128_full_size_fixed_schedule(mp):
    say("case: 128^3 Eq. 5 spheres, tensor phase-mean reference, step 1, fixed 2 iterations, FP64")
    wl = W.anisotropic_spheres_128(n_steps=1)
    plan = mp.Plan(wl.phase_map, wl.phases, tol=wl.tol, ref_mode=wl.ref_mode)
    plan.set_fixed_iterations(2)
    plan.solve(wl.times, wl.E, wl.G)
    out = O.Solver(wl.phase_map, wl.phases, tol=wl.tol, ref_mode=wl.ref_mode).solve(
        wl.times, wl.E, wl.G, schedule=[2], fields_at=(1,))
    f = out["fields"][1]
    errs = {k: rel(plan.field(k), f[k]) for k in ("e", "g", "t", "m", "p", "q")}
    say("field rel errors", errs)
    assert max(errs.values()) < TOL


def test_manufactured_solution_with_tensor_reference(mp):
    """The paper's code verification (App. D.1) with a tensor reference
    medium: the manufactured fields do not depend on the reference, so the
    general Green step and the row-matrix polarization must reproduce them
    within the same bound, and the oracle's fields (same reference) within
    1e-10."""
    from tests.mnms_case import case
    say("case: App. D.1 manufactured solution, 4^3, 25 steps, tensor phase-mean reference")
    n_steps = 25
    c = case(n_steps)
    times, Em, Gm, tm, mm = c["times"], c["Em"], c["Gm"], c["tm"], c["mm"]
    E = times[1:, None] * Em.reshape(1, 9)
    G = times[1:, None] * Gm.reshape(1, 9)
    check = (n_steps // 2, n_steps)
    plan = mp.Plan(c["pm"], c["phases"], h=c["h"], tol=c["eps"], ref_mode="tensor_phase_mean")
    it_gpu, got = [], {}
    for s in range(1, n_steps + 1):
        plan.set_eigenstress(np.concatenate([O.to_f9(tm[s - 1]), O.to_f9(mm[s - 1])]))
        it_gpu += plan.solve(times[s - 1: s + 1], E[s - 1: s], G[s - 1: s])
        if s in check:
            got[s] = {k: plan.field(k) for k in ("e", "g", "t", "m")}
    eig = lambda s: (tm[s - 1], mm[s - 1])
    solver = lambda: O.Solver(c["pm"], c["phases"], h=c["h"], tol=c["eps"], ref_mode="tensor_phase_mean")
    out = solver().solve(times, E, G, eig=eig, fields_at=check)
    say("iterations gpu", it_gpu, "oracle", out["iters"])
    if it_gpu != out["iters"]:
        out = solver().solve(times, E, G, schedule=it_gpu, eig=eig, fields_at=check)
    for s in check:
        tt = times[s]
        man = {"e": O.to_f9(tt * c["De"]), "g": O.to_f9(tt * c["Dg"]),
               "t": O.to_f9(tm[s - 1]), "m": O.to_f9(mm[s - 1])}
        for k, ref in man.items():
            err_man = np.abs(got[s][k] - ref).max()
            err_orc = rel(got[s][k], out["fields"][s][k])
            say(f"step {s} {k}: |gpu - manufactured| {err_man:.2e}, rel vs oracle {err_orc:.2e}")
            assert err_man < c["bound"], (s, k, err_man)
            assert err_orc < TOL, (s, k, err_orc)
    plan.set_eigenstress(None)
