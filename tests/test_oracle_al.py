"""Pins of the augmented-Lagrangian oracle (oracle/augmented.py), the
high-contrast scheme the paper's conclusion (Sec. 4) points to.

- local step: the d it returns satisfies sigma(d) + C0 d = r when sigma is
  evaluated by the oracle's Alg. 1 (radial_return), on elastic and plastic
  voxels of four phases (beta = gamma among them) and two penalties;
- homogeneous cell: one iteration per step and the closed-form uniaxial
  response, as the basic scheme;
- linear elastic heterogeneous 4^3 cell: the fixed point equals the dense
  direct solve of the balance equations (tests/test_oracle_dense.py);
- elastoplastic cell: the converged fields equal the basic scheme's;
- the volume-average reference medium of Alg. 2, with which the basic scheme
  diverges on the 16^3 sphere cell at contrast 5, converges;
- at contrast 20 it needs far fewer iterations than the basic scheme.
"""
import numpy as np
import pytest

from oracle import augmented as AL
from oracle import micropolar as O
from paper_2409_10774_amd import workloads as W
from tests import test_oracle_dense as D

PHASES = [
    W.Phase(lam=1.0, mu=1.0, kappa=0.5, alpha=0.0, beta=0.5, gamma=1.0,
            tY=0.01, tH=0.3, mY=0.02, mH=0.2, a1=1.5, b1=1.5),
    W.matrix_phase(),                      # beta = gamma
    W.matrix_phase().scaled_moduli(5.0),   # elastic inclusion, beta = gamma
    W.Phase(lam=1.5, mu=1.5, kappa=0.75, alpha=0.0, beta=0.25, gamma=1.5,
            tY=0.015, tH=0.0, mY=0.01, mH=0.0, a1=1.2, b1=2.0),
]


@pytest.mark.parametrize("ref", [(2.0, 1.7, 0.4, 0.1, 1.0, 3.0), (2.0, 1.7, 0.4, 0.0, 2.0, 2.0)])
def test_local_step_solves_its_equation(ref):
    rng = np.random.default_rng(0)
    V = 2000
    # a penalty with gamma0 = beta0 is positive definite on every stress-carrying
    # part only for phases with beta = gamma (phases 1, 2)
    pm = np.arange(V) % len(PHASES) if ref[4] != ref[5] else 1 + np.arange(V) % 2
    c = O.voxel_constants(pm, PHASES)
    tab = O.phase_table(PHASES)
    x = {k: rng.standard_normal((V, 3, 3)) * 1e-2 for k in ("e_n", "g_n", "t_n", "m_n", "rt", "rm", "ec", "gc")}
    p_n, q_n = rng.random(V) * 1e-2, rng.random(V) * 1e-2
    A = np.stack([O.stiffness_A(*tab[i, :3]) for i in pm])
    B = np.stack([O.stiffness_B(*tab[i, 3:6]) for i in pm])
    bt = x["t_n"] - O.apply_A(A, x["e_n"])
    bm = x["m_n"] - O.apply_B(B, x["g_n"])
    de, dg = AL.local_step(x["rt"], x["rm"], x["ec"], x["gc"], bt, bm, p_n, q_n, c, ref)
    t, m, p, q = O.radial_return(de, dg, x["e_n"], x["g_n"], x["t_n"], x["m_n"], p_n, q_n, pm, PHASES)
    assert (p > p_n).mean() > 0.4 and (q > q_n).mean() > 0.4 and (p == p_n).any()
    rt = t + O.apply_A(O.stiffness_A(*ref[:3]), de)
    rm = m + O.apply_B(O.stiffness_B(*ref[3:]), dg)
    scale = np.abs(x["rt"]).max()
    assert np.abs(rt - x["rt"]).max() < 1e-13 * scale
    # the skew curvature carries no stress when beta = gamma in the phase and
    # in the penalty: that part has no equation (and d takes the compatible one)
    inert = (tab[pm, 4] == tab[pm, 5]) & (ref[4] == ref[5])
    res = rm - x["rm"]
    res[inert] = O.sym(res[inert])
    assert np.abs(res).max() < 1e-13 * scale
    if inert.any():
        assert np.abs(O.skw(dg[inert]) - O.skw(x["gc"][inert])).max() < 1e-16


def test_semidefinite_penalty_rejected():
    # gamma0 = beta0 leaves the skew curvature without penalty: with a phase
    # whose skew couple modulus is not zero the local step can have no solution
    pm = np.zeros((4, 4, 4), np.uint8)
    with pytest.raises(ValueError):
        AL.ALSolver(pm, [PHASES[0]], ref=(2.0, 1.7, 0.4, 0.0, 2.0, 2.0))
    AL.ALSolver(pm, [PHASES[1]], ref=(2.0, 1.7, 0.4, 0.0, 2.0, 2.0))


def test_homogeneous_one_iteration_closed_form():
    ph = W.matrix_phase()
    pm = np.zeros((6, 6, 6), np.uint8)
    times, E, G = W.ramp_path(6, E_end=W.unit((0, 0), 0.008), t_end=6.0)
    ref = (2.0, 1.5, 0.3, 0.0, 5.0, 6.0)
    out = AL.ALSolver(pm, [ph], tol=1e-10, ref=ref, relax=1.7).solve(times, E, G)
    assert out["iters"] == [1] * 6
    k = np.sqrt(ph.a1 * 2.0 / 3.0) * 2 * ph.mu
    for st, Ev in enumerate(E[:, 0]):
        pp = max(k * Ev - ph.tY, 0.0) / (ph.tH + 2 * ph.a1 * ph.mu)
        fac = (ph.tY + ph.tH * pp) / (k * Ev) if pp > 0 else 1.0
        t11 = (3 * ph.lam + 2 * ph.mu) * Ev / 3 + fac * 4 * ph.mu * Ev / 3
        assert abs(out["resp"][st, 0] - t11) < 1e-15
        assert abs(out["resp"][st, 36] - pp) < 1e-16


def test_linear_elastic_fixed_point_equals_dense_solve():
    N = D.N
    rng = np.random.default_rng(12)
    pm = (rng.random((N, N, N)) < 0.35).astype(np.uint8)
    mat = W.matrix_phase(kappa=0.4, length=1.0, tY=np.inf)
    mat.beta = 0.6 * mat.gamma
    inc = mat.scaled_moduli(4.0)
    inc.beta = 0.3 * inc.gamma
    phases = [mat, inc]
    Ev = np.array([0.3, 0.1, -0.2, 0.05, -0.4, 0.2, 0.1, 0.0, 0.25]) * 1e-2
    Gv = np.array([0.0, 0.2, 0.1, -0.1, 0.05, 0.0, 0.3, -0.2, 0.1]) * 1e-2
    E, G = Ev.reshape(3, 3), Gv.reshape(3, 3)
    n = 6 * len(D.modes())
    r0 = D.residual(np.zeros(n, complex), E, G, pm, phases)
    M = np.empty((len(r0), n), complex)
    for j in range(n):
        z = np.zeros(n, complex)
        z[j] = 1.0
        M[:, j] = D.residual(z, E, G, pm, phases) - r0
    e, g, t, mc = D.fields(np.linalg.solve(M, -r0), E, G, pm, phases)
    out = AL.ALSolver(pm, phases, tol=1e-13, ref_mode="geometric_mean", relax=1.7).solve(
        np.array([0.0, 1.0]), Ev[None], Gv[None], fields_at=(1,))
    f = out["fields"][1]
    for name, ref in (("e", e.real), ("g", g.real), ("t", t.real), ("m", mc.real)):
        got = f[name].reshape((3, 3, N, N, N))
        assert np.abs(got - ref).max() < 1e-10 * np.abs(ref).max(), name


def test_elastoplastic_fixed_point_equals_basic_scheme():
    wl = W.single_sphere_16(20.0)
    pm = wl.phase_map[4:12, 4:12, 4:12].copy()
    E = wl.E * 3
    b = O.Solver(pm, wl.phases, tol=1e-11, max_iter=5000).solve(wl.times[:3], E[:2], wl.G[:2],
                                                                fields_at=(2,))
    a = AL.ALSolver(pm, wl.phases, tol=1e-11, ref_mode="geometric_mean", relax=1.7).solve(
        wl.times[:3], E[:2], wl.G[:2], fields_at=(2,))
    assert b["resp"][:, 36].max() > 0                  # the matrix has yielded
    for k in "egtmp":
        x, y = a["fields"][2][k], b["fields"][2][k]
        assert np.abs(x - y).max() < 1e-10 * np.abs(y).max(), k
    # and in about half the iterations at this contrast
    assert sum(a["iters"]) < 0.6 * sum(b["iters"]), (a["iters"], b["iters"])


def test_volume_mean_reference_converges_where_basic_diverges():
    wl = W.single_sphere_16(5.0)
    b = O.Solver(wl.phase_map, wl.phases, tol=1e-8, max_iter=150, ref_mode="volume_mean")
    ob = b.solve(wl.times[:2], wl.E[:1], wl.G[:1])
    assert not (ob["err"][0] < 1.0)                     # grown far above 1 (or non-finite)
    a = AL.ALSolver(wl.phase_map, wl.phases, tol=1e-8, max_iter=150, ref_mode="volume_mean")
    oa = a.solve(wl.times[:2], wl.E[:1], wl.G[:1])
    assert oa["err"][0] <= 1e-8 and oa["iters"][0] < 150
    ref = O.Solver(wl.phase_map, wl.phases, tol=1e-8).solve(wl.times[:2], wl.E[:1], wl.G[:1])
    assert abs(oa["resp"][0][0] - ref["resp"][0][0]) < 1e-7 * abs(ref["resp"][0][0])
