"""Pins of the oracle's anisotropic elastic phases (Eq. 5: general
centrosymmetric tensors A_klmn, B_lkmn with A_klmn = A_mnkl, B_lkmn = B_mnlk).

- homogeneous anisotropic cell: uniform fields, t_kl = A_klmn E_mn and
  m_kl = B_lkmn Gamma_mn exactly (index sums written out here);
- heterogeneous cell with an anisotropic inclusion in a plastic matrix:
  the converged fields satisfy Eq. 2 (independent spectral derivatives),
  have the prescribed means, and obey Eq. 5 voxel by voxel in the inclusion;
- the isotropic tensors of Eq. 6, built here by applying the Eq. 8 laws to
  unit strains, given as general tensors reproduce the isotropic phase.
"""
import numpy as np

from oracle import micropolar as O
from paper_2409_10774_amd import workloads as W
from tests import helpers as H


def law5_t(A, e):
    t = np.zeros((3, 3) + e.shape[2:])
    for k in range(3):
        for l in range(3):
            for m in range(3):
                for n in range(3):
                    t[k, l] += A[k, l, m, n] * e[m, n]
    return t


def law5_m(B, g):
    """m_kl = B_lkmn gamma_mn, B stored in index order (l, k, m, n)."""
    out = np.zeros((3, 3) + g.shape[2:])
    for k in range(3):
        for l in range(3):
            for m in range(3):
                for n in range(3):
                    out[k, l] += B[l, k, m, n] * g[m, n]
    return out


def test_generated_tensors_have_the_eq5_symmetries():
    ph = W.anisotropic_phase(3)
    A, B = ph.A.reshape(9, 9), ph.B.reshape(9, 9)
    assert np.allclose(A, A.T, rtol=0, atol=1e-14) and np.allclose(B, B.T, rtol=0, atol=1e-14)
    assert np.linalg.eigvalsh(A).min() > 0 and np.linalg.eigvalsh(B).min() > 0
    # no minor symmetry: the pointwise law must use the indices as written
    assert np.abs(ph.A - ph.A.transpose(1, 0, 2, 3)).max() > 0.1


def test_homogeneous_anisotropic_closed_form():
    ph = W.anisotropic_phase(4)
    pm = np.zeros((4, 4, 4), np.uint8)
    Ev = np.array([0.3, 0.1, -0.2, 0.05, -0.4, 0.2, 0.1, 0.0, 0.25]) * 1e-2
    Gv = np.array([0.0, 0.2, 0.1, -0.1, 0.05, 0.0, 0.3, -0.2, 0.1]) * 1e-2
    times = np.array([0.0, 1.0, 2.0])
    s = O.Solver(pm, [ph], tol=1e-12)
    out = s.solve(times, times[1:, None] * Ev, times[1:, None] * Gv, fields_at=(2,))
    assert max(out["iters"]) <= 2
    f = out["fields"][2]
    E = (2.0 * Ev).reshape(3, 3)
    G = (2.0 * Gv).reshape(3, 3)
    t_ref = law5_t(ph.A, E)
    m_ref = law5_m(ph.B, G)
    assert np.abs(f["t"].reshape(3, 3, -1) - t_ref[..., None]).max() < 1e-14 * np.abs(t_ref).max()
    assert np.abs(f["m"].reshape(3, 3, -1) - m_ref[..., None]).max() < 1e-14 * np.abs(m_ref).max()


def test_anisotropic_inclusion_equilibrium_and_law():
    n = (6, 6, 6)
    pm = W.centred_sphere(6, 0.2)
    mat = W.matrix_phase(tY=0.004)
    inc = W.anisotropic_phase(5, t_scale=3.0, m_scale=4.0)
    D = np.array([0.3, 0.1, -0.2, 0.05, -0.4, 0.2, 0.1, 0.0, 0.25]) * 2e-2
    Dg = np.array([0.0, 0.2, 0.1, -0.1, 0.05, 0.0, 0.3, -0.2, 0.1]) * 1e-2
    times = np.array([0.0, 1.0, 2.0])
    s = O.Solver(pm, [mat, inc], tol=1e-11)
    out = s.solve(times, times[1:, None] * D, times[1:, None] * Dg, fields_at=(2,))
    f = out["fields"][2]
    assert f["p"].max() > 0                       # the matrix yields
    t = f["t"].reshape(3, 3, *pm.shape)
    m = f["m"].reshape(3, 3, *pm.shape)
    e = f["e"].reshape(3, 3, *pm.shape)
    g = f["g"].reshape(3, 3, *pm.shape)
    ru, rp = H.balance(t - t.mean(axis=(2, 3, 4), keepdims=True), m, n, 1.0)
    ru, rp = H.band_limit(ru), H.band_limit(rp)
    assert np.abs(ru).max() < 1e-8 * np.abs(t).max()
    assert np.abs(rp).max() < 1e-8 * np.abs(t).max()
    assert np.allclose(f["e"].mean(axis=(1, 2, 3)), 2.0 * D, atol=1e-15, rtol=0)
    sel = pm == 1
    assert np.abs(law5_t(inc.A, e)[:, :, sel] - t[:, :, sel]).max() < 1e-13 * np.abs(t).max()
    assert np.abs(law5_m(inc.B, g)[:, :, sel] - m[:, :, sel]).max() < 1e-13 * np.abs(m).max()


def test_isotropic_tensors_reproduce_isotropic_phase():
    mat = W.matrix_phase(tY=0.004)
    mat.beta = 0.8 * mat.gamma
    inc = mat.scaled_moduli(3.0)
    A = np.zeros((3, 3, 3, 3))
    B = np.zeros((3, 3, 3, 3))
    for mm in range(3):
        for nn in range(3):
            u = np.zeros((3, 3))
            u[mm, nn] = 1.0
            A[:, :, mm, nn] = H.law_t(inc.lam, inc.mu, inc.kappa, u)
            B[:, :, mm, nn] = H.law_m(inc.alpha, inc.beta, inc.gamma, u).T   # index order (l, k)
    tens = W.Phase(**{k: getattr(inc, k) for k in W.PHASE_KEYS}, A=A, B=B)
    pm = W.centred_sphere(6, 0.2)
    times, E, G = W.ramp_path(2, E_end=W.unit((0, 1), 0.01) + W.unit((2, 2), -0.004),
                              G_end=W.unit((1, 0), 0.003))
    a = O.Solver(pm, [mat, inc], tol=1e-11).solve(times, E, G, fields_at=(2,))
    b = O.Solver(pm, [mat, tens], tol=1e-11).solve(times, E, G, fields_at=(2,))
    assert a["iters"] == b["iters"]
    for k in ("e", "g", "t", "m", "p", "q"):
        x, y = a["fields"][2][k], b["fields"][2][k]
        assert np.abs(x - y).max() <= 1e-13 * max(np.abs(x).max(), 1e-300), k
