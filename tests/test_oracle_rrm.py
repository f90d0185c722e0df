"""Pins of the oracle's radial-return mapping (Alg. 1, Eqs. 30, 32).

- elastic branch returns the trial stresses of Eq. 8 (independent sym/skew law);
- plastic branch lands on both yield surfaces (Eqs. 13-18, evaluated by the
  independent tangent module), keeps the trace and the sym/skew directions,
  and never decreases p, q;
- proportional straining from the zero state: any number of Alg. 1 steps equals
  an RK4 integration of the App. C continuum-tangent rate equations;
- homogeneous uniaxial strain: closed-form bilinear response.
"""
import numpy as np
import pytest

from oracle import micropolar as O
from oracle import tangent as T
from paper_2409_10774_amd import workloads as W
from tests import helpers as H

PHASES = [
    W.Phase(lam=1.0, mu=1.0, kappa=0.5, alpha=0.0, beta=0.5, gamma=1.0,
            tY=0.01, tH=0.3, mY=0.02, mH=0.2, a1=1.5, b1=1.5),
    W.Phase(lam=1.5, mu=1.5, kappa=0.75, alpha=0.0, beta=0.25, gamma=1.5,
            tY=0.015, tH=0.0, mY=0.01, mH=0.0, a1=1.2, b1=2.0),
    W.matrix_phase(),                      # beta = gamma
    W.matrix_phase().scaled_moduli(5.0),   # elastic inclusion
]


def t33(a):
    return O.to_t33(a)


def state(nvox, seed, scale):
    d = W.random_state(nvox, seed, scale)
    return {k: (t33(v) if v.ndim == 2 else v) for k, v in d.items()}


def run(st, pm):
    return O.radial_return(st["e"], st["g"], st["e_n"], st["g_n"], st["t_n"], st["m_n"],
                           st["p_n"], st["q_n"], pm, PHASES)


def trial(st, pm):
    tab = O.phase_table(PHASES)[pm]
    de = np.moveaxis(st["e"] - st["e_n"], 0, -1)          # (3, 3, V) after moves
    de = np.moveaxis(st["e"] - st["e_n"], (-2, -1), (0, 1))
    dg = np.moveaxis(st["g"] - st["g_n"], (-2, -1), (0, 1))
    tt = H.law_t(tab[:, 0], tab[:, 1], tab[:, 2], de)
    mt = H.law_m(tab[:, 3], tab[:, 4], tab[:, 5], dg)
    return st["t_n"] + np.moveaxis(tt, (0, 1), (-2, -1)), st["m_n"] + np.moveaxis(mt, (0, 1), (-2, -1))


def consts(pm):
    tab = O.phase_table(PHASES)[pm]
    return {k: tab[:, i] for i, k in enumerate(O.PHASE_KEYS)}


def test_elastic_branch_is_trial():
    V = 400
    pm = np.arange(V) % len(PHASES)
    st = state(V, 1, 1e-5)
    st["t_n"] *= 0.01
    st["m_n"] *= 0.01
    t, m, p, q = run(st, pm)
    tt, mt = trial(st, pm)
    c = consts(pm)
    assert (T.f_yield(c, tt, st["p_n"])[0] < 0).all() and (T.g_yield(c, mt, st["q_n"])[0] < 0).all()
    assert np.abs(t - tt).max() <= 1e-15 * np.abs(tt).max()
    assert np.abs(m - mt).max() <= 1e-15 * np.abs(mt).max()
    assert np.array_equal(p, st["p_n"]) and np.array_equal(q, st["q_n"])


def test_plastic_branch_invariants():
    V = 2000
    pm = np.arange(V) % 3          # plastic phases only
    st = state(V, 2, 5e-2)
    t, m, p, q = run(st, pm)
    tt, mt = trial(st, pm)
    c = consts(pm)
    f_tr, _ = T.f_yield(c, tt, st["p_n"])
    g_tr, _ = T.g_yield(c, mt, st["q_n"])
    f, _ = T.f_yield(c, t, p)
    g, _ = T.g_yield(c, m, q)
    pl_t, pl_m = f_tr >= 0, g_tr >= 0
    assert pl_t.sum() > V // 2 and pl_m.sum() > V // 2
    R1 = c["tY"] + c["tH"] * p
    R2 = c["mY"] + c["mH"] * q
    assert np.abs(f[pl_t]).max() < 1e-13 * R1[pl_t].max()
    assert np.abs(g[pl_m]).max() < 1e-13 * R2[pl_m].max()
    assert (p >= st["p_n"]).all() and (q >= st["q_n"]).all()
    assert np.abs(np.trace(t, axis1=1, axis2=2) - np.trace(tt, axis1=1, axis2=2)).max() < 1e-15
    # direction kept: the sym and skew deviatoric parts are positive multiples of the trial ones
    for X, Y, sel in ((O.dev(t), O.dev(tt), pl_t), (m, mt, pl_m)):
        for part in (O.sym, O.skw):
            a, b = part(X)[sel], part(Y)[sel]
            cross = np.einsum("vkl,vkl->v", a, b)
            na, nb = np.linalg.norm(a, axis=(1, 2)), np.linalg.norm(b, axis=(1, 2))
            ok = nb > 1e-14
            assert np.all(cross[ok] >= 0)
            assert np.abs(cross[ok] - na[ok] * nb[ok]).max() < 1e-12 * (na * nb).max()


@pytest.mark.parametrize("nsteps", [1, 3, 17])
def test_proportional_path_equals_tangent_integration(nsteps):
    """Radial return is exact for proportional straining: Alg. 1 applied over
    any step sizes equals the RK4 integration of the continuum tangent."""
    V = 60
    pm = np.arange(V) % len(PHASES)
    rng = np.random.default_rng(3 + nsteps)
    D = 0.02 * rng.standard_normal((V, 3, 3))
    Dg = 0.02 * rng.standard_normal((V, 3, 3))
    z = np.zeros((V, 3, 3))
    zs = np.zeros(V)
    hist = dict(e=z, g=z, t=z, m=z, p=zs, q=zs)
    Tend = 1.0
    for s in range(1, nsteps + 1):
        tau = Tend * s / nsteps
        t, m, p, q = O.radial_return(tau * D, tau * Dg, hist["e"], hist["g"], hist["t"], hist["m"],
                                     hist["p"], hist["q"], pm, PHASES)
        hist = dict(e=tau * D, g=tau * Dg, t=t, m=m, p=p, q=q)
    c = consts(pm)
    ti, mi, pi_, qi = T.integrate(c, (z, z, zs, zs), D, Dg, Tend, substeps=400)
    assert np.abs(hist["t"] - ti).max() < 1e-10 * np.abs(ti).max()
    assert np.abs(hist["m"] - mi).max() < 1e-10 * np.abs(mi).max()
    assert np.abs(hist["p"] - pi_).max() < 1e-10 * max(pi_.max(), 1e-30)
    assert np.abs(hist["q"] - qi).max() < 1e-10 * max(qi.max(), 1e-30)
    assert pi_.max() > 0 and qi.max() > 0   # the path really is plastic


def test_uniaxial_closed_form():
    """Homogeneous uniaxial strain E11 in the isotropic matrix: bilinear closed form."""
    ph = W.matrix_phase()
    lam, mu, tY, tH, a1 = ph.lam, ph.mu, ph.tY, ph.tH, ph.a1
    Es = np.linspace(0.0005, 0.01, 20)
    z = np.zeros((1, 3, 3))
    hist = dict(e=z, g=z, t=z, m=z, p=np.zeros(1), q=np.zeros(1))
    for E in Es:
        e = np.zeros((1, 3, 3))
        e[0, 0, 0] = E
        t, m, p, q = O.radial_return(e, z, hist["e"], hist["g"], hist["t"], hist["m"],
                                     hist["p"], hist["q"], np.zeros(1, int), [ph])
        hist = dict(e=e, g=z, t=t, m=m, p=p, q=q)
        k = np.sqrt(a1 * 2.0 / 3.0) * 2 * mu          # t_eq of the elastic trial = k E
        if k * E < tY:
            t11, t22, pp = (lam + 2 * mu) * E, lam * E, 0.0
        else:
            pp = (k * E - tY) / (tH + 2 * a1 * mu)
            R = tY + tH * pp
            t11 = (3 * lam + 2 * mu) * E / 3 + R / (k * E) * 4 * mu * E / 3
            t22 = (3 * lam + 2 * mu) * E / 3 - R / (k * E) * 2 * mu * E / 3
        assert abs(t[0, 0, 0] - t11) < 1e-15 * 10
        assert abs(t[0, 1, 1] - t22) < 1e-15 * 10
        assert abs(t[0, 2, 2] - t22) < 1e-15 * 10
        assert abs(p[0] - pp) < 1e-15
