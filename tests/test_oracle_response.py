"""Pins of the oracle's homogenized response (Solver.response): the averages
<t>, <m>, <p>, <q>, <t_eq>, <m_eq> that each load step reports.

- homogeneous uniaxial strain E11 in the elastoplastic matrix: elastically
  t_eq = sqrt(2 a1 / 3) 2 mu E (the deviatoric part of uniaxial strain), and
  on the yield surface t_eq = R1 = tY + tH p (Eqs. 14, 15, Alg. 1);
- homogeneous curvature in a phase with beta != gamma: m = beta Gamma +
  gamma Gamma^T (Eq. 8 with alpha = 0), elastically
  m_eq^2 = b1 (beta + gamma)^2 |Gamma_sym|^2 + b1 (gamma + beta)(gamma - beta)
  |Gamma_skw|^2 (Eq. 17 with b2 = b1 (gamma + beta) / (gamma - beta)), and on
  the yield surface m_eq = R2 = mY + mH q (Eq. 18);
- a hand-made two-voxel state whose equivalent stresses are worked out by
  hand, one phase with beta == gamma (the skew term drops, R7).
A t_eq taken on t instead of dev(t), or an m_eq that mishandles beta == gamma,
fails one of these.
"""
import numpy as np

from oracle import micropolar as O
from paper_2409_10774_amd import workloads as W

T_EQ, M_EQ, P_AVG, Q_AVG = 38, 39, 36, 37


def test_uniaxial_t_eq_elastic_and_on_yield_surface():
    ph = W.matrix_phase()          # lam = mu = 1, tY = 0.005, tH = 0.1, a1 = 1.5
    pm = np.zeros((4, 4, 4), np.uint8)
    times, E, G = W.ramp_path(6, E_end=W.unit((0, 0), 0.006), t_end=6.0)
    out = O.Solver(pm, [ph], tol=1e-12).solve(times, E, G)
    k = np.sqrt(2.0 * ph.a1 / 3.0) * 2.0 * ph.mu
    Ey = ph.tY / k                 # 0.0025: steps 1, 2 elastic, 3.. plastic
    seen = set()
    for s, Ev in enumerate(E[:, 0]):
        r = out["resp"][s]
        if Ev < Ey:
            seen.add("elastic")
            assert abs(r[T_EQ] - k * Ev) < 1e-15
            assert r[P_AVG] == 0.0
        else:
            seen.add("plastic")
            p = (k * Ev - ph.tY) / (ph.tH + 2.0 * ph.a1 * ph.mu)
            assert abs(r[P_AVG] - p) < 1e-16
            assert abs(r[T_EQ] - (ph.tY + ph.tH * p)) < 1e-15
        assert r[M_EQ] == 0.0 and np.abs(r[9:18]).max() == 0.0
    assert seen == {"elastic", "plastic"}


def micro_phase():
    return W.Phase(lam=1.0, mu=1.0, kappa=0.5, alpha=0.0, beta=0.4, gamma=1.1,
                   tY=np.inf, mY=0.02, mH=0.3, a1=1.5, b1=2.0)


def test_curvature_m_and_m_eq_closed_form():
    ph = micro_phase()
    pm = np.zeros((4, 4, 4), np.uint8)
    D = np.array([[0.2, 0.7, 0.0], [-0.3, 0.1, 0.4], [0.5, 0.0, -0.3]])
    times, E, G = W.ramp_path(8, G_end=0.04 * D.reshape(9), t_end=8.0)
    out = O.Solver(pm, [ph], tol=1e-12).solve(times, E, G)
    b, g, b1 = ph.beta, ph.gamma, ph.b1
    seen = set()
    for s in range(len(times) - 1):
        Gm = G[s].reshape(3, 3)
        Gs, Gk = 0.5 * (Gm + Gm.T), 0.5 * (Gm - Gm.T)
        meq_el = np.sqrt(b1 * (b + g) ** 2 * (Gs * Gs).sum() + b1 * (g + b) * (g - b) * (Gk * Gk).sum())
        r = out["resp"][s]
        if meq_el < ph.mY:
            seen.add("elastic")
            m = b * Gm + g * Gm.T
            assert np.abs(r[9:18] - m.reshape(9)).max() < 1e-15
            assert abs(r[M_EQ] - meq_el) < 1e-15
            assert r[Q_AVG] == 0.0
        else:
            seen.add("plastic")
            q = r[Q_AVG]
            assert q > 0.0
            # on the micro yield surface, and q from Eq. 32 out of the trial state
            assert abs(r[M_EQ] - (ph.mY + ph.mH * q)) < 1e-15
            q_prev = out["resp"][s - 1][Q_AVG]
            # trial couple stress = m_n + B (Gamma - Gamma_n): its m_eq by hand
            Gn = G[s - 1].reshape(3, 3)
            mn = out["resp"][s - 1][9:18].reshape(3, 3)
            mt = mn + b * (Gm - Gn) + g * (Gm - Gn).T
            ms, mk = 0.5 * (mt + mt.T), 0.5 * (mt - mt.T)
            meq_tr = np.sqrt(b1 * (ms * ms).sum() + b1 * (g + b) / (g - b) * (mk * mk).sum())
            bg = b1 * (g + b)
            q_ref = q_prev * bg / (ph.mH + bg) + (meq_tr - ph.mY) / (ph.mH + bg)
            assert abs(q - q_ref) < 1e-15
        assert r[T_EQ] == 0.0 and r[P_AVG] == 0.0
    assert seen == {"elastic", "plastic"}


def test_two_voxel_state_by_hand():
    pa = W.Phase(lam=1.0, mu=1.0, kappa=0.5, alpha=0.0, beta=0.5, gamma=1.5,
                 tY=1.0, tH=0.0, mY=1.0, mH=0.0, a1=1.5, b1=2.0)      # a2 = 3, b2 = 4
    pb = W.Phase(lam=1.0, mu=1.0, kappa=1.0, alpha=0.0, beta=0.7, gamma=0.7,
                 tY=1.0, tH=0.0, mY=1.0, mH=0.0, a1=1.5, b1=1.5)      # beta == gamma
    pm = np.array([0, 1], np.uint8).reshape(1, 1, 2)
    s = O.Solver(pm, [pa, pb], tol=1e-8)
    t = np.zeros((1, 1, 2, 3, 3))
    m = np.zeros((1, 1, 2, 3, 3))
    # voxel 0: dev t = 2 e1 (x) e2, |sym|^2 = |skw|^2 = 2: t_eq = sqrt(1.5 * 2 + 3 * 2) = 3
    t[0, 0, 0] = np.eye(3) + 2.0 * np.outer([1, 0, 0], [0, 1, 0])
    # m_23 = 3, m_32 = 1: |sym|^2 = 8, |skw|^2 = 2: m_eq = sqrt(2 * 8 + 4 * 2) = sqrt(24)
    m[0, 0, 0, 1, 2], m[0, 0, 0, 2, 1] = 3.0, 1.0
    # voxel 1: t = 2 I (no deviator): t_eq = 0; m_12 = 2: beta == gamma drops the
    # skew term: m_eq = sqrt(1.5 * 2)
    t[0, 0, 1] = 2.0 * np.eye(3)
    m[0, 0, 1, 0, 1] = 2.0
    st = dict(t=t, m=m, e=np.zeros_like(t), g=np.zeros_like(t),
              p=np.array([0.25, 0.75]).reshape(1, 1, 2), q=np.array([0.5, 0.0]).reshape(1, 1, 2))
    r = s.response(st)
    assert abs(r[T_EQ] - 1.5) < 1e-15
    assert abs(r[M_EQ] - 0.5 * (np.sqrt(24.0) + np.sqrt(3.0))) < 1e-15
    assert r[P_AVG] == 0.5 and r[Q_AVG] == 0.25
    assert np.array_equal(r[0:9], (t[0, 0, 0] + t[0, 0, 1]).reshape(9) / 2)
    assert np.array_equal(r[9:18], (m[0, 0, 0] + m[0, 0, 1]).reshape(9) / 2)
