"""Continuum elastoplastic tangents and an RK4 stress integrator (TEST ONLY).

An independent route to the stresses of the micropolar elastoplastic model,
used to pin the radial-return oracle and to build manufactured solutions:

  * elastic law in its sym/skew form                            -- Eq. 8
  * flow directions df/dt, dg/dm                                -- Eqs. 19, 20
  * rates p_dot, q_dot with the max(., 0) loading switch        -- Eq. 84
  * stress rates t_dot = A:(e_dot - e_dot^p), m_dot likewise    -- Eq. 24

The strain rate is constant inside each integration interval (strain paths
are piecewise linear in time).  The transition from elastic to plastic inside
a sub-step is located by bisection on f (resp. g) before the plastic tangent
takes over, so a kink in the path costs no accuracy.

Vectorised over a leading voxel axis; tensors are (V, 3, 3).
"""
from __future__ import annotations

import numpy as np

I3 = np.eye(3)


def _sym(X):
    return 0.5 * (X + np.swapaxes(X, -1, -2))


def _skw(X):
    return 0.5 * (X - np.swapaxes(X, -1, -2))


def _tr(X):
    return np.trace(X, axis1=-2, axis2=-1)


def _dd(X, Y):
    return np.einsum("...kl,...kl->...", X, Y)


def _s(c, k):
    return np.asarray(c[k], float)[..., None, None]


def law_t(c, e):
    """Eq. 8: t = lam tr(e) I + 2 mu e_(kl) + 2 kappa e_[kl]."""
    return _s(c, "lam") * _tr(e)[..., None, None] * I3 + 2 * _s(c, "mu") * _sym(e) \
        + 2 * _s(c, "kappa") * _skw(e)


def law_m(c, g):
    """Eq. 8: m = alpha tr(g) I + (beta + gamma) g_(kl) + (beta - gamma) g_[kl]."""
    return _s(c, "alpha") * _tr(g)[..., None, None] * I3 \
        + (_s(c, "beta") + _s(c, "gamma")) * _sym(g) + (_s(c, "beta") - _s(c, "gamma")) * _skw(g)


def _b2(c):
    gmb = np.asarray(c["gamma"], float) - np.asarray(c["beta"], float)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(gmb != 0, np.asarray(c["b1"]) * (np.asarray(c["gamma"]) + np.asarray(c["beta"]))
                        / np.where(gmb != 0, gmb, 1.0), 0.0)


def f_yield(c, t, p):
    """Eqs. 13-15."""
    s = t - _tr(t)[..., None, None] * I3 / 3
    a2 = np.asarray(c["a1"]) * np.asarray(c["mu"]) / np.asarray(c["kappa"])
    teq = np.sqrt(np.asarray(c["a1"]) * _dd(_sym(s), _sym(s)) + a2 * _dd(_skw(s), _skw(s)))
    return teq - (np.asarray(c["tY"]) + np.asarray(c["tH"]) * p), teq


def g_yield(c, m, q):
    """Eqs. 16-18 (b2 term dropped where gamma == beta: the skew part is 0)."""
    b2 = _b2(c)
    skw2 = np.where(np.asarray(c["gamma"]) != np.asarray(c["beta"]), _dd(_skw(m), _skw(m)), 0.0)
    meq = np.sqrt(np.asarray(c["b1"]) * _dd(_sym(m), _sym(m)) + b2 * skw2)
    return meq - (np.asarray(c["mY"]) + np.asarray(c["mH"]) * q), meq


def rates(c, t, m, p, q, de, dg, plastic_t, plastic_m):
    """Stress and hardening rates for strain rates de, dg (Eqs. 19-20, 24, 84)."""
    a1 = np.asarray(c["a1"], float)
    a2 = a1 * np.asarray(c["mu"]) / np.asarray(c["kappa"])
    b1 = np.asarray(c["b1"], float)
    b2 = _b2(c)
    # macro
    s = t - _tr(t)[..., None, None] * I3 / 3
    _, teq = f_yield(c, t, p)
    safe = np.where(teq > 0, teq, 1.0)[..., None, None]
    N = (a1[..., None, None] * _sym(s) + a2[..., None, None] * _skw(s)) / safe
    AN = law_t(c, N)
    Ade = law_t(c, de)
    num = np.maximum(_dd(N, Ade), 0.0)
    den = _dd(N, AN) + np.asarray(c["tH"])
    pdot = np.where(plastic_t & (teq > 0), num / np.where(den > 0, den, 1.0), 0.0)
    tdot = Ade - pdot[..., None, None] * AN
    # micro: plastic curvature rate g^p_mn = qdot * (dg/dm)_nm
    _, meq = g_yield(c, m, q)
    safe = np.where(meq > 0, meq, 1.0)[..., None, None]
    Nm = (b1[..., None, None] * _sym(m) + b2[..., None, None] * _skw(m)) / safe
    BNt = law_m(c, np.swapaxes(Nm, -1, -2))
    Bdg = law_m(c, dg)
    num = np.maximum(_dd(Nm, Bdg), 0.0)
    den = _dd(Nm, BNt) + np.asarray(c["mH"])
    qdot = np.where(plastic_m & (meq > 0), num / np.where(den > 0, den, 1.0), 0.0)
    mdot = Bdg - qdot[..., None, None] * BNt
    return tdot, mdot, pdot, qdot


def _rk4(c, y, de, dg, dt, pt, pm):
    t, m, p, q = y
    d = dt[..., None, None]

    def ev(tt, mm, pp, qq):
        return rates(c, tt, mm, pp, qq, de, dg, pt, pm)

    k1 = ev(t, m, p, q)
    k2 = ev(t + 0.5 * d * k1[0], m + 0.5 * d * k1[1], p + 0.5 * dt * k1[2], q + 0.5 * dt * k1[3])
    k3 = ev(t + 0.5 * d * k2[0], m + 0.5 * d * k2[1], p + 0.5 * dt * k2[2], q + 0.5 * dt * k2[3])
    k4 = ev(t + d * k3[0], m + d * k3[1], p + dt * k3[2], q + dt * k3[3])
    t = t + d / 6 * (k1[0] + 2 * k2[0] + 2 * k3[0] + k4[0])
    m = m + d / 6 * (k1[1] + 2 * k2[1] + 2 * k3[1] + k4[1])
    p = p + dt / 6 * (k1[2] + 2 * k2[2] + 2 * k3[2] + k4[2])
    q = q + dt / 6 * (k1[3] + 2 * k2[3] + 2 * k3[3] + k4[3])
    return t, m, p, q


def integrate(c, state, de, dg, T, substeps=200, tol_rel=1e-13):
    """Integrate the rate equations over a time T with constant strain rates.

    state = (t, m, p, q); de, dg (V, 3, 3) strain / curvature rates.
    A voxel is plastic at a level once its yield function reaches zero; while
    elastic, each sub-step that would cross the surface is cut at the
    crossing time (bisection) and finished with the plastic tangent.
    """
    t, m, p, q = (np.array(v, float) for v in state)
    V = p.shape
    h = T / substeps

    def status(t, m, p, q):
        f, teq = f_yield(c, t, p)
        g, meq = g_yield(c, m, q)
        R1 = np.asarray(c["tY"]) + np.asarray(c["tH"]) * p
        R2 = np.asarray(c["mY"]) + np.asarray(c["mH"]) * q
        return (np.isfinite(R1) & (f >= -tol_rel * np.abs(R1)),
                np.isfinite(R2) & (g >= -tol_rel * np.abs(R2)))

    tol_rel = max(tol_rel, 1e-12)

    def yields(y):
        f, _ = f_yield(c, y[0], y[2])
        g, _ = g_yield(c, y[1], y[3])
        return f, g

    def pick(sel, a, b):
        return tuple(np.where(sel[..., None, None] if x.ndim == len(V) + 2 else sel, yb, x)
                     for x, yb in zip(a, b))

    for _ in range(substeps):
        y = (t, m, p, q)
        left = np.full(V, h)
        # each pass either finishes a voxel's sub-step or stops it exactly on
        # a yield surface it was about to cross; a voxel crosses each surface
        # at most once per sub-step, so three passes always suffice
        for _pass in range(3):
            if not np.any(left > 0):
                break
            pt, pm = status(*y)
            full = _rk4(c, y, de, dg, left, pt, pm)
            f1, g1 = yields(full)
            cross = (left > 0) & ((((~pt) & (f1 > 0)) | ((~pm) & (g1 > 0))))
            done = (left > 0) & ~cross
            y = pick(done, y, full)
            left = np.where(done, 0.0, left)
            if not np.any(cross):
                break
            lo = np.zeros(V)
            hi = left.copy()
            for _ in range(80):
                mid = 0.5 * (lo + hi)
                ym = _rk4(c, y, de, dg, mid, pt, pm)
                fm, gm = yields(ym)
                over = ((~pt) & (fm > 0)) | ((~pm) & (gm > 0))
                hi = np.where(over, mid, hi)
                lo = np.where(over, lo, mid)
            tc = np.where(cross, hi, 0.0)
            ycr = _rk4(c, y, de, dg, tc, pt, pm)
            y = pick(cross, y, ycr)
            left = np.where(cross, left - tc, left)
        t, m, p, q = y
    return t, m, p, q
