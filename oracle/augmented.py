"""Augmented-Lagrangian scheme for high phase contrast (TEST INFRASTRUCTURE ONLY).

The paper's conclusion (Sec. 4) names, as the remedy for the basic scheme's
loss of convergence at high phase contrast, the augmented-Lagrangian scheme
of Michel, Moulinec and Suquet extended to the nonlinear micropolar law, and
leaves that extension to a later paper.  This module writes the extension out
for the elastoplastic law of Alg. 1, in the alternating-direction form of
that scheme.

Unknowns at every voxel: a local strain and curvature d = (d_e, d_g), the
generalized stresses sigma(d) = (t, m) that Alg. 1 returns for it with the
step's history, and a multiplier lambda (stress and couple stress).  The
penalty is the reference medium C0 = (A0, B0) of the Green operator.  One
iteration:
  1. compatible step: (e, gamma) = (E, Gamma) + G0(lambda - C0 d), the Green
     operator of Eqs. 33-35 loaded by the polarization lambda - C0 d, so that
     e has mean E and gamma mean Gamma;
  2. local step, voxel by voxel: sigma(d') + C0 d' = lambda + C0 (e, gamma);
  3. multiplier update: lambda' = lambda + C0 ((e, gamma) - d').
After step 2, step 3 gives lambda' = sigma(d'), so the multiplier equals the
stresses of d after every iteration and is not stored: the polarization of
step 1 is sigma(d) - C0 d, the form of Eq. 34 evaluated at d, and the
right-hand side of step 2 is sigma(d) + C0 (e, gamma).  A fixed point has
d = (e, gamma) and is the fixed point of the basic scheme (Alg. 2).

The local step.  Alg. 1 acts on each level separately and, at the macro
level, scales the deviator of the trial stress by f = R1 / t_eq^tr (both the
symmetric and the skew part: 2 a2 kappa = 2 a1 mu), at the micro level the
whole trial couple stress by g = R2 / m_eq^tr.  With the isotropic laws of
Eq. 6 the local equation splits into three parts of each tensor: the
volumetric part tr(V) I / 3, the symmetric deviator and the skew part, on
which A (resp. B, written as m = B gamma) and A0 (B0) act as scalars:
  macro: 3 lam + 2 mu, 2 mu, 2 kappa;  micro: 3 alpha + beta + gamma,
  beta + gamma, beta - gamma.
For a given scale factor s each part of d solves a scalar equation
  s_j (b_j + a_j d_j) + a0_j d_j = r_j,    b = history base t_n - A e_n,
with s_j = f on the two deviatoric macro parts, 1 on the volumetric one, and
g on every micro part.  The factor itself is the root of the consistency
condition of Alg. 1, F(s) = s * eq(t_tr(d(s))) - R(d(s)) = 0 with
R = Y + H * (eq - R_n) / (H + c) the Eq. 32 hardening, which is increasing
in s on (0, 1]: it is found by bisection to machine precision.  An elastic
voxel (trial equivalent stress below R_n at s = 1) keeps s = 1.  A part on
which both the phase and the reference have zero stiffness (the skew
curvature when beta = gamma and beta0 = gamma0) carries no stress; its d is
taken from the compatible field.

Error measure: Eqs. 36-38 applied to the iterates (d, sigma(d)) in place of
(e, sigma(e)).  The strain-like averages in the denominators are the
prescribed E, Gamma (d reaches them only at convergence).

Eq. 5 (anisotropic) phases and tensor reference media are not covered.
"""
from __future__ import annotations

import numpy as np

from oracle import micropolar as O

BISECTIONS = 80


def _parts(V):
    """Volumetric, symmetric-deviatoric and skew parts of (..., 3, 3) tensors."""
    vol = (np.trace(V, axis1=-2, axis2=-1) / 3.0)[..., None, None] * O.DELTA
    return vol, O.sym(V) - vol, O.skw(V)


def _moduli(c, level):
    """Scalar moduli of the three parts, per voxel (or scalars for a medium)."""
    if level == "macro":
        return (3 * c["lam"] + 2 * c["mu"], 2 * c["mu"], 2 * c["kappa"])
    return (3 * c["alpha"] + c["beta"] + c["gamma"], c["beta"] + c["gamma"], c["beta"] - c["gamma"])


def _solve_parts(r, b, comp, a, a0, scale):
    """d with s_j (b_j + a_j d_j) + a0_j d_j = r_j on each part j.

    scale: per-part factors (arrays broadcastable to the voxels); a part with
    a_j = a0_j = 0 takes the compatible field's part."""
    d = np.zeros_like(r)
    for rj, bj, cj, aj, a0j, sj in zip(_parts(r), _parts(b), _parts(comp), a, a0, scale):
        aj = np.broadcast_to(aj, rj.shape[:-2])
        a0j = np.broadcast_to(np.asarray(a0j, float), rj.shape[:-2])
        sj = np.broadcast_to(sj, rj.shape[:-2])
        den = sj * aj + a0j
        inert = (aj == 0.0) & (a0j == 0.0)
        with np.errstate(divide="ignore", invalid="ignore"):
            dj = (rj - sj[..., None, None] * bj) / np.where(inert, 1.0, den)[..., None, None]
        d += np.where(inert[..., None, None], cj, dj)
    return d


def _law(a, x):
    """Isotropic law applied part by part: sum_j a_j x_j."""
    out = np.zeros_like(x)
    for xj, aj in zip(_parts(x), a):
        out += np.broadcast_to(aj, xj.shape[:-2])[..., None, None] * xj
    return out


def local_step(rt, rm, ec, gc, bt, bm, p_n, q_n, c, ref):
    """Solve sigma(d) + C0 d = (rt, rm) voxel by voxel (the local step).

    rt, rm: right-hand sides (..., 3, 3); ec, gc: compatible strain and
    curvature; bt = t_n - A e_n, bm = m_n - B g_n: the history bases; p_n,
    q_n; c: per-voxel constants (micropolar.voxel_constants); ref: the six
    constants of C0.  Returns (d_e, d_g)."""
    lam0, mu0, kap0, alp0, bet0, gam0 = ref
    r0 = dict(lam=lam0, mu=mu0, kappa=kap0, alpha=alp0, beta=bet0, gamma=gam0)
    shape = rt.shape[:-2]
    one = np.ones(shape)

    # macro level: the factor f scales the two deviatoric parts
    a, a0 = _moduli(c, "macro"), _moduli(r0, "macro")
    Rn_t = c["tY"] + c["tH"] * p_n
    ct = 2 * c["a1"] * c["mu"]

    def macro(f):
        d = _solve_parts(rt, bt, ec, a, a0, (one, f, f))
        teq = O.t_eq(bt + _law(a, d), c)
        with np.errstate(invalid="ignore"):
            dp = (teq - c["tY"] - c["tH"] * p_n) / (c["tH"] + ct)
            F = f * teq - (Rn_t + c["tH"] * dp)
        return d, teq, F

    d_e, teq1, _ = macro(one)
    plastic = teq1 >= Rn_t
    f = _bisect(lambda s: macro(s)[2], plastic, shape)
    d_e = np.where(plastic[..., None, None], macro(f)[0], d_e)

    # micro level: the factor g scales the whole couple stress
    a, a0 = _moduli(c, "micro"), _moduli(r0, "micro")
    Rn_m = c["mY"] + c["mH"] * q_n
    cm = c["b1"] * (c["gamma"] + c["beta"])

    def micro(g):
        d = _solve_parts(rm, bm, gc, a, a0, (g, g, g))
        meq = O.m_eq(bm + _law(a, d), c)
        with np.errstate(invalid="ignore"):
            dq = (meq - c["mY"] - c["mH"] * q_n) / (c["mH"] + cm)
            F = g * meq - (Rn_m + c["mH"] * dq)
        return d, meq, F

    d_g, meq1, _ = micro(one)
    plastic = meq1 >= Rn_m
    g = _bisect(lambda s: micro(s)[2], plastic, shape)
    d_g = np.where(plastic[..., None, None], micro(g)[0], d_g)
    return d_e, d_g


def _bisect(F, mask, shape):
    """Root in (0, 1] of the increasing F where mask is set (1 elsewhere)."""
    lo = np.zeros(shape)
    hi = np.ones(shape)
    if not mask.any():
        return hi
    for _ in range(BISECTIONS):
        mid = 0.5 * (lo + hi)
        neg = F(mid) < 0.0
        lo = np.where(neg, mid, lo)
        hi = np.where(neg, hi, mid)
    return np.where(mask, 0.5 * (lo + hi), 1.0)


def field_error_prescribed(a_new, a_old, mean, norm="local"):
    """Eq. 38 (local) or Eq. 37 (average) with a prescribed mean in the
    denominator (rms guard as micropolar.field_error)."""
    d = np.sqrt(O.ddot(a_new - a_old, a_new - a_old))
    num = d.max() if norm == "local" else d.mean()
    if num == 0.0:
        return 0.0
    den = float(np.sqrt(O.ddot(mean, mean)))
    rms = float(np.sqrt(O.ddot(a_new, a_new).mean()))
    if den <= O.GUARD * rms:
        den = rms
    return float(num / den)


class ALSolver(O.Solver):
    """The augmented-Lagrangian scheme in the load-step driver of Alg. 2.

    Same inputs, first iterate (uniform E at the first step, linear
    extrapolation after), history commit and outputs as micropolar.Solver;
    only the loop body differs.  ref_mode "geometric_mean" (the unweighted
    geometric mean of each modulus over the phases present) is the choice of
    Michel, Moulinec and Suquet for this scheme."""

    def __init__(self, *args, relax=1.0, **kw):
        super().__init__(*args, **kw)
        self.relax = float(relax)
        if len(self.ref) != 6:
            raise ValueError("the augmented-Lagrangian oracle takes an isotropic reference medium")
        if any(getattr(p, "A", None) is not None for p in self.phases):
            raise ValueError("the augmented-Lagrangian oracle covers Eq. 6 phases only")
        # the penalty must be positive definite on every part that carries
        # stress: gamma0 = beta0 only where every phase has beta = gamma (the
        # skew curvature then carries no stress anywhere); otherwise the local
        # step can have no solution
        tab = O.phase_table(self.phases)[np.unique(self.pm)]
        if not (self.ref[5] - self.ref[4] > 0 or np.all(tab[:, 5] == tab[:, 4])):
            raise ValueError("the penalty needs gamma0 > beta0 unless every phase has beta = gamma")

    def _bases(self):
        """History bases t_n - A e_n, m_n - B g_n of every voxel."""
        h, c = self.hist, self.c
        bt = h["t"] - _law(_moduli(c, "macro"), h["e"])
        bm = h["m"] - _law(_moduli(c, "micro"), h["g"])
        return bt, bm

    def iteration(self, st, E, G, eig=None):
        """One iteration from the state st = (d, sigma(d), p, q)."""
        tau, mu = self.polarization(st, eig)                 # sigma(d) - C0 d
        de, dg = self.green.apply(O.to_f9(tau), O.to_f9(mu))
        e = O.to_t33(de) + E                                  # compatible step
        g = O.to_t33(dg) + G
        if self.relax != 1.0:
            # over-relaxation: the compatible field enters steps 2 and 3 as
            # relax * e + (1 - relax) * d
            e = self.relax * e + (1.0 - self.relax) * st["e"]
            g = self.relax * g + (1.0 - self.relax) * st["g"]
        rt = st["t"] + O.apply_A(self.green.A0, e)            # lambda + C0 e
        rm = st["m"] + O.apply_B(self.green.B0, g)
        bt, bm = self._bases()
        h = self.hist
        d_e, d_g = local_step(rt, rm, e, g, bt, bm, h["p"], h["q"], self.c, self.ref)
        t, m, p, q = self._return_map(d_e, d_g)
        return dict(e=d_e, g=d_g, t=t, m=m, p=p, q=q)

    def step(self, t_new, E9, G9, iters=None, eig=None):
        E = np.asarray(E9, float).reshape(3, 3)
        G = np.asarray(G9, float).reshape(3, 3)
        if self.steps == 0:
            e = np.broadcast_to(E, self.hist["e"].shape).copy()
            g = np.broadcast_to(G, self.hist["g"].shape).copy()
        else:
            t0 = self.times[0] if self.times[0] is not None else 0.0
            r = (t_new - self.times[1]) / (self.times[1] - t0)
            e = self.hist["e"] + r * (self.hist["e"] - self.e_prev)
            g = self.hist["g"] + r * (self.hist["g"] - self.g_prev)
        t, m, p, q = self._return_map(e, g)
        st = dict(e=e, g=g, t=t, m=m, p=p, q=q)
        err = 2 * self.tol
        it = 0
        while (err > self.tol) if iters is None else (it < iters):
            if iters is None and it >= self.max_iter:
                break
            new = self.iteration(st, E, G, eig)
            err = max(field_error_prescribed(new["e"], st["e"], E, self.norm),
                      O.field_error(new["t"], st["t"], self.norm),
                      field_error_prescribed(new["g"], st["g"], G, self.norm),
                      O.field_error(new["m"], st["m"], self.norm))
            st = new
            it += 1
            if not np.isfinite(err):
                break
        self.cur = st
        self.last_err, self.last_iters = err, it
        return it, err
