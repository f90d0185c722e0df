"""Plain FP64 oracle of the micropolar basic scheme (TEST INFRASTRUCTURE ONLY).

Written from the paper, step by step, in its notation:
  * stiffness tensors A_klmn, B_lkmn of an isotropic phase     -- Eq. 6
  * elastic trial stresses                                      -- Eq. 30
  * equivalent stresses t_eq, m_eq                              -- Eqs. 14, 17
  * closed-form p, q update                                     -- Eq. 32
  * micropolar radial-return mapping                            -- Alg. 1
  * polarization stresses                                       -- Eq. 34
  * reference-medium Green operator, applied per frequency      -- Eqs. 33-35
  * reference medium A0 = <A(x)>, B0 = <B(x)>, isotropic or as
    general tensors of the phases' Eq. 5 / Eq. 6 laws             -- Alg. 2
  * error measure                                               -- Eqs. 36-38
  * elastoplastic FFT-based basic scheme                        -- Alg. 2

Readings of points the paper leaves open (each listed in the design notes):
  - The Green tensors are only cited.  Here they are not written out: for
    every frequency the oracle assembles the 6x6 Fourier symbol of the
    reference-medium balance operator (Eqs. 1, 2 with no body force/couple,
    the reference stiffnesses) by applying it to unit displacement /
    microrotation amplitudes, and inverts it with numpy.linalg.inv.  The uniform part
    A0:E of the second polarization only lives at k = 0, where the
    fluctuation is zero, so it never enters.
  - Continuous frequencies xi = 2 pi m / (n h); at k = 0 and at every
    Nyquist index of an even axis the fluctuating strain and curvature are 0.
  - beta = gamma makes b2 infinite in Alg. 1; the skew couple stress is then
    identically zero, the product b2 * |m_skew|^2 is taken as 0 and the skew
    scaling factor equals the symmetric one.
  - A zero average in the denominator of Eqs. 37/38 is replaced by the rms of
    the field when |<a>| <= 1e-6 rms(a); a zero numerator gives 0.
  - Equality at the yield surface takes the plastic branch (Delta p = 0).

Layout: tensor fields are arrays (9, n2, n1, n0) with component 3k + l for
V_kl, voxel arrays (n2, n1, n0) with x fastest.  Forward DFT unnormalised.
"""
from __future__ import annotations

import numpy as np

# Levi-Civita symbol eps[i, j, k]
EPS = np.zeros((3, 3, 3))
EPS[0, 1, 2] = EPS[1, 2, 0] = EPS[2, 0, 1] = 1.0
EPS[0, 2, 1] = EPS[2, 1, 0] = EPS[1, 0, 2] = -1.0
DELTA = np.eye(3)

PHASE_KEYS = ("lam", "mu", "kappa", "alpha", "beta", "gamma",
              "tY", "tH", "mY", "mH", "a1", "b1")


# ----------------------------------------------------------------------------
# Eq. 6: isotropic stiffness tensors
# ----------------------------------------------------------------------------

def stiffness_A(lam, mu, kappa):
    """A_klmn = lam d_kl d_mn + (mu + kappa) d_km d_ln + (mu - kappa) d_kn d_lm."""
    d = DELTA
    return (lam * np.einsum("kl,mn->klmn", d, d)
            + (mu + kappa) * np.einsum("km,ln->klmn", d, d)
            + (mu - kappa) * np.einsum("kn,lm->klmn", d, d))


def stiffness_B(alpha, beta, gamma):
    """B_lkmn = alpha d_kl d_mn + beta d_km d_ln + gamma d_kn d_lm.

    Returned with its indices in the order (l, k, m, n) so that the couple
    stress is m_kl = B[l, k, m, n] gamma_mn.
    """
    d = DELTA
    return (alpha * np.einsum("kl,mn->lkmn", d, d)
            + beta * np.einsum("km,ln->lkmn", d, d)
            + gamma * np.einsum("kn,lm->lkmn", d, d))


def apply_A(A, e):
    """t_kl = A_klmn e_mn for e of shape (..., 3, 3); A (..., 3, 3, 3, 3)."""
    return np.einsum("...klmn,...mn->...kl", A, e)


def apply_B(B, g):
    """m_kl = B_lkmn gamma_mn, with B stored in index order (l, k, m, n)."""
    return np.einsum("...lkmn,...mn->...kl", B, g)


# ----------------------------------------------------------------------------
# helpers on (..., 3, 3) tensors
# ----------------------------------------------------------------------------

def sym(V):
    """V_(kl) = (V_kl + V_lk) / 2."""
    return 0.5 * (V + np.swapaxes(V, -1, -2))


def skw(V):
    """V_[kl] = (V_kl - V_lk) / 2."""
    return 0.5 * (V - np.swapaxes(V, -1, -2))


def dev(V):
    """s_kl = V_kl - tr(V) d_kl / 3."""
    tr = np.trace(V, axis1=-2, axis2=-1)
    return V - tr[..., None, None] * DELTA / 3.0


def ddot(U, V):
    return np.einsum("...kl,...kl->...", U, V)


def to_t33(f9):
    """(9, ...) -> (..., 3, 3)."""
    f9 = np.asarray(f9)
    return np.moveaxis(f9.reshape((3, 3) + f9.shape[1:]), (0, 1), (-2, -1))


def to_f9(t33):
    """(..., 3, 3) -> (9, ...)."""
    t = np.moveaxis(t33, (-2, -1), (0, 1))
    return t.reshape((9,) + t.shape[2:])


# ----------------------------------------------------------------------------
# per-voxel constants
# ----------------------------------------------------------------------------

def phase_table(phases):
    """(n_phases, 12) array of constants in the order PHASE_KEYS."""
    rows = []
    for p in phases:
        if isinstance(p, dict):
            rows.append([float(p[k]) for k in PHASE_KEYS])
        elif hasattr(p, "as_tuple"):
            rows.append(list(p.as_tuple()))
        else:
            rows.append([float(v) for v in p])
    return np.array(rows, dtype=np.float64)


def voxel_constants(phase_map, phases):
    """dict of per-voxel constant arrays shaped like phase_map."""
    tab = phase_table(phases)
    pm = np.asarray(phase_map).astype(np.intp)
    return {k: tab[:, i][pm] for i, k in enumerate(PHASE_KEYS)}


# ----------------------------------------------------------------------------
# Eqs. 14, 17: equivalent stresses
# ----------------------------------------------------------------------------

def _a2(c):
    # Alg. 1: a2 = a1 mu / kappa
    return c["a1"] * c["mu"] / c["kappa"]


def _skew_ratio_b(c):
    """(b2, finite) with b2 = b1 (gamma + beta) / (gamma - beta) (Alg. 1).

    Where gamma == beta the ratio is infinite; the caller drops the term.
    """
    gmb = c["gamma"] - c["beta"]
    finite = gmb != 0.0
    with np.errstate(divide="ignore", invalid="ignore"):
        b2 = np.where(finite, c["b1"] * (c["gamma"] + c["beta"]) / np.where(finite, gmb, 1.0), 0.0)
    return b2, finite


def t_eq(t, c):
    """Eq. 14 on the deviatoric part s of t."""
    s = dev(t)
    return np.sqrt(c["a1"] * ddot(sym(s), sym(s)) + _a2(c) * ddot(skw(s), skw(s)))


def m_eq(m, c):
    """Eq. 17 on the full couple stress (b2 term dropped where gamma == beta)."""
    b2, finite = _skew_ratio_b(c)
    skew2 = np.where(finite, ddot(skw(m), skw(m)), 0.0)
    return np.sqrt(c["b1"] * ddot(sym(m), sym(m)) + b2 * skew2)


# ----------------------------------------------------------------------------
# Alg. 1: micropolar radial-return mapping (vectorised over voxels)
# ----------------------------------------------------------------------------

def radial_return(e, g, e_n, g_n, t_n, m_n, p_n, q_n, phase_map, phases):
    """Alg. 1 at every voxel.  Tensor inputs (..., 3, 3), scalars (...),
    phase_map (...) of phase ids into `phases`.  Returns (t, m, p, q)."""
    pm = np.asarray(phase_map)
    c = voxel_constants(pm, phases)
    tab = phase_table(phases)

    t_tr = np.empty(np.broadcast_shapes(np.shape(t_n), np.shape(e)))
    m_tr = np.empty(np.broadcast_shapes(np.shape(m_n), np.shape(g)))
    de = np.broadcast_to(e - e_n, t_tr.shape)
    dg = np.broadcast_to(g - g_n, m_tr.shape)
    tn = np.broadcast_to(t_n, t_tr.shape)
    mn = np.broadcast_to(m_n, m_tr.shape)
    for ph in np.unique(pm):
        sel = pm == ph
        lam, mu_, kap, alp, bet, gam = tab[ph, :6]
        # Eq. 30: elastic trial stresses, with the phase's general
        # centrosymmetric tensors of Eq. 5 when it has them (A, B attributes;
        # B in index order (l, k, m, n) as stiffness_B), else those of Eq. 6
        A = getattr(phases[ph], "A", None)
        B = getattr(phases[ph], "B", None)
        A = stiffness_A(lam, mu_, kap) if A is None else np.asarray(A, float)
        B = stiffness_B(alp, bet, gam) if B is None else np.asarray(B, float)
        t_tr[sel] = tn[sel] + apply_A(A, de[sel])
        m_tr[sel] = mn[sel] + apply_B(B, dg[sel])

    # a2 = a1 mu / kappa, b2 = b1 (gamma + beta) / (gamma - beta)
    a1, b1 = c["a1"], c["b1"]
    a2 = _a2(c)
    b2, b2_finite = _skew_ratio_b(c)

    # Eqs. 14, 17 at the trial state
    s_tr = dev(t_tr)
    ss_sym, ss_skw = sym(s_tr), skw(s_tr)
    teq_tr = np.sqrt(a1 * ddot(ss_sym, ss_sym) + a2 * ddot(ss_skw, ss_skw))
    ms_sym, ms_skw = sym(m_tr), skw(m_tr)
    meq_tr = np.sqrt(b1 * ddot(ms_sym, ms_sym)
                     + b2 * np.where(b2_finite, ddot(ms_skw, ms_skw), 0.0))

    mu, kappa, beta, gamma = c["mu"], c["kappa"], c["beta"], c["gamma"]
    tY, tH, mY, mH = c["tY"], c["tH"], c["mY"], c["mH"]

    with np.errstate(invalid="ignore", divide="ignore", over="ignore"):
        # macro level
        elastic_t = teq_tr < tY + tH * p_n
        p_pl = p_n * (2 * a1 * mu) / (tH + 2 * a1 * mu) + (teq_tr - tY) / (tH + 2 * a1 * mu)  # Eq. 32
        R1 = tY + tH * p_pl
        f_sym = R1 / (R1 + 2 * (p_pl - p_n) * a1 * mu)
        f_skw = R1 / (R1 + 2 * (p_pl - p_n) * a2 * kappa)
        vol = (np.trace(t_tr, axis1=-2, axis2=-1) / 3.0)[..., None, None] * DELTA
        t_pl = vol + f_sym[..., None, None] * ss_sym + f_skw[..., None, None] * ss_skw
        t = np.where(elastic_t[..., None, None], t_tr, t_pl)
        p = np.where(elastic_t, p_n, p_pl)

        # micro level
        elastic_m = meq_tr < mY + mH * q_n
        q_pl = q_n * (b1 * (gamma + beta)) / (mH + b1 * (gamma + beta)) \
            + (meq_tr - mY) / (mH + b1 * (gamma + beta))  # Eq. 32
        R2 = mY + mH * q_pl
        g_sym = R2 / (R2 + (q_pl - q_n) * b1 * (gamma + beta))
        # b2 (gamma - beta) -> b1 (gamma + beta) when gamma == beta
        b2gmb = np.where(b2_finite, b2 * (gamma - beta), b1 * (gamma + beta))
        g_skw = R2 / (R2 + (q_pl - q_n) * b2gmb)
        m_pl = g_sym[..., None, None] * ms_sym + g_skw[..., None, None] * ms_skw
        m = np.where(elastic_m[..., None, None], m_tr, m_pl)
        q = np.where(elastic_m, q_n, q_pl)
    return t, m, p, q


# ----------------------------------------------------------------------------
# Reference medium and Green operator (Eqs. 33-35)
# ----------------------------------------------------------------------------

def reference_medium(phase_map, phases, mode="phase_mean"):
    """Elastic constants (lam, mu, kappa, alpha, beta, gamma) of the reference.

    "volume_mean": <A(x)>, <B(x)> over the cell (Alg. 2).  For isotropic
    phases this is the volume average of each modulus.
    "phase_mean": unweighted mean of each modulus over the phases present.
    "geometric_mean": unweighted geometric mean of each modulus over the
    phases present (the augmented-Lagrangian scheme's penalty).
    "tensor_mean", "tensor_phase_mean": the same two means taken over every
    phase's own tensors; they return the pair (A0, B0) of tensors instead of
    constants (see reference_tensors).
    """
    if mode == "tensor_mean":
        return reference_tensors(phase_map, phases)
    if mode == "tensor_phase_mean":
        return reference_tensors(phase_map, phases, weights="phase")
    tab = phase_table(phases)[:, :6]
    pm = np.asarray(phase_map).astype(np.intp)
    if mode == "volume_mean":
        return tuple(float(v) for v in tab[pm.ravel()].mean(axis=0))
    if mode == "phase_mean":
        present = np.unique(pm)
        return tuple(float(v) for v in tab[present].mean(axis=0))
    if mode == "geometric_mean":
        # the penalty of the augmented-Lagrangian scheme: the unweighted
        # geometric mean of each modulus over the phases present (0 where a
        # phase has a zero modulus)
        present = np.unique(pm)
        return tuple(float(np.prod(tab[present, k]) ** (1.0 / len(present))) for k in range(6))
    raise ValueError(mode)


def reference_tensors(phase_map, phases, weights="volume"):
    """Alg. 2 taken literally: A0 = <A(x)>, B0 = <B(x)> over the cell, with
    the Eq. 5 tensors of a phase that has them (A, B attributes) and the
    Eq. 6 tensors of the others.  weights="phase": the unweighted mean over
    the phases present instead.  B0 in index order (l, k, m, n)."""
    pm = np.asarray(phase_map).astype(np.intp)
    tab = phase_table(phases)[:, :6]
    present = np.unique(pm)
    A0 = np.zeros((3, 3, 3, 3))
    B0 = np.zeros((3, 3, 3, 3))
    for ph in present:
        w = np.count_nonzero(pm == ph) / pm.size if weights == "volume" else 1.0 / len(present)
        lam, mu, kap, alp, bet, gam = tab[ph]
        A = getattr(phases[ph], "A", None)
        B = getattr(phases[ph], "B", None)
        A0 += w * (stiffness_A(lam, mu, kap) if A is None else np.asarray(A, float))
        B0 += w * (stiffness_B(alp, bet, gam) if B is None else np.asarray(B, float))
    return A0, B0


def frequencies(n, h, half=True):
    """xi_k = 2 pi m_k / (n_k h) on the rfftn grid (last array axis = x halved).

    Returns (xi1, xi2, xi3, nyquist_mask) broadcastable to (n2, n1, n0//2+1).
    """
    n0, n1, n2 = n
    m0 = np.fft.rfftfreq(n0) * n0 if half else np.fft.fftfreq(n0) * n0
    m1 = np.fft.fftfreq(n1) * n1
    m2 = np.fft.fftfreq(n2) * n2
    xi1 = (2 * np.pi * m0 / (n0 * h))[None, None, :]
    xi2 = (2 * np.pi * m1 / (n1 * h))[None, :, None]
    xi3 = (2 * np.pi * m2 / (n2 * h))[:, None, None]
    nyq = np.zeros((n2, n1, len(m0)), bool)
    if n0 % 2 == 0:
        nyq |= (np.abs(m0) == n0 // 2)[None, None, :]
    if n1 % 2 == 0:
        nyq |= (np.abs(m1) == n1 // 2)[None, :, None]
    if n2 % 2 == 0:
        nyq |= (np.abs(m2) == n2 // 2)[:, None, None]
    return xi1, xi2, xi3, nyq


def strain_of_amplitudes(xi, u, phi):
    """Fourier amplitudes of Eq. 1: e_kl = i xi_k u_l + eps_lkm phi_m,
    gamma_kl = i xi_l phi_k.  xi (F, 3) real, u, phi (F, 3) complex."""
    e = 1j * xi[:, :, None] * u[:, None, :] + np.einsum("lkm,fm->fkl", EPS, phi)
    g = 1j * phi[:, :, None] * xi[:, None, :]
    return e, g


def balance_residual(xi, t_hat, m_hat):
    """Fourier form of Eq. 2 with f = l = 0:
    r_u_l = i xi_k t_kl,  r_phi_l = i xi_k m_kl + eps_lkm t_km."""
    ru = 1j * np.einsum("fk,fkl->fl", xi, t_hat)
    rp = 1j * np.einsum("fk,fkl->fl", xi, m_hat) + np.einsum("lkm,fkm->fl", EPS, t_hat)
    return ru, rp


class GreenOperator:
    """Polarization (tau, mu) -> fluctuating (e~, gamma~) of the reference medium.

    For each frequency, solve the balance equations of the homogeneous
    reference medium loaded by the polarization stresses (Eq. 34): with
    t = A0 e~ + tau and m = B0 gamma~ + mu, Eq. 2 must hold for the periodic
    fluctuation of Eq. 1.  The 6x6 symbol of the operator (u, phi) ->
    balance residual is assembled column by column from unit amplitudes and
    inverted once per frequency (the paper allows the Green tensors to be
    pre-computed and stored).

    ref: the six Eq. 6 constants of an isotropic reference medium, or a pair
    (A0, B0) of general tensors (B0 in index order (l, k, m, n)).
    """

    def __init__(self, n, h, ref, chunk=1 << 16):
        self.n, self.h = tuple(int(v) for v in n), float(h)
        if len(ref) == 2:
            self.A0 = np.asarray(ref[0], float).reshape(3, 3, 3, 3)
            self.B0 = np.asarray(ref[1], float).reshape(3, 3, 3, 3)
        else:
            lam, mu, kappa, alpha, beta, gamma = ref
            self.A0 = stiffness_A(lam, mu, kappa)
            self.B0 = stiffness_B(alpha, beta, gamma)
        xi1, xi2, xi3, nyq = frequencies(self.n, self.h, half=True)
        shp = nyq.shape
        X = np.stack(np.broadcast_arrays(xi1 + 0 * xi2 + 0 * xi3,
                                         xi2 + 0 * xi1 + 0 * xi3,
                                         xi3 + 0 * xi1 + 0 * xi2), axis=-1).reshape(-1, 3)
        zero = (X[:, 0] == 0) & (X[:, 1] == 0) & (X[:, 2] == 0)
        self.active = ~(zero | nyq.reshape(-1))
        self.xi = X
        self.shape = shp
        idx = np.nonzero(self.active)[0]
        self.idx = idx
        self.Minv = np.empty((len(idx), 6, 6), np.complex128)
        for s in range(0, len(idx), chunk):
            sl = idx[s:s + chunk]
            self.Minv[s:s + len(sl)] = np.linalg.inv(self._symbol(X[sl]))

    def _symbol(self, xi):
        F = xi.shape[0]
        M = np.empty((F, 6, 6), np.complex128)
        for j in range(6):
            u = np.zeros((F, 3), np.complex128)
            phi = np.zeros((F, 3), np.complex128)
            (u if j < 3 else phi)[:, j % 3] = 1.0
            e, g = strain_of_amplitudes(xi, u, phi)
            ru, rp = balance_residual(xi, apply_A(self.A0, e), apply_B(self.B0, g))
            M[:, :3, j] = ru
            M[:, 3:, j] = rp
        return M

    def apply_hat(self, tau_hat, mu_hat):
        """tau_hat, mu_hat: (F, 3, 3) complex on the rfftn grid (flattened).
        Returns (e_hat, g_hat) of the fluctuation, zero where inactive."""
        e_hat = np.zeros_like(tau_hat)
        g_hat = np.zeros_like(mu_hat)
        idx = self.idx
        xi = self.xi[idx]
        # source: balance residual of the polarization alone
        bu, bp = balance_residual(xi, tau_hat[idx], mu_hat[idx])
        b = np.concatenate([bu, bp], axis=1)
        x = -np.einsum("fij,fj->fi", self.Minv, b)
        e, g = strain_of_amplitudes(xi, x[:, :3], x[:, 3:])
        e_hat[idx] = e
        g_hat[idx] = g
        return e_hat, g_hat

    def apply(self, tau, mu):
        """Real fields (9, n2, n1, n0) -> fluctuating strain, curvature (9, ...)."""
        axes = (-3, -2, -1)
        th = np.fft.rfftn(tau, axes=axes)
        mh = np.fft.rfftn(mu, axes=axes)
        th = to_t33(th).reshape(-1, 3, 3)
        mh = to_t33(mh).reshape(-1, 3, 3)
        eh, gh = self.apply_hat(th, mh)
        eh = to_f9(eh.reshape(self.shape + (3, 3)))
        gh = to_f9(gh.reshape(self.shape + (3, 3)))
        s = (self.n[2], self.n[1], self.n[0])
        return (np.fft.irfftn(eh, s=s, axes=axes), np.fft.irfftn(gh, s=s, axes=axes))


# ----------------------------------------------------------------------------
# Eqs. 36-38: error measure
# ----------------------------------------------------------------------------

GUARD = 1e-6


def field_error(a_new, a_old, norm="local"):
    """err_a of Eq. 38 (local) or Eq. 37 (average), fields (..., 3, 3)."""
    d = np.sqrt(ddot(a_new - a_old, a_new - a_old))
    num = d.max() if norm == "local" else d.mean()
    if num == 0.0:
        return 0.0
    mean = a_new.reshape(-1, 3, 3).mean(axis=0)
    den = float(np.sqrt(ddot(mean, mean)))
    rms = float(np.sqrt(ddot(a_new, a_new).mean()))
    if den <= GUARD * rms:
        den = rms
    return float(num / den)


def error(new, old, norm="local"):
    """Eq. 36: max over a in {e, t, gamma, m}."""
    return max(field_error(new[k], old[k], norm) for k in ("e", "t", "g", "m"))


# ----------------------------------------------------------------------------
# Alg. 2: elastoplastic FFT-based basic scheme
# ----------------------------------------------------------------------------

class Solver:
    """Alg. 2 on a periodic voxel grid.

    phase_map (n2, n1, n0) uint8; phases: list of constant records; h voxel
    size; tol = epsilon; norm "local" (Eq. 38) or "average" (Eq. 37).
    ref_mode "phase_mean", "volume_mean" (isotropic reference media) or
    "tensor_mean", "tensor_phase_mean" (the same means of the phases'
    tensors); ref overrides it with six constants or a pair of tensors.
    eigen_t, eigen_m: optional manufactured stresses subtracted inside the
    polarization (verification form of the first loop line), callable
    step -> (9, n2, n1, n0) arrays.
    """

    def __init__(self, phase_map, phases, h=1.0, tol=1e-8, norm="local",
                 ref_mode="phase_mean", ref=None, max_iter=20000):
        self.pm = np.asarray(phase_map)
        n2, n1, n0 = self.pm.shape
        self.n = (n0, n1, n2)
        self.phases = phases
        self.c = voxel_constants(self.pm, phases)
        self.ref = tuple(ref) if ref is not None else reference_medium(self.pm, phases, ref_mode)
        self.green = GreenOperator(self.n, h, self.ref)
        self.tol, self.norm, self.max_iter = float(tol), norm, int(max_iter)
        shp = self.pm.shape + (3, 3)
        z = lambda: np.zeros(shp)
        # converged history: step n (last) and n-1 (before last)
        self.hist = dict(e=z(), g=z(), t=z(), m=z(),
                         p=np.zeros(self.pm.shape), q=np.zeros(self.pm.shape))
        self.e_prev, self.g_prev = z(), z()
        self.times = [None, None]   # t_{n-1}, t_n of the committed steps
        self.steps = 0
        self.cur = None

    def _return_map(self, e, g):
        h = self.hist
        return radial_return(e, g, h["e"], h["g"], h["t"], h["m"], h["p"], h["q"],
                             self.pm, self.phases)

    def polarization(self, st, eig=None):
        """Eq. 34: tau = t - A0 e, mu_kl = m_kl - B0_lkmn gamma_mn."""
        tau = st["t"] - apply_A(self.green.A0, st["e"])
        mu = st["m"] - apply_B(self.green.B0, st["g"])
        if eig is not None:
            tau = tau - eig[0]
            mu = mu - eig[1]
        return tau, mu

    def step(self, t_new, E9, G9, iters=None, eig=None):
        """Solve one load step to time t_new with macro strain E9, curvature G9.

        iters: run exactly this many loop iterations instead of testing err.
        Returns (iterations, err).
        """
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
            tau, mu = self.polarization(st, eig)
            de, dg = self.green.apply(to_f9(tau), to_f9(mu))
            e = to_t33(de) + E
            g = to_t33(dg) + G
            t, m, p, q = self._return_map(e, g)
            new = dict(e=e, g=g, t=t, m=m, p=p, q=q)
            err = error(new, st, self.norm)
            st = new
            it += 1
        self.cur = st
        self.last_err, self.last_iters = err, it
        return it, err

    def response(self, st=None):
        """Volume averages of one state: T, M, Ebar, Gbar (9 each), P, Q, Teq, Meq."""
        st = self.cur if st is None else st
        avg = lambda a: a.reshape(-1, 9).mean(axis=0)
        return np.concatenate([avg(st["t"]), avg(st["m"]), avg(st["e"]), avg(st["g"]),
                               [st["p"].mean(), st["q"].mean(),
                                t_eq(st["t"], self.c).mean(), m_eq(st["m"], self.c).mean()]])

    def solve(self, times, E, G, schedule=None, eig=None, fields_at=()):
        """Run the load path: times (S+1,) with times[0] the current time.

        Returns dict with per-step iterations, errors, responses (S, 40) and
        full fields at the steps listed in fields_at (1-based step numbers).
        """
        times = np.asarray(times, float)
        S = len(times) - 1
        if self.steps == 0:
            self.times = [float(times[0]), float(times[0])]
        out = dict(iters=[], err=[], resp=[], fields={})
        for s in range(1, S + 1):
            it, err = self.step(times[s], E[s - 1], G[s - 1],
                                iters=None if schedule is None else schedule[s - 1],
                                eig=None if eig is None else eig(s))
            out["iters"].append(it)
            out["err"].append(err)
            out["resp"].append(self.response())
            if s in fields_at:
                out["fields"][s] = {k: (to_f9(v) if v.ndim == 5 else v.copy())
                                    for k, v in self.cur.items()}
            self._commit(times[s])
        out["resp"] = np.array(out["resp"])
        return out

    def _commit(self, t_new):
        self.e_prev, self.g_prev = self.hist["e"], self.hist["g"]
        self.hist = {k: v.copy() for k, v in self.cur.items()}
        self.times = [self.times[1], float(t_new)]
        self.steps += 1


def fields9(st):
    """State dict of (..., 3, 3) tensors -> dict of (9, n2, n1, n0) arrays."""
    return {k: (to_f9(v) if v.ndim == 5 else v) for k, v in st.items()}
