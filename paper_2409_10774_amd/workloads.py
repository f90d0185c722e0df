"""Seeded synthetic inputs: voxel phase maps, per-phase constants, load paths.

This module holds no arithmetic of the solver itself.  It only draws the
inputs that the paper's problem statement asks for (Alg. 2 inputs): a voxel
phase image, the isotropic constants of each phase (Eq. 6 moduli, Eqs. 13-18
plastic constants), and a macroscopic strain / curvature path E(t), Gamma(t).
Both the HIP path and the CPU oracle take their inputs from here.

Tensor components use the 9-vector index 3*k + l for V_kl (k = row).
Phase images are uint8 arrays of shape (n2, n1, n0) = (z, y, x): x fastest.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict

import numpy as np

INF = float("inf")

PHASE_KEYS = ("lam", "mu", "kappa", "alpha", "beta", "gamma",
              "tY", "tH", "mY", "mH", "a1", "b1")


@dataclass
class Phase:
    """Isotropic micropolar elastoplastic constants of one phase.

    Elastic moduli of Eq. 6 (lam, mu, kappa, alpha, beta, gamma); macro yield
    stress / hardening tY, tH (Eq. 15); micro yield / hardening mY, mH (Eq. 18);
    plastic weights a1, b1 (Eqs. 14, 17).  tY = mY = inf gives an elastic phase.
    """
    lam: float
    mu: float
    kappa: float
    alpha: float
    beta: float
    gamma: float
    tY: float = INF
    tH: float = 0.0
    mY: float = INF
    mH: float = 0.0
    a1: float = 1.5
    b1: float = 1.5
    # optional general elastic tensors of Eq. 5 (elastic phases only):
    # A[k, l, m, n] = A_klmn and B[l, k, m, n] = B_lkmn, so that
    # t_kl = A_klmn e_mn and m_kl = B_lkmn gamma_mn; the isotropic constants
    # above then serve the reference medium and the Eqs. 14, 17 weights
    A: "np.ndarray | None" = None
    B: "np.ndarray | None" = None

    def as_tuple(self):
        return tuple(float(getattr(self, k)) for k in PHASE_KEYS)

    def scaled_moduli(self, c: float, elastic: bool = True) -> "Phase":
        """Same phase with every elastic modulus multiplied by c."""
        p = Phase(**asdict(self))
        for k in ("lam", "mu", "kappa", "alpha", "beta", "gamma"):
            setattr(p, k, getattr(p, k) * c)
        if elastic:
            p.tY = p.mY = INF
            p.tH = p.mH = 0.0
        return p


def matrix_phase(lam=1.0, mu=1.0, kappa=0.1, length=2.0, h=1.0,
                 tY=0.005, tH=0.1, mY=None, mH=None, a1=1.5, b1=1.5) -> Phase:
    """Matrix of the sphere-inclusion workloads.

    beta = gamma = mu * l^2 with l given in voxels (times the voxel size h),
    alpha = 0; micro yield and hardening equal the macro ones unless given.
    """
    lg = length * h
    bg = mu * lg * lg
    return Phase(lam=lam, mu=mu, kappa=kappa, alpha=0.0, beta=bg, gamma=bg,
                 tY=tY, tH=tH, mY=tY if mY is None else mY,
                 mH=tH if mH is None else mH, a1=a1, b1=b1)


# ----------------------------------------------------------------------------
# microstructures
# ----------------------------------------------------------------------------

def _voxel_centres(n):
    """Continuous coordinates of voxel centres, h = 1, arrays shaped (z, y, x)."""
    z, y, x = np.meshgrid(np.arange(n[2]) + 0.5, np.arange(n[1]) + 0.5,
                          np.arange(n[0]) + 0.5, indexing="ij")
    return x, y, z


def _paint_sphere(phase, n, c, r, value):
    """Mark voxels whose centre lies within r of c (periodic minimum image).

    Only the sphere's bounding box is visited (indices wrapped periodically).
    """
    idx = []
    for ax, L in ((0, n[0]), (1, n[1]), (2, n[2])):
        lo = int(np.floor(c[ax] - r - 0.5)) - 1
        hi = int(np.ceil(c[ax] + r - 0.5)) + 1
        j = np.arange(lo, hi + 1)
        if len(j) >= L:
            j = np.arange(L)
        d = (np.mod(j, L) + 0.5) - c[ax]
        d -= L * np.round(d / L)
        idx.append((np.mod(j, L), d))
    (ix, dx), (iy, dy), (iz, dz) = idx
    d2 = dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2
    zz, yy, xx = np.nonzero(d2 <= r * r)
    phase[iz[zz], iy[yy], ix[xx]] = value


def centred_sphere(n: int, vf: float) -> np.ndarray:
    """One sphere at the cell centre with nominal volume fraction vf."""
    r = (3.0 * vf * n ** 3 / (4.0 * math.pi)) ** (1.0 / 3.0)
    ph = np.zeros((n, n, n), np.uint8)
    _paint_sphere(ph, (n, n, n), (n / 2.0, n / 2.0, n / 2.0), r, 1)
    return ph


def random_spheres(n: int, seed: int, count: int | None, rmin: float, rmax: float,
                   target_vf: float | None = None, max_tries: int = 200000):
    """Random sequential addition of non-overlapping periodic spheres.

    Radii ~ U[rmin, rmax], centres ~ U[0, n)^3; a candidate is kept when its
    periodic distance to every kept centre is at least the sum of the radii.
    Stops after `count` spheres, or once the painted volume fraction reaches
    target_vf.  Returns (phase image, list of (cx, cy, cz, r)).
    """
    rng = np.random.default_rng(seed)
    spheres = []
    centres = np.zeros((0, 3))
    radii = np.zeros(0)
    ph = np.zeros((n, n, n), np.uint8)
    painted = 0
    tries = 0
    while tries < max_tries:
        if count is not None and len(spheres) >= count:
            break
        if target_vf is not None and len(spheres) and painted >= target_vf * ph.size:
            break
        tries += 1
        r = rng.uniform(rmin, rmax)
        c = rng.uniform(0.0, n, size=3)
        if len(spheres):
            d = centres - c
            d -= n * np.round(d / n)
            if np.any(np.sqrt((d * d).sum(axis=1)) < r + radii):
                continue
        spheres.append((float(c[0]), float(c[1]), float(c[2]), float(r)))
        centres = np.vstack([centres, c])
        radii = np.append(radii, r)
        before = int(np.count_nonzero(ph))
        _paint_sphere(ph, (n, n, n), c, r, 1)
        painted += int(np.count_nonzero(ph)) - before if target_vf is not None else 0
    return ph, spheres


def laminate(n: int, axis: int = 0) -> np.ndarray:
    """Two-phase laminate, 50 % volume fraction, layers normal to `axis` (0 = x)."""
    ph = np.zeros((n, n, n), np.uint8)
    idx = [slice(None)] * 3
    idx[2 - axis] = slice(n // 2, n)
    ph[tuple(idx)] = 1
    return ph


# ----------------------------------------------------------------------------
# load paths
# ----------------------------------------------------------------------------

def ramp_path(n_steps: int, E_end=None, G_end=None, t_end: float = 1.0):
    """Linear ramp from the zero state: times[0] = 0, times[s] = s * t_end / S.

    Returns times (S+1,), E (S, 9), G (S, 9); E[s-1] is the target at times[s].
    """
    times = np.linspace(0.0, t_end, n_steps + 1)
    E_end = np.zeros(9) if E_end is None else np.asarray(E_end, float).reshape(9)
    G_end = np.zeros(9) if G_end is None else np.asarray(G_end, float).reshape(9)
    frac = times[1:] / t_end
    return times, frac[:, None] * E_end[None, :], frac[:, None] * G_end[None, :]


def unit(idx_kl, value=1.0):
    v = np.zeros(9)
    v[3 * idx_kl[0] + idx_kl[1]] = value
    return v


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    phase_map: np.ndarray            # (n2, n1, n0) uint8
    phases: list                     # list[Phase]
    times: np.ndarray                # (S+1,)
    E: np.ndarray                    # (S, 9)
    G: np.ndarray                    # (S, 9)
    tol: float
    h: float = 1.0
    err_norm: str = "local"          # Eq. 38 ("local") or Eq. 37 ("average")
    ref_mode: str = "phase_mean"
    info: dict = field(default_factory=dict)

    @property
    def n(self):
        s = self.phase_map.shape
        return (s[2], s[1], s[0])

    @property
    def voxels(self):
        return int(self.phase_map.size)


def single_sphere_16(contrast: float = 5.0) -> Workload:
    """16^3 cell, one centred elastic sphere (vf 0.2) in an elastoplastic matrix;
    uniaxial E11 ramped to 0.01 in 10 equal steps; tolerance 1e-8."""
    mat = matrix_phase()
    inc = mat.scaled_moduli(contrast)
    times, E, G = ramp_path(10, E_end=unit((0, 0), 0.01), t_end=10.0)
    return Workload("sphere16_fp64", centred_sphere(16, 0.2), [mat, inc], times, E, G,
                    tol=1e-8, info={"contrast": contrast})


def random_spheres_128(seed: int = 1, n_steps: int = 50) -> Workload:
    """128^3 cell, 40 random elastic spheres r ~ U[6, 12], contrast 10;
    E11 ramped to 0.02 with curvature Gamma12 ramped to 0.002 over 50 steps."""
    ph, sp = random_spheres(128, seed, 40, 6.0, 12.0)
    mat = matrix_phase()
    inc = mat.scaled_moduli(10.0)
    S = 50
    times, E, G = ramp_path(S, E_end=unit((0, 0), 0.02), G_end=unit((0, 1), 0.002),
                            t_end=float(S))
    times, E, G = times[: n_steps + 1], E[:n_steps], G[:n_steps]
    return Workload("spheres128_fp64", ph, [mat, inc], times, E, G, tol=1e-8,
                    info={"spheres": len(sp), "vf": float(ph.mean())})


def anisotropic_spheres_128(seed: int = 1, n_steps: int = 50) -> Workload:
    """The 128^3 cell of random_spheres_128 with Eq. 5 spheres: general
    tensors of mean eigenvalue 17 (A) and 50 (B), about those of the
    contrast-10 isotropic spheres, and the unweighted mean of the two phases'
    tensors as the reference medium; same load path and tolerance."""
    ph, sp = random_spheres(128, seed, 40, 6.0, 12.0)
    mat = matrix_phase()
    inc = anisotropic_phase(seed + 10, t_scale=17.0, m_scale=50.0)
    S = 50
    times, E, G = ramp_path(S, E_end=unit((0, 0), 0.02), G_end=unit((0, 1), 0.002),
                            t_end=float(S))
    times, E, G = times[: n_steps + 1], E[:n_steps], G[:n_steps]
    return Workload("aniso128_fp64", ph, [mat, inc], times, E, G, tol=1e-8,
                    ref_mode="tensor_phase_mean", info={"spheres": len(sp), "vf": float(ph.mean())})


def random_spheres_256(seed: int = 2, n_steps: int = 20) -> Workload:
    """256^3 cell, spheres r ~ U[5, 15] added until the volume fraction is
    at least 0.25, contrast 10; E11 ramped to 0.01 over 20 steps; tol 1e-6."""
    ph, sp = random_spheres(256, seed, None, 5.0, 15.0, target_vf=0.25)
    mat = matrix_phase()
    inc = mat.scaled_moduli(10.0)
    S = 20
    times, E, G = ramp_path(S, E_end=unit((0, 0), 0.01), t_end=float(S))
    times, E, G = times[: n_steps + 1], E[:n_steps], G[:n_steps]
    return Workload("spheres256_mixed", ph, [mat, inc], times, E, G, tol=1e-6,
                    info={"spheres": len(sp), "vf": float(ph.mean())})


def random_rve(seed: int, n: int, n_steps: int = 20) -> Workload:
    """One RVE of the many-RVE batch: 1-60 spheres r ~ U[n/20, n/10], contrast
    U[2, 20], l ~ U[0.5, 4] voxels, tY ~ U[0.003, 0.01]; random symmetric unit
    strain direction with norm ramped to 0.01; tol 1e-6."""
    rng = np.random.default_rng(seed)
    count = int(rng.integers(1, 61))
    contrast = float(rng.uniform(2.0, 20.0))
    length = float(rng.uniform(0.5, 4.0))
    tY = float(rng.uniform(0.003, 0.01))
    v = rng.standard_normal(6)
    sym = np.array([[v[0], v[5], v[4]], [v[5], v[1], v[3]], [v[4], v[3], v[2]]])
    sym /= np.linalg.norm(sym)
    ph, sp = random_spheres(n, int(rng.integers(0, 2**31)), count, n / 20.0, n / 10.0)
    mat = matrix_phase(length=length, tY=tY)
    inc = mat.scaled_moduli(contrast)
    times, E, G = ramp_path(n_steps, E_end=0.01 * sym.reshape(9), t_end=float(n_steps))
    return Workload(f"rve{n}_s{seed}", ph, [mat, inc], times, E, G, tol=1e-6,
                    info={"spheres": len(sp), "contrast": contrast, "l": length, "tY": tY})


def batch_rves(seed: int = 3, count: int = 64, sizes=(32, 64, 96, 128), n_steps: int = 20):
    """The many-RVE batch: `count` RVEs, edge drawn uniformly from `sizes`,
    each a random_rve of its own seed (mixed precision, tol 1e-6)."""
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.asarray(sizes), size=count)
    seeds = rng.integers(0, 2**31, size=count)
    return [random_rve(int(sd), int(n), n_steps) for sd, n in zip(seeds, ns)]


def serve_trace(seed: int = 4, n_req: int = 200, rate: float = 1.0,
                sizes=(32, 64, 128, 256), weights=(0.4, 0.3, 0.2, 0.1), steps=(10, 40)):
    """Poisson request trace: arrival times (s) with mean rate `rate` per
    second, and per request a random_rve of edge drawn from `sizes` with
    `weights` and a load path of U{steps[0]..steps[1]} steps.  Returns
    [(arrival, Workload)]."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n_req)
    arrivals = np.cumsum(gaps) - gaps[0]
    ns = rng.choice(np.asarray(sizes), size=n_req, p=np.asarray(weights) / np.sum(weights))
    st = rng.integers(steps[0], steps[1] + 1, size=n_req)
    seeds = rng.integers(0, 2**31, size=n_req)
    return [(float(a), random_rve(int(sd), int(n), int(k)))
            for a, n, k, sd in zip(arrivals, ns, st, seeds)]


def mnms_cube4():
    """4^3 cube used for manufactured solutions: inner centred 2^3 block is
    phase 0, the outer layer phase 1 (constants of the paper's code check)."""
    ph = np.ones((4, 4, 4), np.uint8)
    ph[1:3, 1:3, 1:3] = 0
    p1 = Phase(lam=1.0, mu=1.0, kappa=0.5, alpha=0.0, beta=0.5, gamma=1.0,
               tY=4.0, tH=0.0, mY=4.0, mH=0.0, a1=1.5, b1=1.5)
    p2 = Phase(lam=1.5, mu=1.5, kappa=0.75, alpha=0.0, beta=0.25, gamma=1.5,
               tY=4.5, tH=0.0, mY=4.5, mH=0.0, a1=1.5, b1=1.5)
    return ph, [p1, p2]


def ratchet_laminate(cycles: int = 10, dt: float = 0.01, rate: float = 1.0, tY: float = 2.5,
                     mH: float = 0.0025, mY: float = 0.005, tol: float = 1e-5) -> Workload:
    """Micro-plastic ratcheting cell of Sec. 3.2: a 4^3 laminate at 50 %
    volume fraction (layers normal to x2), unit cube (h = 1/4), the phase
    constants of Tab. 2, and `cycles` one-second shear cycles with
    dE12/dt = +rate for the first half of each cycle and -rate for the second
    (E12 from 0 up to rate / 2 and back), time step dt, all other strain and
    curvature components zero.  tY, mH and mY override Tab. 2's (tY = 1.9,
    mH = 0 is the variant of the second ratcheting study; mY = inf turns the
    micro level elastic)."""
    ph = laminate(4, axis=1)
    p1 = Phase(lam=1.0, mu=1.0, kappa=1.0, alpha=0.0, beta=1.0, gamma=2.0,
               tY=tY, tH=0.0, mY=mY, mH=mH, a1=1.5, b1=1.5)
    p2 = Phase(lam=2.0, mu=2.0, kappa=2.0, alpha=0.0, beta=2.0, gamma=4.0,
               tY=tY, tH=0.0, mY=mY, mH=mH, a1=1.5, b1=1.5)
    per = int(round(1.0 / dt))
    S = cycles * per
    times = dt * np.arange(S + 1)
    k = np.arange(1, S + 1) % per                   # steps into the current cycle
    E = np.zeros((S, 9))
    E[:, 1] = rate * dt * np.minimum(k, per - k)
    return Workload(f"ratchet_{cycles}c", ph, [p1, p2], times, E, np.zeros((S, 9)), tol=tol, h=0.25,
                    info=dict(cycles=cycles, dt=dt, tY=tY, mH=mH, mY=mY))


def anisotropic_phase(seed: int, t_scale: float = 4.0, m_scale: float = 2.0) -> Phase:
    """Elastic phase with general centrosymmetric tensors of Eq. 5: A_klmn
    and B_lkmn from random symmetric positive definite 9 x 9 matrices over
    the index pairs (kl, mn) and (lk, mn), mean eigenvalue t_scale and
    m_scale (eigenvalues within a factor of about 2).  Its isotropic constants
    (used for the reference medium and the Eqs. 14, 17 weights) bound the
    tensors from above: every eigenvalue of their Eq. 6 tensors equals the
    largest eigenvalue of A or B (lam = alpha = beta = 0, mu = kappa =
    max eig A / 2, gamma = max eig B), which keeps a phase-mean reference
    medium above half of every phase's stiffness."""
    rng = np.random.default_rng(seed)

    def spd(scale):
        R = rng.standard_normal((9, 9))
        M = 0.25 * (R @ R.T) / 9.0 + np.eye(9)
        return M * (9.0 * scale / np.trace(M))

    MA, MB = spd(t_scale), spd(m_scale)
    a_max, b_max = np.linalg.eigvalsh(MA).max(), np.linalg.eigvalsh(MB).max()
    return Phase(lam=0.0, mu=0.5 * a_max, kappa=0.5 * a_max, alpha=0.0, beta=0.0, gamma=b_max,
                 A=MA.reshape(3, 3, 3, 3), B=MB.reshape(3, 3, 3, 3))


def four_spheres_16(seed: int = 5, vf: float = 0.2) -> np.ndarray:
    """16^3 matrix (phase 0) with four equal non-overlapping periodic spheres
    (phase 1) of nominal total volume fraction vf, centres by random
    sequential addition (the length-scale cell of Sec. 3.3; the paper's
    sphere positions are not given)."""
    n = 16
    r = (3.0 * vf * n ** 3 / (4 * 4.0 * math.pi)) ** (1.0 / 3.0)
    ph, _ = random_spheres(n, seed, 4, r, r)
    return ph


def length_scale_rve(le: float, lp: float, seed: int = 5, n_steps: int = 100,
                     tol: float = 1e-5) -> Workload:
    """One cell of the Sec. 3.3 length-scale study: the constants of Tab. 3
    for elastic length le = sqrt(gamma / mu) and plastic length
    lp = sqrt(a / b) (gamma and b fixed; lambda = mu = kappa = gamma / le^2,
    beta = gamma / 2, a1 = b1 lp^2), matrix = phase 1 of the table, spheres
    = phase 2, on the unit cube (h = 1/16); monotone dE32/dt = 1 and
    dGamma11/dt = 1 over N steps of dt = 0.01."""
    def phase(gam, tY, tH):
        m = gam / le ** 2
        return Phase(lam=m, mu=m, kappa=m, alpha=0.0, beta=gam / 2.0, gamma=gam,
                     tY=tY, tH=tH, mY=tY, mH=tH, a1=1.5 * lp ** 2, b1=1.5)
    ph = four_spheres_16(seed)
    dt = 0.01
    times = dt * np.arange(n_steps + 1)
    E = np.zeros((n_steps, 9))
    G = np.zeros((n_steps, 9))
    E[:, 7] = times[1:]          # E32 (component 3k + l with k = 2, l = 1)
    G[:, 0] = times[1:]          # Gamma11
    return Workload(f"lscale_le{le:g}_lp{lp:g}", ph, [phase(1.0, 0.5, 0.125), phase(2.0, 0.75, 0.25)],
                    times, E, G, tol=tol, h=1.0 / 16, info=dict(le=le, lp=lp, seed=seed))


def random_state(nvox: int, seed: int, scale: float = 1e-2):
    """Random pointwise inputs for return-map checks: e, g, e_n, g_n, t_n, m_n
    as (9, nvox) arrays, p_n, q_n >= 0 as (nvox,)."""
    rng = np.random.default_rng(seed)
    f = lambda: scale * rng.standard_normal((9, nvox))
    return dict(e=f(), g=f(), e_n=f(), g_n=f(), t_n=f(), m_n=f(),
                p_n=np.abs(scale * rng.standard_normal(nvox)),
                q_n=np.abs(scale * rng.standard_normal(nvox)))
