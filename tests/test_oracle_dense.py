"""Brute-force pin of the oracle's whole Alg. 2 solve in the linear elastic
case: on a heterogeneous 4^3 micropolar cell, the converged fixed point of
the basic scheme equals the solution of the equilibrium equations (Eq. 2
with the Eq. 8 laws, no body force or couple) solved directly.

The direct solve is written from the balance laws, independently of the
oracle's Green operator and iteration: the unknowns are the Fourier
coefficients of the displacement and micro-rotation fluctuations at every
non-zero, non-Nyquist frequency (continuous frequencies 2 pi m / (N h)); the
strains are e_kl = E_kl + u_l,k + eps_lkm phi_m and gamma_kl = Gamma_kl +
phi_k,l; the residuals are the Fourier coefficients of t_kl,k and
m_kl,k + eps_lkm t_km at the same frequencies.  The residual is affine in
the unknowns; its matrix is assembled column by column and the system
solved with LAPACK.
"""
import numpy as np

from oracle import micropolar as O
from paper_2409_10774_amd import workloads as W
from tests import helpers as H

N, h = 4, 1.0


def modes():
    """Frequency indices (z, y, x) in {0, 1, N-1}^3 without the zero mode."""
    idx = [0, 1, N - 1]
    return [(a, b, c) for a in idx for b in idx for c in idx if (a, b, c) != (0, 0, 0)]


def xi_of(m):
    f = lambda i: 2 * np.pi * (i if i < N // 2 else i - N) / (N * h)
    return np.array([f(m[2]), f(m[1]), f(m[0])])          # (x1, x2, x3)


def fields(z, E, G, pm, phases):
    """Strain, curvature, stress, couple stress (3, 3, z, y, x) of unknowns z
    (per mode: u_1..3, phi_1..3)."""
    Eh = np.zeros((3, 3, N, N, N), complex)
    Gh = np.zeros((3, 3, N, N, N), complex)
    for j, m in enumerate(modes()):
        u, phi = z[6 * j: 6 * j + 3], z[6 * j + 3: 6 * j + 6]
        xi = xi_of(m)
        for k in range(3):
            for l in range(3):
                Eh[(k, l) + m] = 1j * xi[k] * u[l] + sum(H.LC[l, k, mm] * phi[mm] for mm in range(3))
                Gh[(k, l) + m] = 1j * xi[l] * phi[k]
    e = np.fft.ifftn(Eh, axes=(-3, -2, -1)) * N ** 3 + E[:, :, None, None, None]
    g = np.fft.ifftn(Gh, axes=(-3, -2, -1)) * N ** 3 + G[:, :, None, None, None]
    t = np.zeros_like(e)
    mc = np.zeros_like(g)
    for ph_id, p in enumerate(phases):
        sel = pm == ph_id
        t[:, :, sel] = H.law_t(p.lam, p.mu, p.kappa, e[:, :, sel])
        mc[:, :, sel] = H.law_m(p.alpha, p.beta, p.gamma, g[:, :, sel])
    return e, g, t, mc


def residual(z, E, G, pm, phases):
    _, _, t, mc = fields(z, E, G, pm, phases)
    th = np.fft.fftn(t, axes=(-3, -2, -1)) / N ** 3
    mh = np.fft.fftn(mc, axes=(-3, -2, -1)) / N ** 3
    r = []
    for m in modes():
        xi = xi_of(m)
        for l in range(3):
            r.append(sum(1j * xi[k] * th[(k, l) + m] for k in range(3)))
        for l in range(3):
            r.append(sum(1j * xi[k] * mh[(k, l) + m] for k in range(3))
                     + sum(H.LC[l, k, mm] * th[(k, mm) + m] for k in range(3) for mm in range(3)))
    return np.array(r)


def test_fixed_point_equals_dense_direct_solve():
    rng = np.random.default_rng(12)
    pm = (rng.random((N, N, N)) < 0.35).astype(np.uint8)
    mat = W.matrix_phase(kappa=0.4, length=1.0, tY=np.inf)   # linear elastic
    mat.beta = 0.6 * mat.gamma
    inc = mat.scaled_moduli(4.0)
    inc.beta = 0.3 * inc.gamma
    phases = [mat, inc]
    Ev = np.array([0.3, 0.1, -0.2, 0.05, -0.4, 0.2, 0.1, 0.0, 0.25]) * 1e-2
    Gv = np.array([0.0, 0.2, 0.1, -0.1, 0.05, 0.0, 0.3, -0.2, 0.1]) * 1e-2
    E, G = Ev.reshape(3, 3), Gv.reshape(3, 3)

    n = 6 * len(modes())
    r0 = residual(np.zeros(n, complex), E, G, pm, phases)
    M = np.empty((len(r0), n), complex)
    for j in range(n):
        z = np.zeros(n, complex)
        z[j] = 1.0
        M[:, j] = residual(z, E, G, pm, phases) - r0
    z = np.linalg.solve(M, -r0)
    e, g, t, mc = fields(z, E, G, pm, phases)
    assert np.abs(e.imag).max() < 1e-14 and np.abs(t.imag).max() < 1e-14

    out = O.Solver(pm, phases, h=h, tol=1e-13).solve(np.array([0.0, 1.0]), Ev[None], Gv[None],
                                                    fields_at=(1,))
    f = out["fields"][1]
    shape = (3, 3, N, N, N)
    for name, ref in (("e", e.real), ("g", g.real), ("t", t.real), ("m", mc.real)):
        got = f[name].reshape(shape)
        err = np.abs(got - ref).max() / np.abs(ref).max()
        assert err < 1e-10, (name, err)
