"""Test-side helpers written independently of the oracle and of the HIP path.

Spectral derivatives of band-limited periodic fields, the Levi-Civita symbol
built from permutation parity, and the isotropic laws in their sym/skew form
(Eq. 8) -- so that checks of the oracle do not reuse the oracle's own code.
"""
import itertools

import numpy as np


def levi_civita():
    e = np.zeros((3, 3, 3))
    for perm in itertools.permutations(range(3)):
        inv = sum(1 for i in range(3) for j in range(i + 1, 3) if perm[i] > perm[j])
        e[perm] = -1.0 if inv % 2 else 1.0
    return e


LC = levi_civita()


def wavenumbers(n, h):
    """Angular wavenumbers per array axis (z, y, x) with Nyquist set to 0."""
    out = []
    for L in (n[2], n[1], n[0]):
        m = np.fft.fftfreq(L) * L
        if L % 2 == 0:
            m[L // 2] = 0.0
        out.append(2 * np.pi * m / (L * h))
    return out


def band_limit(f):
    """Remove every Fourier mode at a Nyquist index of an even axis."""
    F = np.fft.fftn(f, axes=(-3, -2, -1))
    for ax in (-3, -2, -1):
        L = f.shape[ax]
        if L % 2 == 0:
            idx = [slice(None)] * F.ndim
            idx[ax] = L // 2
            F[tuple(idx)] = 0
    return np.fft.ifftn(F, axes=(-3, -2, -1)).real


def grad(f, n, h):
    """d f / d x_k for k = 1, 2, 3 of a periodic field shaped (..., z, y, x).

    Returns an array with a new leading axis k."""
    kz, ky, kx = wavenumbers(n, h)
    F = np.fft.fftn(f, axes=(-3, -2, -1))
    dx = np.fft.ifftn(1j * kx[None, None, :] * F, axes=(-3, -2, -1)).real
    dy = np.fft.ifftn(1j * ky[None, :, None] * F, axes=(-3, -2, -1)).real
    dz = np.fft.ifftn(1j * kz[:, None, None] * F, axes=(-3, -2, -1)).real
    return np.stack([dx, dy, dz])


def law_t(lam, mu, kappa, e):
    """Eq. 8 with e shaped (3, 3, ...): t = lam tr e I + 2 mu e_(kl) + 2 kappa e_[kl]."""
    eT = np.swapaxes(e, 0, 1)
    tr = e[0, 0] + e[1, 1] + e[2, 2]
    t = (mu + kappa) * e + (mu - kappa) * eT
    for k in range(3):
        t[k, k] = t[k, k] + lam * tr
    return t


def law_m(alpha, beta, gamma, g):
    """Eq. 8: m = alpha tr g I + (beta + gamma) g_(kl) + (beta - gamma) g_[kl]."""
    gT = np.swapaxes(g, 0, 1)
    tr = g[0, 0] + g[1, 1] + g[2, 2]
    m = beta * g + gamma * gT
    for k in range(3):
        m[k, k] = m[k, k] + alpha * tr
    return m


def balance(t, m, n, h):
    """Residuals of Eq. 2 (no body force / couple) for fields (3, 3, z, y, x):
    r_u_l = t_kl,k ;  r_phi_l = m_kl,k + eps_lkm t_km."""
    ru = np.zeros((3,) + t.shape[2:])
    rp = np.zeros((3,) + t.shape[2:])
    for l in range(3):
        for k in range(3):
            ru[l] += grad(t[k, l], n, h)[k]
            rp[l] += grad(m[k, l], n, h)[k]
            for mm in range(3):
                rp[l] += LC[l, k, mm] * t[k, mm]
    return ru, rp
