"""Pins of the oracle's FFT use and reference-medium Green operator.

- numpy's rfftn / irfftn against a brute-force DFT on tiny grids, and
  against the DFT written out as one dense matrix per axis (its separable
  definition) on grids with axes of up to 256 points, the lengths the solver
  runs (the oracle uses them as its transform step);
- equilibrium: the stresses of the reference medium loaded by a polarization
  satisfy the balance laws (Eq. 2) -- checked with independent spectral
  derivatives and the sym/skew laws of Eq. 8;
- projection: an admissible (compatible) field is reproduced exactly;
- classical limit: with kappa0 = 0 and symmetric tau the symmetric strain is
  the textbook isotropic Moulinec-Suquet Green operator;
- closed form: a longitudinal / transverse split of the 6x6 symbol agrees
  with the dense per-frequency solve.
"""
import numpy as np
import pytest

from oracle import micropolar as O
from tests import helpers as H

REFS = [
    (3.0, 3.0, 0.3, 0.0, 12.0, 12.0),      # beta = gamma (singular skew couple modulus)
    (1.25, 1.25, 0.625, 0.0, 0.375, 1.25),  # two-phase mean of the manufactured-solution cell
    (2.0, 0.7, 1.3, 0.4, 0.2, 0.9),
]


def brute_dft(a):
    nz, ny, nx = a.shape
    out = np.zeros(a.shape, complex)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    for kz in range(nz):
        for ky in range(ny):
            for kx in range(nx):
                ph = np.exp(-2j * np.pi * (kz * z / nz + ky * y / ny + kx * x / nx))
                out[kz, ky, kx] = (a * ph).sum()
    return out


@pytest.mark.parametrize("shape", [(4, 4, 4), (3, 4, 6), (6, 6, 6), (8, 4, 2)])
def test_rfftn_matches_brute_force(shape):
    rng = np.random.default_rng(1)
    a = rng.standard_normal(shape)
    ref = brute_dft(a)
    got = np.fft.rfftn(a)
    assert np.abs(got - ref[..., : shape[2] // 2 + 1]).max() < 1e-12 * np.abs(ref).max()
    back = np.fft.irfftn(got, s=shape, axes=(0, 1, 2))
    assert np.abs(back - a).max() < 1e-13


def dft_matrix(n):
    k = np.arange(n)
    # exponent reduced mod n before the sin/cos, so the entries are exact to rounding
    return np.exp(-2j * np.pi * ((np.outer(k, k) % n) / n))


@pytest.mark.parametrize("shape", [(6, 8, 256), (256, 4, 6), (12, 192, 8), (24, 16, 96), (32, 32, 128)])
def test_rfftn_matches_axis_dft_matrices(shape):
    """rfftn(a) = F_z F_y F_x a with F_n[k, j] = exp(-2 pi i k j / n), on the
    half spectrum of the last axis; and irfftn inverts it."""
    rng = np.random.default_rng(2)
    a = rng.standard_normal(shape)
    nz, ny, nx = shape
    ref = np.einsum("kx,zyx->zyk", dft_matrix(nx)[: nx // 2 + 1], a)
    ref = np.einsum("ky,zyx->zkx", dft_matrix(ny), ref)
    ref = np.einsum("kz,zyx->kyx", dft_matrix(nz), ref)
    got = np.fft.rfftn(a)
    scale = np.abs(ref).max()
    assert np.abs(got - ref).max() < 1e-12 * scale
    back = np.fft.irfftn(got, s=shape, axes=(0, 1, 2))
    assert np.abs(back - a).max() < 1e-13 * np.abs(a).max() * max(shape)


def rand_fields(n, seed):
    rng = np.random.default_rng(seed)
    f = lambda: H.band_limit(rng.standard_normal((3, 3, n[2], n[1], n[0])))
    return f(), f()


@pytest.mark.parametrize("ref", REFS)
@pytest.mark.parametrize("n,h", [((8, 8, 8), 1.0), ((6, 4, 10), 0.3), ((5, 7, 6), 2.0)])
def test_green_output_is_equilibrated(ref, n, h):
    tau, mu = rand_fields(n, 3)
    G = O.GreenOperator(n, h, ref)
    e9, g9 = G.apply(tau.reshape(9, *tau.shape[2:]), mu.reshape(9, *mu.shape[2:]))
    e = e9.reshape(3, 3, *e9.shape[1:])
    g = g9.reshape(3, 3, *g9.shape[1:])
    lam, mu0, kap, alp, bet, gam = ref
    t = H.law_t(lam, mu0, kap, e) + tau
    m = H.law_m(alp, bet, gam, g) + mu
    # remove the uniform parts: the k = 0 balance is not imposed (means are prescribed)
    t -= t.mean(axis=(2, 3, 4), keepdims=True)
    ru, rp = H.balance(t, m, n, h)
    scale = np.abs(tau).max() / h + np.abs(mu).max() / h ** 2
    assert np.abs(ru).max() < 1e-12 * scale
    assert np.abs(rp).max() < 1e-12 * scale
    assert np.abs(e9.mean(axis=(1, 2, 3))).max() < 1e-14
    assert np.abs(g9.mean(axis=(1, 2, 3))).max() < 1e-14


@pytest.mark.parametrize("ref", REFS)
def test_green_reproduces_compatible_fields(ref):
    n, h = (8, 6, 4), 0.5
    rng = np.random.default_rng(7)
    u = H.band_limit(rng.standard_normal((3, n[2], n[1], n[0])))
    phi = H.band_limit(rng.standard_normal((3, n[2], n[1], n[0])))
    phi -= phi.mean(axis=(1, 2, 3), keepdims=True)
    # Eq. 1: e_kl = u_l,k + eps_lkm phi_m ; gamma_kl = phi_k,l
    e = np.zeros((3, 3) + u.shape[1:])
    g = np.zeros_like(e)
    for l in range(3):
        du = H.grad(u[l], n, h)
        for k in range(3):
            e[k, l] += du[k]
            for mm in range(3):
                e[k, l] += H.LC[l, k, mm] * phi[mm]
    for k in range(3):
        dphi = H.grad(phi[k], n, h)
        for l in range(3):
            g[k, l] = dphi[l]
    lam, mu0, kap, alp, bet, gam = ref
    tau = -H.law_t(lam, mu0, kap, e)
    mu = -H.law_m(alp, bet, gam, g)
    G = O.GreenOperator(n, h, ref)
    e9, g9 = G.apply(tau.reshape(9, *n[::-1]), mu.reshape(9, *n[::-1]))
    assert np.abs(e9 - e.reshape(9, *n[::-1])).max() < 1e-12 * np.abs(e).max()
    assert np.abs(g9 - g.reshape(9, *n[::-1])).max() < 1e-12 * np.abs(g).max()


def test_classical_limit_moulinec_suquet():
    lam, mu0 = 1.7, 0.9
    ref = (lam, mu0, 0.0, 0.0, 0.5, 0.8)
    n, h = (8, 8, 8), 1.0
    rng = np.random.default_rng(11)
    tau = rng.standard_normal((3, 3, 8, 8, 8))
    tau = H.band_limit(0.5 * (tau + np.swapaxes(tau, 0, 1)))
    G = O.GreenOperator(n, h, ref)
    e9, _ = G.apply(tau.reshape(9, 8, 8, 8), np.zeros((9, 8, 8, 8)))
    e = e9.reshape(3, 3, 8, 8, 8)
    esym = 0.5 * (e + np.swapaxes(e, 0, 1))
    # textbook isotropic operator: e_kh = -Gamma_khij tau_ij
    kz, ky, kx = H.wavenumbers(n, h)
    T = np.fft.fftn(tau, axes=(-3, -2, -1))
    X = np.stack(np.broadcast_arrays(kx[None, None, :], ky[None, :, None], kz[:, None, None]))
    s2 = (X ** 2).sum(0)
    s2s = np.where(s2 > 0, s2, 1.0)
    d = np.eye(3)
    out = np.zeros_like(T)
    for k in range(3):
        for hh in range(3):
            acc = 0
            for i in range(3):
                for j in range(3):
                    gam = (d[k, i] * X[hh] * X[j] + d[hh, i] * X[k] * X[j]
                           + d[k, j] * X[hh] * X[i] + d[hh, j] * X[k] * X[i]) / (4 * mu0 * s2s) \
                        - (lam + mu0) / (mu0 * (lam + 2 * mu0)) * X[i] * X[j] * X[k] * X[hh] / s2s ** 2
                    acc = acc + gam * T[i, j]
            out[k, hh] = -np.where(s2 > 0, acc, 0)
    ref_e = np.fft.ifftn(out, axes=(-3, -2, -1)).real
    assert np.abs(esym - ref_e).max() < 1e-12 * np.abs(ref_e).max()


def closed_form(xi, bu, bp, ref):
    """Longitudinal / transverse split of the 6x6 symbol (independent formula)."""
    lam, mu, kap, alp, bet, gam = ref
    s = np.linalg.norm(xi, axis=1)
    nn = xi / s[:, None]
    nbu = (nn * bu).sum(1)[:, None]
    nbp = (nn * bp).sum(1)[:, None]
    buT = bu - nn * nbu
    bpT = bp - nn * nbp
    a = (mu + kap) * s ** 2
    c = gam * s ** 2 + 4 * kap
    D = s ** 2 * ((mu + kap) * gam * s ** 2 + 4 * mu * kap)
    uT = (c[:, None] * buT + 2j * kap * s[:, None] * np.cross(nn, bpT)) / D[:, None]
    pT = (2j * kap * s[:, None] * np.cross(nn, buT) + a[:, None] * bpT) / D[:, None]
    uL = nn * nbu / ((lam + 2 * mu) * s ** 2)[:, None]
    pL = nn * nbp / ((alp + bet + gam) * s ** 2 + 4 * kap)[:, None]
    return uT + uL, pT + pL


@pytest.mark.parametrize("ref", REFS)
def test_dense_symbol_matches_closed_form(ref):
    rng = np.random.default_rng(5)
    xi = rng.standard_normal((64, 3)) * rng.uniform(0.1, 5.0, (64, 1))
    G = O.GreenOperator((4, 4, 4), 1.0, ref)
    M = G._symbol(xi)
    b = rng.standard_normal((64, 6)) + 1j * rng.standard_normal((64, 6))
    x = np.linalg.solve(M, b[..., None])[..., 0]
    # M is minus the closed-form K (the symbol maps amplitudes to residuals)
    u, p = closed_form(xi, -b[:, :3], -b[:, 3:], ref)
    assert np.abs(x[:, :3] - u).max() < 1e-12 * np.abs(u).max()
    assert np.abs(x[:, 3:] - p).max() < 1e-12 * np.abs(p).max()
    # Hermitian symbol
    assert np.abs(M - np.conj(np.swapaxes(M, 1, 2))).max() < 1e-13 * np.abs(M).max()
