"""Pins of the oracle's general reference medium (Alg. 2 with every phase's
own tensors: A0 = <A(x)>, B0 = <B(x)>, anisotropic when an Eq. 5 phase is
present).

- equilibrium: loaded by a polarization, the stresses of an anisotropic
  reference medium satisfy Eq. 2 (independent spectral derivatives, the
  Eq. 5 law with its index sums written out);
- projection: a compatible field (Eq. 1) is reproduced exactly;
- the tensor means of isotropic phases (volume and unweighted) are the
  Eq. 6 tensors of the averaged constants, built here by applying the Eq. 8
  laws to unit strains;
- the converged fields of the scheme do not depend on the reference medium
  (its fixed point is the equilibrium of the cell): an anisotropic tensor
  mean and an isotropic reference give the same solution within the
  tolerance.
"""
import numpy as np
import pytest

from oracle import micropolar as O
from paper_2409_10774_amd import workloads as W
from tests import helpers as H
from tests.test_oracle_aniso import law5_m, law5_t


def aniso_pair(seed):
    ph = W.anisotropic_phase(seed, t_scale=2.0, m_scale=1.5)
    return ph.A, ph.B


def eq6_tensors(lam, mu, kappa, alpha, beta, gamma):
    A = np.zeros((3, 3, 3, 3))
    B = np.zeros((3, 3, 3, 3))
    for mm in range(3):
        for nn in range(3):
            u = np.zeros((3, 3))
            u[mm, nn] = 1.0
            A[:, :, mm, nn] = H.law_t(lam, mu, kappa, u)
            B[:, :, mm, nn] = H.law_m(alpha, beta, gamma, u).T   # index order (l, k)
    return A, B


@pytest.mark.parametrize("n,h", [((8, 8, 8), 1.0), ((6, 4, 10), 0.3)])
@pytest.mark.parametrize("seed", [2, 9])
def test_general_reference_green_is_equilibrated(n, h, seed):
    A0, B0 = aniso_pair(seed)
    rng = np.random.default_rng(seed)
    f = lambda: H.band_limit(rng.standard_normal((3, 3, n[2], n[1], n[0])))
    tau, mu = f(), f()
    G = O.GreenOperator(n, h, (A0, B0))
    e9, g9 = G.apply(tau.reshape(9, *tau.shape[2:]), mu.reshape(9, *mu.shape[2:]))
    e = e9.reshape(3, 3, *e9.shape[1:])
    g = g9.reshape(3, 3, *g9.shape[1:])
    t = law5_t(A0, e) + tau
    m = law5_m(B0, g) + mu
    t -= t.mean(axis=(2, 3, 4), keepdims=True)
    ru, rp = H.balance(t, m, n, h)
    scale = np.abs(tau).max() / h + np.abs(mu).max() / h ** 2
    assert np.abs(ru).max() < 1e-12 * scale
    assert np.abs(rp).max() < 1e-12 * scale
    assert np.abs(e9.mean(axis=(1, 2, 3))).max() < 1e-14
    assert np.abs(g9.mean(axis=(1, 2, 3))).max() < 1e-14


def test_general_reference_reproduces_compatible_fields():
    n, h = (8, 6, 4), 0.5
    A0, B0 = aniso_pair(4)
    rng = np.random.default_rng(5)
    u = H.band_limit(rng.standard_normal((3, n[2], n[1], n[0])))
    phi = H.band_limit(rng.standard_normal((3, n[2], n[1], n[0])))
    phi -= phi.mean(axis=(1, 2, 3), keepdims=True)
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
    G = O.GreenOperator(n, h, (A0, B0))
    e9, g9 = G.apply(-law5_t(A0, e).reshape(9, *n[::-1]), -law5_m(B0, g).reshape(9, *n[::-1]))
    assert np.abs(e9 - e.reshape(9, *n[::-1])).max() < 1e-12 * np.abs(e).max()
    assert np.abs(g9 - g.reshape(9, *n[::-1])).max() < 1e-12 * np.abs(g).max()


def test_tensor_mean_of_isotropic_phases():
    pm = W.centred_sphere(6, 0.25)
    mat = W.matrix_phase(tY=0.004)
    mat.beta = 0.8 * mat.gamma
    inc = mat.scaled_moduli(3.0)
    A0, B0 = O.reference_tensors(pm, [mat, inc])
    f = np.count_nonzero(pm == 1) / pm.size
    keys = ("lam", "mu", "kappa", "alpha", "beta", "gamma")
    mean = [(1 - f) * getattr(mat, k) + f * getattr(inc, k) for k in keys]
    A, B = eq6_tensors(*mean)
    assert np.abs(A0 - A).max() < 1e-14 * np.abs(A).max()
    assert np.abs(B0 - B).max() < 1e-14 * np.abs(B).max()
    # unweighted over the two phases present
    Ap, Bp = O.reference_tensors(pm, [mat, inc], weights="phase")
    A2, B2 = eq6_tensors(*[0.5 * (getattr(mat, k) + getattr(inc, k)) for k in keys])
    assert np.abs(Ap - A2).max() < 1e-14 * np.abs(A2).max()
    assert np.abs(Bp - B2).max() < 1e-14 * np.abs(B2).max()
    # and the isotropic operator of those constants is the same operator
    rng = np.random.default_rng(1)
    n = (6, 6, 6)
    tau, mu = rng.standard_normal((2, 9) + n)
    a = O.GreenOperator(n, 1.0, tuple(mean)).apply(tau, mu)
    b = O.GreenOperator(n, 1.0, (A0, B0)).apply(tau, mu)
    for x, y in zip(a, b):
        assert np.abs(x - y).max() < 1e-12 * np.abs(x).max()


@pytest.mark.parametrize("mode", ["tensor_mean", "tensor_phase_mean"])
def test_fixed_point_does_not_depend_on_the_reference(mode):
    pm = W.centred_sphere(6, 0.2)
    mat = W.matrix_phase(kappa=0.5, tY=0.004)
    inc = W.anisotropic_phase(5, t_scale=3.0, m_scale=4.0)
    times, E, G = W.ramp_path(2, E_end=W.unit((0, 0), 0.01) + W.unit((1, 2), 0.004),
                              G_end=W.unit((0, 1), 0.002))
    tol = 1e-11
    a = O.Solver(pm, [mat, inc], tol=tol, ref_mode=mode).solve(times, E, G, fields_at=(2,))
    b = O.Solver(pm, [mat, inc], tol=tol).solve(times, E, G, fields_at=(2,))
    assert a["fields"][2]["p"].max() > 0
    for k in ("e", "g", "t", "m", "p", "q"):
        x, y = a["fields"][2][k], b["fields"][2][k]
        assert np.abs(x - y).max() <= 1e-9 * np.abs(y).max(), k
    # the tensor mean is the closer reference: fewer iterations
    assert sum(a["iters"]) < sum(b["iters"]), (a["iters"], b["iters"])
