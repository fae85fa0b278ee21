"""Pins of the oracle's screened kernel, G = exp(-kappa r) / (4 pi r).

The paper builds its method on interpolation of an asymptotically smooth
kernel (Sec. 1, Sec. 2) and uses Helmholtz as the oscillatory case; the
screened kernel is the non-oscillatory case, on low-frequency expansions
only.  Each test checks the oracle against something other than itself: the
spherical-mean closed forms of the two kernels, the Hermitian symmetry that a
real kernel forces on its spectrum, brute force on node grids, and geometric
convergence in L against the direct sum.
"""
import numpy as np
import pytest

import oracle
from paper_2202_04894_amd import workloads as W


def _sphere_quadrature(R, n_theta=48, n_phi=96):
    """Gauss-Legendre in cos(theta) times the trapezoid rule in phi on the sphere
    |y| = R; the weights sum to 1, so sum_j w_j f(y_j) is the mean of f."""
    t, wt = np.polynomial.legendre.leggauss(n_theta)
    phi = 2 * np.pi * (np.arange(n_phi) + 0.5) / n_phi
    st = np.sqrt(1 - t ** 2)
    Y = np.stack([np.outer(st, np.cos(phi)), np.outer(st, np.sin(phi)), np.outer(t, np.ones(n_phi))], -1)
    w = np.outer(wt / 2.0, np.full(n_phi, 1.0 / n_phi))
    return R * Y.reshape(-1, 3), w.reshape(-1)


@pytest.mark.parametrize("mu", [0.0, 3.0, 11.0])
def test_screened_direct_sum_spherical_mean(mu):
    """The mean of G(x - y) over the sphere |y| = R solves (Delta - mu^2) u = 0 off
    the sphere and is radial, so it is sinh(mu s)/(mu s) * G(R) for s = |x| < R and
    sinh(mu R)/(mu R) * G(|x|) for |x| > R (mu = 0: the Laplace mean value)."""
    R = 1.3
    Y, w = _sphere_quadrature(R)
    dirs = np.array([[0.36, -0.48, 0.8], [-0.6, 0.0, -0.8]])
    s = np.array([0.2, 0.55, 2.4, 3.1])
    X = np.concatenate([si * dirs for si in s])
    p = oracle.direct_sum(X, Y, w.astype(complex), mu, 1e-12, kernel=oracle.YUKAWA)
    G = lambda r: np.exp(-mu * r) / (4 * np.pi * r)
    shc = lambda z: np.sinh(z) / z if z > 0 else 1.0
    ref = []
    for si in s:
        v = shc(mu * si) * G(R) if si < R else shc(mu * R) * G(si)
        ref += [v, v]
    np.testing.assert_allclose(p.real, ref, rtol=1e-12, atol=0)
    assert np.abs(p.imag).max() == 0.0


def test_helmholtz_direct_sum_spherical_mean():
    """The oscillatory counterpart, pinning the sign of the phase: the mean of
    exp(i k |x - y|)/(4 pi |x - y|) over |y| = R is sin(k s)/(k s) * G(R) inside."""
    k, R = 7.0, 1.0
    Y, w = _sphere_quadrature(R, 64, 128)
    x = np.array([[0.12, 0.3, -0.24]])
    sx = np.linalg.norm(x)
    p = oracle.direct_sum(x, Y, w.astype(complex), k, 1e-12)
    ref = np.sin(k * sx) / (k * sx) * np.exp(1j * k * R) / (4 * np.pi * R)
    assert abs(p[0] - ref) <= 1e-12 * abs(ref)


@pytest.mark.parametrize("L", [3, 4, 5])
def test_screened_spectrum_hermitian_and_m2l_forms_agree(L):
    """A real kernel gives a real circulant column, hence D[-xi] = conj(D[xi]);
    the circulant M2L equals the dense one (eqs. FactorizedM2LMatrix1 /
    FourierDiagonal); the dense one is the kernel between node grids."""
    P, h, mu = 2 * L - 1, 0.4, 6.0
    rng = np.random.default_rng(L)
    for delta in [(2, 0, 0), (-3, 2, 1), (0, 4, -4)]:
        D = oracle.spectrum(mu, h, L, delta, kernel=oracle.YUKAWA)
        Dm = D[(-np.arange(P)) % P][:, (-np.arange(P)) % P][:, :, (-np.arange(P)) % P]
        assert np.abs(Dm - np.conj(D)).max() <= 1e-14 * np.abs(D).max()
        Dh = oracle.spectrum(mu, h, L, delta)  # the Helmholtz spectrum is not Hermitian
        Dhm = Dh[(-np.arange(P)) % P][:, (-np.arange(P)) % P][:, :, (-np.arange(P)) % P]
        assert np.abs(Dhm - np.conj(Dh)).max() > 1e-3 * np.abs(Dh).max()
        M = rng.standard_normal(L ** 3) + 1j * rng.standard_normal(L ** 3)
        a = oracle.m2l_fft(mu, h, L, delta, M, kernel=oracle.YUKAWA)
        b = oracle.m2l_dense(mu, h, L, delta, M, kernel=oracle.YUKAWA)
        assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(b)
        g = np.arange(L) / (L - 1)
        nodes = np.array([[g[i], g[j], g[k]] for k in range(L) for j in range(L) for i in range(L)])
        ys = h * nodes
        xt = h * np.asarray(delta) + h * nodes
        ref = oracle.direct_sum(xt, ys, M, mu, 1e-12, kernel=oracle.YUKAWA)
        np.testing.assert_allclose(b, ref, rtol=1e-13)


def _fmm_error(X, q, mu, prm, tg):
    F = oracle.FMM(X, None, mu, prm)
    p = F.apply(q)
    D, _ = F.geometry()
    pd = oracle.direct_sum(X, X, q, mu, 1e-12 * D, tg, kernel=oracle.YUKAWA)
    return np.linalg.norm(p[tg] - pd) / np.linalg.norm(pd), F


@pytest.mark.parametrize("geom,mu", [("sphere", 20.0), ("cube_volume", 20.0)])
def test_screened_fmm_low_frequency_and_geometric_convergence(geom, mu):
    """Thm. 1 carried to the screened kernel: on low-frequency expansions only
    (no level is high-frequency, whatever mu D) the relative error against the
    direct sum decreases geometrically in L."""
    n = 4000
    X = W.GENERATORS[geom](n, 71)
    q = W.charges(n, 72)
    tg = W.sample_targets(n, 300, 73)
    errs = []
    for L in range(2, 8):
        e, F = _fmm_error(X, q, mu, oracle.Params(L=L, ncrit=32, kernel=oracle.YUKAWA), tg)
        info = F.info()
        assert info["lstar"] == -1 and info["m2l_pairs"] > 0
        errs.append(e)
    errs = np.array(errs)
    assert (errs[1:] < errs[:-1]).all()
    assert errs[-1] < 1e-5
    assert (errs[-1] / errs[0]) ** (1.0 / (len(errs) - 1)) < 0.35
    # the Helmholtz kernel at the same kappa D would need directional levels
    assert oracle.FMM(X, None, mu, oracle.Params(L=4, ncrit=32)).info()["lstar"] >= 0


def test_screened_at_zero_is_laplace():
    """kappa = 0: the screened and the Helmholtz kernels are both 1/(4 pi r), and the
    two oracle runs build the same lists and give the same potentials."""
    n = 2500
    X = W.sphere(n, 81)
    q = W.charges(n, 82)
    a = oracle.FMM(X, None, 0.0, oracle.Params(L=4, ncrit=24, kernel=oracle.YUKAWA))
    b = oracle.FMM(X, None, 0.0, oracle.Params(L=4, ncrit=24))
    assert a.info() == b.info()
    pa, pb = a.apply(q), b.apply(q)
    assert np.linalg.norm(pa - pb) <= 1e-15 * np.linalg.norm(pb)
