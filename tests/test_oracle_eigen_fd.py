"""Pins of the eigen-channel equilibrium and of the polynomial Fermi-Dirac fit.

* Prop. 1: (rho, eps) fix (beta, nu_up, nu_dn); a round trip through the
  forward Fermi-Dirac formulas recovers the parameters.
* The equilibrium built through U and the Fermi-Dirac parameters
  (Eq. WeqDiscr) equals the direct form of Eq. WeqAlgo (Sec. 3.3 says U and
  F_k need not be computed).
* Sec. 3.2: the continuum moments of the polynomial equilibrium of
  Eq. WeqPoly equal those of the exact Fermi-Dirac function, checked by
  direct numerical integration at the parameters of Fig. 2.
* Sec. 3.2, discussion of Fig. 2: the deviation grows when beta0 overshoots
  the physical beta.  The figure carries no numbers and the paper states no
  pointwise bound, so only this ordering is asserted.
"""
import numpy as np
import pytest
from scipy import integrate, special

from oracle import constants, eigen, fermi, pauli, qlbm
from paper_1309_1656_amd import synthetic


@pytest.mark.parametrize("d", [2, 3])
def test_parameter_round_trip(d):
    beta = np.array([0.7, 1.0, 1.3, 0.95])
    nu_up = np.array([-2.1, -3.0, -0.6, -1.2])
    nu_dn = np.array([-2.9, -3.5, -1.4, -0.7])
    lam_up = fermi.channel_density(d, beta, nu_up)
    lam_dn = fermi.channel_density(d, beta, nu_dn)
    eps = fermi.internal_energy(d, beta, nu_up, nu_dn)
    b, u, dn = eigen.solve_parameters(d, lam_up, lam_dn, eps)
    assert np.max(np.abs(b / beta - 1)) < 1e-12
    assert np.max(np.abs(u - nu_up)) < 1e-11
    assert np.max(np.abs(dn - nu_dn)) < 1e-11


@pytest.mark.parametrize("d,shape", [(2, (4, 5)), (3, (3, 3, 4))])
def test_eigen_route_equals_direct(d, shape):
    lat = qlbm.Lattice(d)
    f = synthetic.macroscopic_fields(shape, 4)
    W = qlbm.init_equilibrium(lat, f["trrho"], f["r"], lat.xi * f["u_lat"], f["T"])
    rng = np.random.default_rng(2)
    a = rng.normal(0, 0.02, size=(4,) + W.shape[:-2]) * lat.w.reshape((1, -1) + (1,) * d)
    W = W + pauli.matrix_from_pauli(a)
    rho, T, u, eps = qlbm.moments(lat, W)
    direct = qlbm.equilibrium(lat, rho, u, eps)
    via_eigen = eigen.equilibrium_eigen(lat, W)
    assert np.max(np.abs(via_eigen - direct)) < 1e-12 * np.abs(direct).max()


def _wfd_diag(beta, mu, u, p):
    return special.expit(-beta * (0.5 * ((p - u) ** 2).sum(-1) - mu))


def _weq_poly(d, beta0, beta, mus, u):
    """Diagonal entries of Eq. WeqPoly with U = I, as a function of momenta p [..., d]."""
    al = {k: float(v) for k, v in constants.alpha_coefficients(d).items()}
    n = [fermi.channel_density(d, beta, np.array([beta * m]))[0] for m in mus]
    eps = fermi.internal_energy(d, beta, np.array([beta * mus[0]]), np.array([beta * mus[1]]))[0]
    b = beta0 * eps
    a1 = al["a1_0"] + al["a1_b"] * b
    a2 = al["a2_0"] + al["a2_b"] * b
    n0 = fermi.channel_density(d, beta0, np.array([0.0]))[0]

    def f(p):
        pu = (p * u).sum(-1)
        p2 = (p ** 2).sum(-1)
        P = a1 + a2 * beta0 * 0.5 * p2 + al["a3"] * beta0 * pu + al["a4"] * (beta0 * pu) ** 2 \
            + al["a5"] * beta0 * 0.5 * (u ** 2).sum()
        wgt = special.expit(-beta0 * 0.5 * p2) / n0
        return [wgt * nn * P for nn in n]
    return f


FIG2 = dict(beta=1.0, mus=(0.2, -0.35), u={2: np.array([0.2, 0.3]), 3: np.array([0.2, 0.3, -0.2])})


def _integrate(d, fn, center):
    """int fn(p) dp over R^d in polar / spherical coordinates about ``center``.

    The angular rule (trapezoid in phi, Gauss-Legendre in cos theta) is exact
    for the low-degree polynomials times radial functions integrated here; the
    radial integral is adaptive (scipy quad).
    """
    M = 32
    ph = 2 * np.pi * np.arange(M) / M
    if d == 2:
        dirs = np.stack([np.cos(ph), np.sin(ph)], -1)
        wts = np.full(M, 2 * np.pi / M)
        rpow = 1
    else:
        x, wx = np.polynomial.legendre.leggauss(16)
        st = np.sqrt(1 - x * x)
        dirs = np.stack([np.outer(st, np.cos(ph)), np.outer(st, np.sin(ph)),
                         np.outer(x, np.ones(M))], -1).reshape(-1, 3)
        wts = np.outer(wx, np.full(M, 2 * np.pi / M)).ravel()
        rpow = 2
    g = lambda r: r ** rpow * (wts * fn(center + r * dirs)).sum()
    return integrate.quad(g, 0, 40, epsabs=0, epsrel=1e-13, limit=400)[0]


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("beta0", [0.8, 1.2])
def test_polynomial_equilibrium_has_fd_moments(d, beta0):
    u = FIG2["u"][d]
    beta, mus = FIG2["beta"], FIG2["mus"]
    zero = np.zeros(d)
    tol = 1e-10
    weq = _weq_poly(d, beta0, beta, mus, u)
    for s in range(2):
        dens = _integrate(d, lambda p: weq(p)[s], zero)
        n_fd = _integrate(d, lambda p: _wfd_diag(beta, mus[s], u, p), u)
        assert abs(dens / n_fd - 1) < tol
    trW = lambda p: sum(weq(p))
    trF = lambda p: sum(_wfd_diag(beta, m, u, p) for m in mus)
    for a in range(d):
        mom = _integrate(d, lambda p: p[..., a] * trW(p), zero)
        mom_fd = _integrate(d, lambda p: p[..., a] * trF(p), u)
        assert abs(mom - mom_fd) < tol * max(1.0, abs(mom_fd))
    en = _integrate(d, lambda p: 0.5 * (p ** 2).sum(-1) * trW(p), zero)
    en_fd = _integrate(d, lambda p: 0.5 * (p ** 2).sum(-1) * trF(p), u)
    assert abs(en / en_fd - 1) < tol


@pytest.mark.parametrize("d", [2, 3])
def test_deviation_grows_when_beta0_overshoots(d):
    """Ordering only: sup over the p1 axis of |W_eq - W_FD| (the paper prints no values)."""
    u = FIG2["u"][d]
    p = np.zeros((801, d))
    p[:, 0] = np.linspace(-4, 4, 801)
    dev = {}
    for beta0 in (0.8, 1.2):
        weq = _weq_poly(d, beta0, FIG2["beta"], FIG2["mus"], u)(p)
        dev[beta0] = max(np.abs(weq[s] - _wfd_diag(FIG2["beta"], FIG2["mus"][s], u, p)).max() for s in range(2))
    assert dev[1.2] > dev[0.8]
