"""Pins of the oracle's lattice constants, weights and Appendix coefficients.

Each check compares the oracle with something other than its own formula:
decimals printed in the paper, the general-mu cubature formulas, direct
numerical integration of the Fermi-Dirac weight, and the exact discrete
conservation that the Appendix coefficients must produce (Sec. 3.3).
"""
import itertools
import os

import mpmath as mp
import numpy as np
import pytest
from scipy import integrate, special

from oracle import constants, lattice, qlbm

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "printed_constants.txt")


def _printed():
    out = {}
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            name, val = line.split()[:2]
            out[name] = val
    return out


def _matches_printed(value, printed):
    decimals = len(printed.split(".")[1])
    return abs(float(value) - float(printed)) <= 0.5 * 10.0 ** (-decimals) + 1e-15


def test_printed_decimals():
    p = _printed()
    a2, xi2 = constants.cubature_mu0(2, 1)
    a3, xi3 = constants.cubature_mu0(3, 1)
    assert _matches_printed(a2, p["a_d2"])
    assert _matches_printed(xi2, p["xi_sqrt_beta_d2"])
    assert _matches_printed(a3, p["a_d3"])
    assert _matches_printed(xi3, p["xi_sqrt_beta_d3"])
    assert _matches_printed(constants.alpha_coefficients(2)["fac"], p["alpha_fac_d2"])
    assert _matches_printed(constants.alpha_coefficients(3)["fac"], p["alpha_fac_d3"])
    assert _matches_printed(qlbm.Lattice(2, 1.0).xi, p["xi_beta0_1_d2"])


def test_xi_scales_with_beta0():
    for d in (2, 3):
        _, x1 = constants.cubature_mu0(d, 1)
        _, x = constants.cubature_mu0(d, mp.mpf("0.7"))
        assert abs(x * mp.sqrt(mp.mpf("0.7")) - x1) < mp.mpf(10) ** -30


@pytest.mark.parametrize("d", [2, 3])
def test_general_mu_forms_reduce_to_mu0(d):
    for beta in (mp.mpf(1), mp.mpf("0.8"), mp.mpf("1.3")):
        a, xi = constants.cubature_general(d, beta, 0)
        a0, xi0 = constants.cubature_mu0(d, beta)
        assert abs(a - a0) < mp.mpf(10) ** -25
        assert abs(xi - xi0) < mp.mpf(10) ** -25


@pytest.mark.parametrize("d", [2, 3])
def test_velocity_set_definition(d):
    c = lattice.velocities(d)
    expect = {v for v in itertools.product((-1, 0, 1), repeat=d)
              if d == 2 or sum(abs(t) for t in v) <= 2}
    got = {tuple(int(t) for t in v) for v in c}
    assert got == expect and len(c) == len(expect)
    opp = lattice.opposite(c)
    assert opp[0] == 0
    for i in range(1, len(c)):
        assert opp[i] == (i + 1 if i % 2 == 1 else i - 1)


@pytest.mark.parametrize("d", [2, 3])
def test_weights_sum_to_one(d):
    lat = qlbm.Lattice(d)
    assert abs(lat.w.sum() - 1.0) < 1e-15
    assert (lat.w > 0).all()


def _fd_weight_moment(d, beta0, m):
    """(1/n) int p^m f(p) dp for a monomial exponent tuple m, f the mu=0 FD weight.

    Radial and angular parts are integrated numerically (scipy) and separately.
    """
    f = lambda r: special.expit(-beta0 * r * r / 2.0)
    deg = sum(m)
    rad = lambda k: integrate.quad(lambda r: r ** k * f(r), 0, 60, epsabs=0, epsrel=1e-13, limit=200)[0]
    if d == 2:
        ang = integrate.quad(lambda t: np.cos(t) ** m[0] * np.sin(t) ** m[1], 0, 2 * np.pi,
                             epsabs=1e-15, epsrel=1e-13, limit=200)[0]
        return rad(deg + 1) * ang / (rad(1) * 2 * np.pi)
    ang = integrate.dblquad(lambda ph, t: np.sin(t) * (np.sin(t) * np.cos(ph)) ** m[0]
                            * (np.sin(t) * np.sin(ph)) ** m[1] * np.cos(t) ** m[2],
                            0, np.pi, 0, 2 * np.pi, epsabs=1e-15, epsrel=1e-13)[0]
    return rad(deg + 2) * ang / (rad(2) * 4 * np.pi)


@pytest.mark.parametrize("d", [2, 3])
def test_cubature_degree_five(d):
    """Sec. 3.1: exact for every monomial of degree <= 5, not for all of degree 6."""
    k = constants.as_float(d, 1.0)
    xi, w = k["xi"], k["class_w"]
    c = lattice.velocities(d)
    cls = lattice.velocity_class(c)

    def cub(m):
        return sum(w[q] * np.prod([(xi * float(ci[a])) ** m[a] for a in range(d)])
                   for ci, q in zip(c, cls))

    worst6 = 0.0
    for m in itertools.product(range(7), repeat=d):
        deg = sum(m)
        if deg > 6:
            continue
        if any(e % 2 for e in m):
            assert abs(cub(m)) < 1e-14  # odd moments vanish on both sides
            continue
        exact = _fd_weight_moment(d, 1.0, m)
        err = abs(cub(m) - exact)
        if deg <= 5:
            assert err < 1e-11 * max(1.0, abs(exact)), (m, err)
        else:
            worst6 = max(worst6, err)
    assert worst6 > 1e-3


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("beta0", [0.8, 1.0, 1.2])
def test_appendix_coefficients_conserve(d, beta0):
    """The Appendix coefficients make W_eq's discrete moments exact (Sec. 3.3):

    sum_i w_i P_i = 1, sum_i w_i e_i P_i = u, sum_i w_i |e_i|^2/2 P_i = eps + |u|^2/2,
    for any u and eps.  Five conditions that fix all five coefficients.
    """
    lat = qlbm.Lattice(d, beta0)
    rng = np.random.default_rng(7)
    for _ in range(5):
        u = rng.normal(0, 0.3, size=(d, 1)) * lat.xi
        eps = np.array([rng.uniform(0.5, 2.5)])
        P = qlbm.poly_factor(lat, u, eps)[:, 0]
        wP = lat.w * P
        assert abs(wP.sum() - 1.0) < 1e-13
        assert np.allclose(lat.e.T @ wP, u[:, 0], rtol=0, atol=1e-13)
        e2 = 0.5 * (lat.e ** 2).sum(axis=1)
        assert abs(e2 @ wP - (eps[0] + 0.5 * (u[:, 0] ** 2).sum())) < 1e-13
