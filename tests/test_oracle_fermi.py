"""Pins of the oracle's Fermi-Dirac integrals and their inversion (Sec. 2.2).

References used: mpmath's polylogarithm (F_k(x) = -Li_{k+1}(-e^x)), the
closed forms F_{-1}(x) = 1/(1 + e^-x) and F_0(x) = log(1 + e^x), the relation
dF_k/dx = F_{k-1}, F_k(0) = eta(k+1) (Dirichlet eta), and direct numerical
integration of the Fermi-Dirac distribution over momentum space for the
density and energy formulas (Eqs. rhoFDstdOmega, nFDstdOmega,
energyFDstdOmega).
"""
import mpmath as mp
import numpy as np
import pytest
from scipy import integrate, special

from oracle import fermi

KS = [-1.0, -0.5, 0.0, 0.5, 1.0, 1.5, 2.0, 2.5]


@pytest.mark.parametrize("k", KS)
def test_series_against_polylog(k):
    xs = np.linspace(-8.0, -0.5, 31)
    got = fermi.fd(k, xs)
    ref = np.array([float(mp.re(-mp.polylog(k + 1, -mp.exp(mp.mpf(x))))) for x in xs])
    assert np.max(np.abs(got / ref - 1.0)) < 2e-15


def test_closed_forms():
    xs = np.linspace(-7.0, -0.5, 27)
    assert np.allclose(fermi.fd(-1.0, xs), 1.0 / (1.0 + np.exp(-xs)), rtol=2e-15, atol=0)
    assert np.allclose(fermi.fd(0.0, xs), np.log1p(np.exp(xs)), rtol=2e-15, atol=0)


@pytest.mark.parametrize("k", [0.5, 1.5, 2.5, 1.0])
def test_derivative_relation(k):
    xs = np.array([-6.0, -3.0, -1.5, -0.8])
    h = 1e-5
    num = (fermi.fd(k, xs + h) - fermi.fd(k, xs - h)) / (2 * h)
    assert np.allclose(num, fermi.fd(k - 1.0, xs), rtol=1e-9, atol=0)


@pytest.mark.parametrize("k", [0.5, 1.5, 2.5, 1.0, 2.0])
def test_value_at_zero_is_eta(k):
    s = k + 1.0
    eta = float((1 - mp.mpf(2) ** (1 - s)) * mp.zeta(s))
    assert abs(fermi.fd(k, np.array([0.0]))[0] / eta - 1.0) < 1e-14


@pytest.mark.parametrize("k", [0.5, 0.0, -0.5])
def test_inversion_round_trip(k):
    nu = np.array([-5.0, -3.7, -2.2, -1.1, -0.6, 0.3, 1.7])
    c = fermi.fd(k, nu)
    back = fermi.invert_density(k, c)
    assert np.max(np.abs(back - nu)) < 1e-13


def test_two_dimensional_closed_form_inverse():
    # d = 2: n = (2 pi / beta) F_0(nu) = (2 pi / beta) log(1 + e^nu)  =>  nu = log(expm1(n beta / 2 pi))
    beta = np.array([0.9, 1.0, 1.1])
    n = np.array([0.31, 0.45, 0.66])
    nu = fermi.chemical_potential_scaled(2, beta, n)
    assert np.allclose(nu, np.log(np.expm1(n * beta / (2 * np.pi))), rtol=0, atol=1e-14)


def _fd_occupation(beta, mu, r):
    return special.expit(-beta * (0.5 * r * r - mu))


@pytest.mark.parametrize("d", [2, 3])
def test_density_and_energy_formulas_by_integration(d):
    """Eqs. nFDstdOmega and energyFDstdOmega against direct radial integration."""
    surface = 2 * np.pi if d == 2 else 4 * np.pi
    for beta, mu_up, mu_dn in [(1.0, 0.2, -0.35), (0.8, -2.0, -3.0), (1.3, -1.5, -2.5)]:
        dens = []
        energy = 0.0
        for mu in (mu_up, mu_dn):
            n = surface * integrate.quad(lambda r: r ** (d - 1) * _fd_occupation(beta, mu, r),
                                         0, 60, epsabs=0, epsrel=1e-13, limit=200)[0]
            dens.append(n)
            energy += surface * integrate.quad(lambda r: 0.5 * r * r * r ** (d - 1) * _fd_occupation(beta, mu, r),
                                               0, 60, epsabs=0, epsrel=1e-13, limit=200)[0]
            assert abs(fermi.channel_density(d, beta, np.array([beta * mu]))[0] / n - 1.0) < 1e-12
        eps = fermi.internal_energy(d, beta, np.array([beta * mu_up]), np.array([beta * mu_dn]))[0]
        assert abs(eps / (energy / sum(dens)) - 1.0) < 1e-12
