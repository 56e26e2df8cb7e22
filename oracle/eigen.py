"""Equilibrium through the eigen-decomposition of rho and the Fermi-Dirac parameters.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 2.2 (Prop. 1) says the moments (rho, u, eps) fix (beta, mu_up, mu_dn, u)
uniquely; the unitary U is recovered by diagonalising rho (remark after
Prop. 1).  Eq. WeqDiscr then builds
    W_eq_i = w_i U diag(n_{d,beta,mu_up}, n_{d,beta,mu_dn}) U* P_i(u, eps_FD).
The algorithm of Sec. 3.3 skips U and F_k because the result is the same;
this module takes the long way round so that the identity can be tested.

Inversion used here (plain and slow): for a trial beta each channel's
nu_s = beta mu_s follows from its density by Newton (fermi.invert_density);
eps_FD(beta) of Eq. energyFDstdOmega then decreases monotonically in beta, so
beta is found by bisection in log(beta).  The bracket starts from the
classical value beta = d / (2 eps), a lower bound because the ratio
F_{d/2}/F_{d/2-1} is at least 1 for fermions.
"""
import numpy as np

from . import fermi
from .qlbm import moments, poly_factor, _bshape


def _eps_of_beta(d, beta, lam_up, lam_dn):
    nu_up = fermi.chemical_potential_scaled(d, beta, lam_up)
    nu_dn = fermi.chemical_potential_scaled(d, beta, lam_dn)
    return fermi.internal_energy(d, beta, nu_up, nu_dn), nu_up, nu_dn


def solve_parameters(d, lam_up, lam_dn, eps, maxit=200):
    """(beta, nu_up, nu_dn) with channel densities lam_up/dn and internal energy eps."""
    lo = d / (2.0 * eps)
    hi = lo.copy()
    for _ in range(200):
        e_hi, _, _ = _eps_of_beta(d, hi, lam_up, lam_dn)
        grow = e_hi > eps
        if not grow.any():
            break
        hi = np.where(grow, hi * 2.0, hi)
    else:
        raise RuntimeError("no bracket for beta")
    llo, lhi = np.log(lo), np.log(hi)
    for _ in range(maxit):
        mid = 0.5 * (llo + lhi)
        e_mid, _, _ = _eps_of_beta(d, np.exp(mid), lam_up, lam_dn)
        above = e_mid > eps           # energy too high -> beta too small
        llo = np.where(above, mid, llo)
        lhi = np.where(above, lhi, mid)
        if np.all(lhi - llo <= 4e-16 * np.maximum(1.0, np.abs(lhi))):
            break
    beta = np.exp(0.5 * (llo + lhi))
    _, nu_up, nu_dn = _eps_of_beta(d, beta, lam_up, lam_dn)
    return beta, nu_up, nu_dn


def equilibrium_eigen(lat, W):
    """W_eq built as in Eq. WeqDiscr from the Fermi-Dirac parameters of each cell."""
    d = lat.d
    rho, T, u, eps = moments(lat, W)
    lam, V = np.linalg.eigh(rho)               # ascending eigenvalues
    lam_dn, lam_up = lam[..., 0], lam[..., 1]
    beta, nu_up, nu_dn = solve_parameters(d, lam_up, lam_dn, eps)
    n_up = fermi.channel_density(d, beta, nu_up)
    n_dn = fermi.channel_density(d, beta, nu_dn)
    eps_fd = fermi.internal_energy(d, beta, nu_up, nu_dn)
    D = np.zeros(rho.shape, dtype=np.complex128)
    D[..., 0, 0] = n_dn
    D[..., 1, 1] = n_up
    rho_eq = V @ D @ np.conj(np.swapaxes(V, -1, -2))
    P = poly_factor(lat, u, eps_fd)
    g = u.ndim - 1
    return _bshape(lat.w, g + 2) * P[..., None, None] * rho_eq[None]
