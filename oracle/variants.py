"""Two variants of the collision that the paper describes without pursuing.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Isothermal model (Sec. 3.1, paragraph on beta0 and mu0): the physical inverse
temperature of every cell is held at beta = beta0.  The equilibrium then has
the Fermi-Dirac parameters (beta0, nu_up, nu_dn) that reproduce the cell's
density matrix, so its internal energy is eps_FD(beta0; n_up, n_dn) of
Eq. energyFDstdOmega instead of the moment eps, and energy is no longer
conserved.  Reading: the Appendix coefficients are taken with
eps_FD := eps_FD(beta0; n_up, n_dn), everything else as in Eq. WeqAlgo.

Positivity-preserving relaxation (Sec. 3.3, paragraph after the algorithm):
1/tau is lowered per cell so that every W_coll_i is positive semidefinite.
Reading: per cell the largest omega' in [0, omega] such that for every
population i the smaller eigenvalue of (1 - omega') W_i + omega' W_eq_i is at
least min(0, smaller eigenvalue of W_i): positive semidefinite populations
stay so, and one that is already slightly negative (rounding of a population
left on the boundary by the previous step) is not made worse, which keeps the
rate a continuous function of the state.  The smallest eigenvalue is concave
in omega', so the admissible set of each population is an interval
[0, omega_i*].  Here omega_i* is found by bisection on eigvalsh.
"""
import numpy as np

from . import fermi
from .qlbm import _bshape, equilibrium, moments


def isothermal_energy(d, beta0, rho):
    """eps_FD(beta0; n_up, n_dn) of the cell density matrices rho [*grid, 2, 2]."""
    ev = np.linalg.eigvalsh(rho)               # ascending: n_dn, n_up
    nu_dn = fermi.chemical_potential_scaled(d, beta0, ev[..., 0])
    nu_up = fermi.chemical_potential_scaled(d, beta0, ev[..., 1])
    return fermi.internal_energy(d, beta0, nu_up, nu_dn)


def collide_isothermal(lat, W, tau, dt=1.0):
    rho, T, u, eps = moments(lat, W)
    Weq = equilibrium(lat, rho, u, isothermal_energy(lat.d, lat.beta0, rho))
    return W + (dt / tau) * (Weq - W)


def _min_eig(X):
    return np.linalg.eigvalsh(X)[..., 0]


def positive_omega(lat, W, Weq, omega, iters=80):
    """Per-cell relaxation rate omega' of the positivity-preserving collision."""
    floor = np.minimum(0.0, _min_eig(W))                        # [Q, *grid]
    need = _min_eig((1.0 - omega) * W + omega * Weq) < floor
    if not need.any():
        return np.full(W.shape[1:-2], float(omega))
    lo = np.zeros(W.shape[:-2])                                 # admissible
    hi = np.full(W.shape[:-2], float(omega))                    # not admissible where `need`
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        ok = _min_eig((1.0 - mid[..., None, None]) * W + mid[..., None, None] * Weq) >= floor
        lo = np.where(ok, mid, lo)
        hi = np.where(ok, hi, mid)
    return np.where(need, lo, float(omega)).min(axis=0)


def collide_positive(lat, W, tau, dt=1.0, isothermal=False):
    rho, T, u, eps = moments(lat, W)
    e = isothermal_energy(lat.d, lat.beta0, rho) if isothermal else eps
    Weq = equilibrium(lat, rho, u, e)
    om = positive_omega(lat, W, Weq, dt / tau)
    om = _bshape(om, 2)[None]
    return W + om * (Weq - W)


def step_variant(lat, W, tau, isothermal=False, positive=False):
    from .qlbm import stream
    if positive:
        return stream(lat, collide_positive(lat, W, tau, isothermal=isothermal))
    if isothermal:
        return stream(lat, collide_isothermal(lat, W, tau))
    from .qlbm import collide
    return stream(lat, collide(lat, W, tau))


def run_variant(lat, W, tau, nsteps, isothermal=False, positive=False):
    for _ in range(nsteps):
        W = step_variant(lat, W, tau, isothermal, positive)
    return W
