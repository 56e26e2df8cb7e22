"""Collision with an external magnetic field (Sec. 5, Eq. sigmaB_comm).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 5 adds the local commutator -i [mu sigma.B(x, t), W] to the right-hand
side of the Boltzmann equation and says it can simply be added to the
collision operator.  Reading used here: over one time step the commutator
term is integrated exactly, W -> U W U* with U = exp(-i mu Delta t sigma.B(x)),
and composed with the BGK collision of Eq. CollisionStep.  The two commute
cell by cell (the BGK collision is covariant under one SU(2) matrix per cell:
rho rotates, u and eps are traces), so the order does not matter.

U is taken from scipy's matrix exponential (a library primitive); the tests
pin it against direct numerical integration of dW/dt = -i [mu sigma.B, W].
"""
import numpy as np
from scipy.linalg import expm

from . import adjoint
from .pauli import SIGMA
from .qlbm import collide, stream


def precession_unitary(mu_b, dt=1.0):
    """U = exp(-i dt sigma.(mu B)) for each cell; mu_b has shape [3, *grid]."""
    grid = mu_b.shape[1:]
    H = sum(mu_b[k][..., None, None] * SIGMA[k + 1] for k in range(3))   # [*grid, 2, 2]
    flat = H.reshape(-1, 2, 2)
    U = np.stack([expm(-1j * dt * h) for h in flat])
    return U.reshape(grid + (2, 2))


def precess(W, mu_b, dt=1.0):
    """W_i -> U W_i U* in every cell (the same U for all populations of a cell)."""
    U = precession_unitary(mu_b, dt)
    return U[None] @ W @ np.conj(np.swapaxes(U, -1, -2))[None]


def collide_with_field(lat, W, tau, mu_b, dt=1.0):
    """BGK collision followed by the exact precession of the commutator term."""
    return precess(collide(lat, W, tau, dt), mu_b, dt)


def step_with_field(lat, W, tau, mu_b):
    return stream(lat, collide_with_field(lat, W, tau, mu_b))


def run_with_field(lat, W, tau, mu_b, nsteps):
    for _ in range(nsteps):
        W = step_with_field(lat, W, tau, mu_b)
    return W


def step_vjp_with_field(lat, W, Lam_next, tau, mu_b, dt=1.0):
    """(Lam_n, dL/dw) of one step with the field: W_{n+1} = S(P(C(W_n))) with
    P(X) = U X U*.  Under the pairing Re tr(Lam X) the adjoint of P is
    Y -> U* Y U, so the adjoint of the streamed output is turned back before
    the collision's adjoint."""
    G = stream(lat, Lam_next, sign=-1)
    U = precession_unitary(mu_b, dt)
    Uh = np.conj(np.swapaxes(U, -1, -2))
    return adjoint.collision_vjp(lat, W, Uh[None] @ G @ U[None], tau, dt)
