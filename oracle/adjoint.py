"""Reverse-mode derivative of the step and of the final spin-density loss.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Derived here from Sec. 3.3 (Eqs. DiscrAvr, WeqAlgo, CollisionStep,
TransportStep); the paper itself has no adjoint.  An adjoint field Lam has the
same [Q, *grid, 2, 2] Hermitian form as W, paired with a variation by
dL = sum_{x,i} Re tr(Lam_i(x) dW_i(x)).  (Its Pauli coefficients
l_k = Re tr(Lam s_k) / 2 are then the partial derivatives of L with respect to
the coefficients a_k of W.)

One step is W_{n+1} = S(C(W_n)) with S the streaming permutation and
C_i(W) = (1 - w) W_i + w w_i rho P_i(u, eps), w = Delta t / tau.  Its adjoint:
  g_i(x)     = Lam_{n+1,i}(x + c_i)                       (inverse permutation)
  G_i        = w_i Re tr(g_i rho)
  Lam_{n,j}  = (1 - w) g_j + w sum_i w_i P_i g_i
               + w I [ G_u . (e_j - u) + G_eps (|e_j - u|^2/2 - eps) ] / T
  with G_u = sum_i G_i dP_i/du, G_eps = sum_i G_i dP_i/deps, which follow from
  du/d(tr W_j) = (e_j - u)/T and deps/d(tr W_j) = (|e_j - u|^2/2 - eps)/T;
  dL/dw     += sum_{x,i} Re tr(g_i (W_eq_i - W_i)),  dL/dtau = -dL/dw / tau^2.
"""
import numpy as np

from . import qlbm
from .pauli import SIGMA
from .qlbm import _bshape, moments, poly_factor, stream


def poly_factor_grad(lat, u, eps):
    """(dP_i/du [Q, d, *grid], dP_i/deps [Q, *grid]) of the Eq. WeqAlgo polynomial."""
    g = u.ndim - 1
    k = lat.coef
    b0 = lat.beta0
    eu = sum(_bshape(lat.e[:, a], g) * u[a][None] for a in range(lat.d))
    dPdu = np.stack([
        k["a3"] * b0 * _bshape(lat.e[:, a], g)
        + 2.0 * k["a4"] * b0 ** 2 * eu * _bshape(lat.e[:, a], g)
        + k["a5"] * b0 * u[a][None]
        for a in range(lat.d)], axis=1)
    e2 = (lat.e ** 2).sum(axis=1)
    dPde = b0 * (k["a1_b"] + k["a2_b"] * b0 * 0.5 * _bshape(e2, g)) * np.ones_like(eps)[None]
    return dPdu, dPde


def step_vjp(lat, W, Lam_next, tau, dt=1.0):
    """(Lam_n, dL/dw) for one step from the pre-collision state W = W_n."""
    return collision_vjp(lat, W, stream(lat, Lam_next, sign=-1), tau, dt)


def collision_vjp(lat, W, G, tau, dt=1.0):
    """(Lam_n, dL/dw) of the collision alone, G being the adjoint of its output."""
    om = dt / tau
    g = W.ndim - 3
    rho, T, u, eps = moments(lat, W)
    P = poly_factor(lat, u, eps)
    wP = _bshape(lat.w, g) * P
    Weq = wP[..., None, None] * rho[None]
    dL_dom = float(np.real((G * np.swapaxes(Weq - W, -1, -2)).sum()))
    Gs = _bshape(lat.w, g) * np.real((G * np.swapaxes(rho, -1, -2)[None]).sum(axis=(-1, -2)))
    dPdu, dPde = poly_factor_grad(lat, u, eps)
    Gu = (Gs[:, None] * dPdu).sum(axis=0)              # [d, *grid]
    Ge = (Gs * dPde).sum(axis=0)                        # [*grid]
    mix = (wP[..., None, None] * G).sum(axis=0)         # sum_i w_i P_i g_i
    scal = np.zeros((lat.Q,) + T.shape)
    dev2 = np.zeros_like(scal)
    for a in range(lat.d):
        diff = _bshape(lat.e[:, a], g) - u[a][None]
        scal += Gu[a][None] * diff
        dev2 += diff ** 2
    scal = om * (scal + Ge[None] * (0.5 * dev2 - eps[None])) / T[None]
    Lam = (1.0 - om) * G + om * mix[None] + scal[..., None, None] * SIGMA[0]
    return Lam, dL_dom


def spin_loss(lat, W, r_target):
    """(L, Lam_N): L = mean_x |r(x) - r_target(x)|^2 with r the Bloch vector of rho.

    Lam_N,i(x) = (2 / |grid|) sum_k (r_k - r_target_k) s_k for every i.
    """
    rho = W.sum(axis=0)
    r = qlbm.bloch(rho)
    diff = r - r_target
    ncell = r[0].size
    L = float((diff ** 2).sum() / ncell)
    lam = np.zeros(rho.shape, dtype=np.complex128)
    for k in range(3):
        lam = lam + (2.0 / ncell) * diff[k][..., None, None] * SIGMA[k + 1]
    return L, np.broadcast_to(lam[None], W.shape).copy()


def rollout_loss(lat, W0, tau, nsteps, r_target):
    return spin_loss(lat, qlbm.run(lat, W0, tau, nsteps), r_target)[0]


def rollout_grad(lat, W0, tau, nsteps, r_target):
    """(L, dL/dW0 as a Hermitian adjoint field, dL/dtau) by storing every state."""
    states = [W0]
    for _ in range(nsteps):
        states.append(qlbm.step(lat, states[-1], tau))
    L, Lam = spin_loss(lat, states[-1], r_target)
    dom = 0.0
    for n in range(nsteps - 1, -1, -1):
        Lam, d = step_vjp(lat, states[n], Lam, tau)
        dom += d
    return L, Lam, -dom / tau ** 2
