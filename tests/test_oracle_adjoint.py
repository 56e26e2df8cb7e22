"""Pins of the oracle's hand-derived adjoint by central finite differences.

The adjoint is checked against the oracle's forward step only through
difference quotients, so a wrong sign, a dropped term or a transposed
streaming direction in the derivation shows up as a mismatch.
"""
import numpy as np
import pytest

from oracle import adjoint, pauli, qlbm
from paper_1309_1656_amd import synthetic

GRIDS = {2: (5, 6), 3: (3, 4, 5)}


def _state(d, seed=3):
    lat = qlbm.Lattice(d)
    shape = GRIDS[d]
    f = synthetic.macroscopic_fields(shape, seed)
    W = qlbm.init_equilibrium(lat, f["trrho"], f["r"], lat.xi * f["u_lat"], f["T"])
    rng = np.random.default_rng(seed)
    a = rng.normal(0, 0.02, size=(4,) + W.shape[:-2]) * lat.w.reshape((1, -1) + (1,) * d)
    return lat, W + pauli.matrix_from_pauli(a)


def _rand_herm(shape, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return pauli.matrix_from_pauli(rng.normal(0, scale, size=(4,) + shape))


def _pair(A, B):
    return float(np.real((A * np.swapaxes(B, -1, -2)).sum()))


@pytest.mark.parametrize("d", [2, 3])
def test_single_step_vjp_matches_finite_differences(d):
    lat, W = _state(d)
    tau = 0.7
    Lam_next = _rand_herm(W.shape[:-2], 17)
    Lam, dom = adjoint.step_vjp(lat, W, Lam_next, tau)
    for seed in (1, 2, 3):
        dW = _rand_herm(W.shape[:-2], 100 + seed, 1e-2)
        h = 1e-5
        fd = (_pair(Lam_next, qlbm.step(lat, W + h * dW, tau))
              - _pair(Lam_next, qlbm.step(lat, W - h * dW, tau))) / (2 * h)
        assert abs(_pair(Lam, dW) - fd) <= 1e-8 * max(1.0, abs(fd))
    # derivative with respect to omega = 1/tau
    h = 1e-6
    om = 1.0 / tau
    fd = (_pair(Lam_next, qlbm.step(lat, W, 1.0 / (om + h)))
          - _pair(Lam_next, qlbm.step(lat, W, 1.0 / (om - h)))) / (2 * h)
    assert abs(dom - fd) <= 1e-7 * max(1.0, abs(fd))


@pytest.mark.parametrize("d", [2, 3])
def test_rollout_gradient_matches_finite_differences(d):
    lat, W0 = _state(d, seed=8)
    shape = GRIDS[d]
    r_t = synthetic.target_bloch_field(shape, 99)
    tau, n = 0.8, 4
    L, Lam0, dtau = adjoint.rollout_grad(lat, W0, tau, n, r_t)
    assert abs(L - adjoint.rollout_loss(lat, W0, tau, n, r_t)) < 1e-15
    for seed in (4, 5):
        dW = _rand_herm(W0.shape[:-2], seed, 1e-2)
        h = 1e-5
        fd = (adjoint.rollout_loss(lat, W0 + h * dW, tau, n, r_t)
              - adjoint.rollout_loss(lat, W0 - h * dW, tau, n, r_t)) / (2 * h)
        assert abs(_pair(Lam0, dW) - fd) <= 1e-7 * max(1e-3, abs(fd))
    # one entry at a time: Pauli coefficient k of population i at one cell
    for (k, i) in [(0, 0), (2, 3), (3, lat.Q - 1), (1, 1)]:
        cell = tuple(s // 2 for s in shape)
        da = np.zeros((4,) + W0.shape[:-2])
        da[(k, i) + cell] = 1.0
        dW = pauli.matrix_from_pauli(da)
        h = 1e-5
        fd = (adjoint.rollout_loss(lat, W0 + h * dW, tau, n, r_t)
              - adjoint.rollout_loss(lat, W0 - h * dW, tau, n, r_t)) / (2 * h)
        grad_k = pauli.pauli_from_matrix(Lam0)[(k, i) + cell] / 2.0   # l_k = Re tr(Lam s_k)/2
        assert abs(grad_k - fd) <= 1e-7 * max(1e-4, abs(fd)), (k, i, grad_k, fd)
    h = 1e-6
    fd = (adjoint.rollout_loss(lat, W0, tau + h, n, r_t) - adjoint.rollout_loss(lat, W0, tau - h, n, r_t)) / (2 * h)
    assert abs(dtau - fd) <= 1e-7 * max(1e-4, abs(fd))


def test_spin_loss_seed_has_no_trace_part():
    lat, W = _state(2)
    r_t = synthetic.target_bloch_field(GRIDS[2], 5)
    L, Lam = adjoint.spin_loss(lat, W, r_t)
    assert np.all(pauli.pauli_from_matrix(Lam)[0] == 0)
    assert L > 0
