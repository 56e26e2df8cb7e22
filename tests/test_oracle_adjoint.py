"""Pins of the oracle's hand-derived adjoint.

* Central finite differences of the oracle's forward step: a wrong sign, a
  dropped term or a transposed streaming direction shows up as a mismatch.
* Exact checks against a separate transcription of the step in plain PyTorch
  (CPU, float64): reverse-mode autograd equals the adjoint and dL/domega to
  1e-12, and the dot-product identity <J v, w> = <v, J^T w> holds with J v
  from forward-mode differentiation.
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


# ---- exact checks: torch autograd on an independent transcription ------------

def _torch_step(lat, a, om):
    """One collide-and-stream step in Pauli coefficients a [4, Q, *grid], plain
    PyTorch float64, transcribed separately from the oracle (Eqs. DiscrAvr,
    WeqAlgo, CollisionStep, TransportStep)."""
    import torch
    d = lat.d
    g = a.dim() - 2
    bs = lambda v: torch.as_tensor(v, dtype=torch.float64).reshape((-1,) + (1,) * g)
    e = torch.as_tensor(lat.e, dtype=torch.float64)
    w = bs(lat.w)
    rho = a.sum(dim=1)                                  # [4, *grid]
    T = rho[0]
    u = torch.stack([(bs(e[:, c]) * a[0]).sum(dim=0) / T for c in range(d)])
    dev2 = sum((bs(e[:, c]) - u[c][None]) ** 2 for c in range(d))
    eps = (0.5 * dev2 * a[0]).sum(dim=0) / T
    k, b0 = lat.coef, lat.beta0
    b = b0 * eps
    eu = sum(bs(e[:, c]) * u[c][None] for c in range(d))
    e2 = bs((lat.e ** 2).sum(axis=1))
    P = ((k["a1_0"] + k["a1_b"] * b)[None] + (k["a2_0"] + k["a2_b"] * b)[None] * b0 * 0.5 * e2
         + k["a3"] * b0 * eu + k["a4"] * (b0 * eu) ** 2 + k["a5"] * b0 * 0.5 * (u ** 2).sum(dim=0)[None])
    Weq = (w * P)[None] * rho[:, None]
    C = (1 - om) * a + om * Weq
    out = torch.empty_like(C)
    for i in range(lat.Q):
        shifts = tuple(int(lat.c[i, c]) for c in range(d))
        dims = tuple(2 + (d - 1 - c) for c in range(d))   # grid axes (z,) y, x after [4, Q]
        out[:, i] = torch.roll(C[:, i], shifts=shifts, dims=tuple(x - 1 for x in dims))
    return out


@pytest.mark.parametrize("d", [2, 3])
def test_vjp_equals_torch_autograd(d):
    import torch
    lat, W = _state(d, seed=5)
    tau = 0.7
    Lam_next = _rand_herm(W.shape[:-2], 23)
    Lam, dom = adjoint.step_vjp(lat, W, Lam_next, tau)
    a = torch.tensor(pauli.pauli_from_matrix(W), dtype=torch.float64, requires_grad=True)
    om = torch.tensor(1.0 / tau, dtype=torch.float64, requires_grad=True)
    m_next = torch.tensor(pauli.pauli_from_matrix(Lam_next) / 2.0, dtype=torch.float64)
    # the transcription reproduces the oracle's forward step
    fwd = _torch_step(lat, a, om).detach().numpy()
    assert np.max(np.abs(fwd - pauli.pauli_from_matrix(qlbm.step(lat, W, tau)))) < 1e-14
    L = (m_next * _torch_step(lat, a, om)).sum()
    ga, gom = torch.autograd.grad(L, (a, om))
    m_n = pauli.pauli_from_matrix(Lam) / 2.0
    assert np.max(np.abs(ga.numpy() - m_n)) < 1e-12 * np.max(np.abs(m_n))
    assert abs(gom.item() - dom) < 1e-12 * max(1.0, abs(dom))


@pytest.mark.parametrize("d", [2, 3])
def test_dot_product_identity(d):
    """<J v, w> = <v, J^T w> with J v by forward-mode differentiation of the
    transcription and J^T w from the oracle's adjoint."""
    import torch
    from torch.func import jvp
    lat, W = _state(d, seed=6)
    tau = 0.65
    a0 = torch.tensor(pauli.pauli_from_matrix(W), dtype=torch.float64)
    for seed in (1, 2):
        rng = np.random.default_rng(seed)
        v = torch.tensor(rng.normal(0, 1, size=a0.shape), dtype=torch.float64)
        wv = rng.normal(0, 1, size=a0.shape)
        _, Jv = jvp(lambda x: _torch_step(lat, x, 1.0 / tau), (a0,), (v,))
        lhs = float((Jv.numpy() * wv).sum())
        Lam, _ = adjoint.step_vjp(lat, W, pauli.matrix_from_pauli(2.0 * wv), tau)
        rhs = float((v.numpy() * pauli.pauli_from_matrix(Lam) / 2.0).sum())
        assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))
