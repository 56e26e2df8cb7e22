"""GPU parity of the magnetic-field collision (Sec. 5, Eq. sigmaB_comm)
against the oracle's exact precession, through the C ABI.

Bars as for the plain step: F64 within 1e-12 normwise, F32 within 1e-5;
a zero field map reproduces the plain step bit for bit; on a uniform
equilibrium state only the precession acts and every Bloch vector turns by
2 n |mu B| about B.
"""
import numpy as np
import pytest
import torch

from helpers import fields, from_pauli, gpu_init, make_handle, normwise_rel_err, oracle_init, oracle_pauli, to_pauli_np
from oracle import magnetic, pauli, qlbm
from paper_1309_1656_amd import mlbm

pytestmark = pytest.mark.gpu


def _flush(msg):
    print(msg, flush=True)


def _state(shape, seed=11):
    """A non-equilibrium state: equilibrium of smooth fields plus a seeded deviation."""
    f = fields(shape, seed)
    lat, Wo = oracle_init(shape, f)
    rng = np.random.default_rng(seed)
    a = rng.normal(0, 0.02, size=(4,) + Wo.shape[:-2]) * lat.w.reshape((1, -1) + (1,) * lat.d)
    return lat, Wo + pauli.matrix_from_pauli(a)


def _mu_b(shape, seed, uniform):
    rng = np.random.default_rng(seed)
    if uniform:
        b = rng.normal(0, 0.3, size=3)
        return b, np.broadcast_to(b.reshape((3,) + (1,) * len(shape)), (3,) + shape).copy()
    m = rng.normal(0, 0.3, size=(3,) + shape)
    return m, m


def _run_gpu(h, Wo, field, uniform, nsteps):
    W = from_pauli(h, oracle_pauli(Wo))
    tmp = h.empty_field()
    if uniform:
        mlbm.mlbm_set_magnetic_field(h, field)
        dmap = None
    else:
        dmap = torch.from_numpy(np.ascontiguousarray(field)).cuda()
        mlbm.mlbm_set_magnetic_field_map(h, dmap)
    mlbm.mlbm_step(h, W, tmp, nsteps)
    torch.cuda.synchronize()
    return to_pauli_np(h, W)


@pytest.mark.parametrize("shape", [(37, 70), (13, 9, 11), (6, 5, 70)])
@pytest.mark.parametrize("uniform", [True, False])
@pytest.mark.parametrize("storage,tol", [(mlbm.MLBM_STORE_F64, 1e-12), (mlbm.MLBM_STORE_F32, 1e-5)])
def test_field_step_matches_oracle(shape, uniform, storage, tol):
    _flush(f"field step {shape} uniform={uniform} storage={storage}")
    lat, Wo = _state(shape)
    field, mu_b = _mu_b(shape, 2, uniform)
    nsteps = 5
    h = make_handle(shape, tau=0.8, storage=storage)
    got = _run_gpu(h, Wo, field, uniform, nsteps)
    ref = oracle_pauli(magnetic.run_with_field(lat, Wo, 0.8, mu_b, nsteps))
    assert normwise_rel_err(got, ref) < tol
    # the field changes the result well beyond the bar
    plain = oracle_pauli(qlbm.run(lat, Wo, 0.8, nsteps))
    assert normwise_rel_err(plain, ref) > 1e3 * tol


@pytest.mark.parametrize("shape", [(37, 70), (13, 9, 11)])
def test_field_collide_matches_oracle(shape):
    _flush(f"field collide {shape}")
    lat, Wo = _state(shape, 4)
    _, mu_b = _mu_b(shape, 6, False)
    h = make_handle(shape, tau=0.7)
    W = from_pauli(h, oracle_pauli(Wo))
    dmap = torch.from_numpy(mu_b).cuda()
    mlbm.mlbm_set_magnetic_field_map(h, dmap)
    out = h.empty_field()
    mlbm.mlbm_collide(h, W, out)
    torch.cuda.synchronize()
    ref = oracle_pauli(magnetic.collide_with_field(lat, Wo, 0.7, mu_b))
    assert normwise_rel_err(to_pauli_np(h, out), ref) < 1e-13


@pytest.mark.parametrize("shape", [(37, 70), (13, 9, 11)])
@pytest.mark.parametrize("storage", [mlbm.MLBM_STORE_F64, mlbm.MLBM_STORE_F32])
def test_zero_field_map_is_plain_step_bitwise(shape, storage):
    _flush(f"zero field {shape} storage={storage}")
    _, Wo = _state(shape)
    h = make_handle(shape, storage=storage)
    a = _run_gpu(h, Wo, np.zeros((3,) + shape), False, 4)
    mlbm.mlbm_set_magnetic_field_map(h, None)
    b = _run_gpu(h, Wo, None, True, 4)            # None switches the field off
    assert np.array_equal(a, b)


def test_pure_precession_angle():
    """Uniform equilibrium: the BGK term vanishes and the Bloch vectors turn about B."""
    shape = (20, 70)
    h = make_handle(shape)
    f = {"trrho": np.ones(shape), "r": np.zeros((3,) + shape), "u_lat": np.zeros((2,) + shape),
         "T": np.ones(shape)}
    f["r"][0] = 0.2
    f["r"][2] = 0.1
    W = gpu_init(h, f)
    a0 = to_pauli_np(h, W)
    B = np.array([0.3, -0.2, 0.5])
    mlbm.mlbm_set_magnetic_field(h, B)
    n = 7
    mlbm.mlbm_step(h, W, h.empty_field(), n)
    torch.cuda.synchronize()
    an = to_pauli_np(h, W)
    axis = B / np.linalg.norm(B)
    th = 2 * n * np.linalg.norm(B)
    v = a0[1:]
    ax = axis.reshape((3, 1, 1, 1))
    cross = np.stack([ax[1] * v[2] - ax[2] * v[1], ax[2] * v[0] - ax[0] * v[2], ax[0] * v[1] - ax[1] * v[0]])
    dot = (ax * v).sum(axis=0)
    expect = v * np.cos(th) + cross * np.sin(th) + ax * dot * (1 - np.cos(th))
    assert np.max(np.abs(an[1:] - expect)) < 1e-14
    assert np.max(np.abs(an[0] - a0[0])) < 1e-15


def test_field_map_update_between_steps():
    """The map is read by every step: a time-dependent field is stepped segment by segment."""
    shape = (9, 8, 10)
    lat, Wo = _state(shape, 8)
    _, m1 = _mu_b(shape, 1, False)
    _, m2 = _mu_b(shape, 3, False)
    h = make_handle(shape)
    W = from_pauli(h, oracle_pauli(Wo))
    tmp = h.empty_field()
    dmap = torch.from_numpy(m1).cuda()
    mlbm.mlbm_set_magnetic_field_map(h, dmap)
    mlbm.mlbm_step(h, W, tmp, 2)
    dmap.copy_(torch.from_numpy(m2))
    mlbm.mlbm_step(h, W, tmp, 3)
    torch.cuda.synchronize()
    ref = magnetic.run_with_field(lat, magnetic.run_with_field(lat, Wo, 0.8, m1, 2), 0.8, m2, 3)
    assert normwise_rel_err(to_pauli_np(h, W), oracle_pauli(ref)) < 1e-12


# ---- the adjoint with a field ---------------------------------------------------

@pytest.mark.parametrize("shape", [(37, 70), (13, 9, 11)])
@pytest.mark.parametrize("uniform", [True, False])
def test_field_adjoint_step_matches_oracle(shape, uniform):
    _flush(f"field adjoint step {shape} uniform={uniform}")
    lat, Wo = _state(shape, 13)
    field, mu_b = _mu_b(shape, 5, uniform)
    rng = np.random.default_rng(4)
    lam1 = rng.standard_normal((4, lat.Q) + tuple(shape))
    h = make_handle(shape, tau=0.7)
    keep = None
    if uniform:
        mlbm.mlbm_set_magnetic_field(h, field)
    else:
        keep = torch.from_numpy(np.ascontiguousarray(field)).cuda()
        mlbm.mlbm_set_magnetic_field_map(h, keep)
    lam0 = h.empty_field()
    dom = torch.zeros(1, dtype=torch.float64, device="cuda")
    mlbm.mlbm_adjoint_step(h, from_pauli(h, oracle_pauli(Wo)), from_pauli(h, lam1), lam0, dom)
    torch.cuda.synchronize()
    L0, dom_o = magnetic.step_vjp_with_field(lat, Wo, pauli.matrix_from_pauli(2.0 * lam1), 0.7, mu_b)
    assert normwise_rel_err(to_pauli_np(h, lam0), pauli.pauli_from_matrix(L0) / 2.0) < 1e-12
    assert abs(dom.item() - dom_o) <= 1e-11 * abs(dom_o)


@pytest.mark.parametrize("K", [3, 10])
def test_field_rollout_gradient_matches_oracle(K):
    from oracle import adjoint
    from paper_1309_1656_amd import synthetic
    from paper_1309_1656_amd.rollout import MLBMRollout
    shape, tau, steps = (16, 16), 0.8, 10
    _flush(f"field rollout K={K}")
    f = fields(shape, synthetic.BASE_SEED + 5)
    rt_np = synthetic.target_bloch_field(shape, synthetic.BASE_SEED + 105)
    mu_b = np.random.default_rng(8).normal(0, 0.2, size=(3,) + shape)
    h = make_handle(shape, tau=tau)
    bmap = torch.from_numpy(mu_b).cuda()
    mlbm.mlbm_set_magnetic_field_map(h, bmap)
    W0 = gpu_init(h, f).requires_grad_(True)
    tau_t = torch.tensor(tau, dtype=torch.float64, requires_grad=True)
    loss = MLBMRollout.apply(W0, tau_t, h, steps, K, torch.from_numpy(rt_np).cuda())
    loss.backward()
    # oracle: every state stored, adjoint with the field
    lat, Wo = oracle_init(shape, f)
    states = [Wo]
    for _ in range(steps):
        states.append(magnetic.step_with_field(lat, states[-1], tau, mu_b))
    Lo, Lam = adjoint.spin_loss(lat, states[-1], rt_np)
    dom = 0.0
    for n in range(steps - 1, -1, -1):
        Lam, d = magnetic.step_vjp_with_field(lat, states[n], Lam, tau, mu_b)
        dom += d
    assert abs(loss.item() / Lo - 1) < 1e-12
    assert normwise_rel_err(to_pauli_np(h, W0.grad), pauli.pauli_from_matrix(Lam) / 2.0) < 1e-11
    assert abs(tau_t.grad.item() / (-dom / tau ** 2) - 1) < 1e-11
