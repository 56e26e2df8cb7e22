"""GPU adjoint against the oracle's hand-derived adjoint and against finite
differences of the GPU forward step, through the C ABI and the autograd
wrapper."""
import numpy as np
import pytest
import torch

from helpers import fields, from_pauli, gpu_init, make_handle, normwise_rel_err, oracle_init, oracle_pauli, to_pauli_np
from oracle import adjoint, pauli, qlbm
from paper_1309_1656_amd import mlbm, synthetic
from paper_1309_1656_amd.rollout import MLBMRollout

pytestmark = pytest.mark.gpu


def _perturbed(lat, W, seed=5, amp=0.02):
    rng = np.random.default_rng(seed)
    a = rng.normal(0, amp, size=(4,) + W.shape[:-2]) * lat.w.reshape((1, -1) + (1,) * lat.d)
    return W + pauli.matrix_from_pauli(a)


@pytest.mark.parametrize("shape", [(37, 70), (13, 9, 11)])
def test_adjoint_step_matches_oracle(shape):
    print(f"adjoint step {shape}", flush=True)
    f = fields(shape, 12)
    lat, Wo = oracle_init(shape, f)
    Wo = _perturbed(lat, Wo)
    rng = np.random.default_rng(4)
    lam1 = rng.standard_normal((4, lat.Q) + tuple(shape))
    h = make_handle(shape, tau=0.7)
    lam0 = h.empty_field()
    dom = torch.full((1,), 0.25, dtype=torch.float64, device="cuda")
    mlbm.mlbm_adjoint_step(h, from_pauli(h, oracle_pauli(Wo)), from_pauli(h, lam1), lam0, dom)
    L0, dom_o = adjoint.step_vjp(lat, Wo, pauli.matrix_from_pauli(2.0 * lam1), 0.7)
    ref = pauli.pauli_from_matrix(L0) / 2.0
    assert normwise_rel_err(to_pauli_np(h, lam0), ref) < 1e-12
    assert abs((dom.item() - 0.25) - dom_o) <= 1e-11 * abs(dom_o)


def _loss_and_grad(h, W0, tau, steps, K, rt):
    W0 = W0.clone().requires_grad_(True)
    tau_t = torch.tensor(tau, dtype=torch.float64, requires_grad=True)
    loss = MLBMRollout.apply(W0, tau_t, h, steps, K, rt)
    loss.backward()
    return loss.item(), W0.grad, tau_t.grad.item()


@pytest.mark.parametrize("K", [3, 10, 20])
def test_rollout_gradient_matches_oracle(K):
    shape, tau, steps = (16, 16), 0.8, 10
    f = fields(shape, synthetic.BASE_SEED + 5)
    rt_np = synthetic.target_bloch_field(shape, synthetic.BASE_SEED + 105)
    h = make_handle(shape, tau=tau)
    W0 = gpu_init(h, f)
    L, gW, gtau = _loss_and_grad(h, W0, tau, steps, K, torch.from_numpy(rt_np).cuda())
    lat, Wo = oracle_init(shape, f)
    Lo, Lam0, dtau_o = adjoint.rollout_grad(lat, Wo, tau, steps, rt_np)
    assert abs(L / Lo - 1) < 1e-12
    assert normwise_rel_err(to_pauli_np(h, gW), pauli.pauli_from_matrix(Lam0) / 2.0) < 1e-11
    assert abs(gtau / dtau_o - 1) < 1e-11


def test_rollout_gradient_matches_gpu_finite_differences():
    shape, tau, steps = (16, 16), 0.8, 10
    f = fields(shape, synthetic.BASE_SEED + 5)
    rt = torch.from_numpy(synthetic.target_bloch_field(shape, synthetic.BASE_SEED + 105)).cuda()
    h = make_handle(shape, tau=tau)
    W0 = gpu_init(h, f)
    L, gW, gtau = _loss_and_grad(h, W0, tau, steps, 4, rt)

    def loss_at(W, t):
        with torch.no_grad():
            return MLBMRollout.apply(W, torch.tensor(t, dtype=torch.float64), h, steps, 4, rt).item()

    rng = np.random.default_rng(9)
    for _ in range(3):
        dW = torch.from_numpy(rng.standard_normal(W0.shape) * 1e-3).cuda()
        e = 1e-4
        fd = (loss_at(W0 + e * dW, tau) - loss_at(W0 - e * dW, tau)) / (2 * e)
        an = float((gW * dW).sum())
        assert abs(an - fd) <= 1e-6 * max(abs(fd), 1e-8)
    e = 1e-5
    fd = (loss_at(W0, tau + e) - loss_at(W0, tau - e)) / (2 * e)
    assert abs(gtau - fd) <= 1e-6 * abs(fd)


def test_f32_rollout_against_f64_oracle():
    """FP32 forward + adjoint (checkpoints every 20) vs the FP64 oracle: error reported."""
    shape, tau, steps = (64, 64), 0.8, 200
    f = fields(shape, synthetic.BASE_SEED + 5)
    rt_np = synthetic.target_bloch_field(shape, synthetic.BASE_SEED + 105)
    h = make_handle(shape, tau=tau, storage=mlbm.MLBM_STORE_F32)
    W0 = gpu_init(h, f)
    L, gW, gtau = _loss_and_grad(h, W0, tau, steps, 20, torch.from_numpy(rt_np).cuda())
    lat, Wo = oracle_init(shape, f)
    Lo, Lam0, dtau_o = adjoint.rollout_grad(lat, Wo, tau, steps, rt_np)
    gerr = normwise_rel_err(to_pauli_np(h, gW), pauli.pauli_from_matrix(Lam0) / 2.0)
    print(f"f32 rollout: loss rel err {abs(L / Lo - 1):.2e}, grad W0 {gerr:.2e}, grad tau {abs(gtau / dtau_o - 1):.2e}")
    assert abs(L / Lo - 1) < 1e-5
    assert gerr < 1e-4
    assert abs(gtau / dtau_o - 1) < 1e-4


def test_spin_loss_matches_oracle():
    shape = (13, 9, 11)
    f = fields(shape, 3)
    rt_np = synthetic.target_bloch_field(shape, 77)
    h = make_handle(shape)
    W = gpu_init(h, f)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    lam = h.empty_field()
    mlbm.mlbm_spin_loss(h, W, torch.from_numpy(rt_np).cuda(), loss=loss, lam=lam)
    lat, Wo = oracle_init(shape, f)
    Lo, Lam = adjoint.spin_loss(lat, Wo, rt_np)
    assert abs(loss.item() / Lo - 1) < 1e-13
    ref = pauli.pauli_from_matrix(Lam) / 2.0
    got = to_pauli_np(h, lam)
    assert np.all(got[0] == 0)
    assert np.max(np.abs(got[1:] - ref[1:])) <= 1e-13 * np.abs(ref[1:]).max()


@pytest.mark.parametrize("shape,n", [((37, 70), 7), ((13, 9, 11), 4), ((16, 16), 1)])
def test_adjoint_segment_equals_stepwise(shape, n):
    """One mlbm_adjoint_segment call == n recomputed states + n mlbm_adjoint_step calls."""
    f = fields(shape, 31)
    h = make_handle(shape, tau=0.7)
    W0 = gpu_init(h, f)
    rng = np.random.default_rng(6)
    lamN = from_pauli(h, rng.standard_normal((4, h.Q) + tuple(shape)))
    # step by step
    states = [W0.clone()]
    W = W0.clone()
    for _ in range(n - 1):
        mlbm.mlbm_step(h, W, h.empty_field(), 1)
        states.append(W.clone())
    lam = lamN.clone()
    out = h.empty_field()
    dom_a = torch.zeros(1, dtype=torch.float64, device="cuda")
    for j in range(n - 1, -1, -1):
        mlbm.mlbm_adjoint_step(h, states[j], lam, out, dom_a)
        lam, out = out, lam
    # one call
    lam_b = lamN.clone()
    buf = torch.empty((max(n - 1, 1),) + tuple(W0.shape), dtype=W0.dtype, device="cuda") if n > 1 else None
    dom_b = torch.zeros(1, dtype=torch.float64, device="cuda")
    mlbm.mlbm_adjoint_segment(h, W0, buf, n, lam_b, h.empty_field(), dom_b)
    assert torch.equal(lam, lam_b)
    # the segment sums dL/domega per block over all steps before the one final
    # sum, the stepwise calls per step: same terms, other rounding order
    assert abs(dom_a.item() - dom_b.item()) <= 1e-13 * abs(dom_a.item())


@pytest.mark.parametrize("shape", [(37, 70), (13, 9, 11)])
@pytest.mark.parametrize("n", [0, 1, 2, 5])
def test_step_states_equals_step(shape, n):
    """mlbm_step_states (out of place, nstates = 2 or n) gives mlbm_step's result bit for bit and
    keeps the post-collision states: streaming state j gives the state after j + 1 steps."""
    print(f"step_states {shape} n={n}", flush=True)
    f = fields(shape, 41)
    h = make_handle(shape, tau=0.7)
    W0 = gpu_init(h, f)
    ref = W0.clone()
    mlbm.mlbm_step(h, ref, h.empty_field(), n)
    for nstates in sorted({2, max(n, 1)}):
        states = torch.empty((nstates,) + tuple(W0.shape), dtype=W0.dtype, device="cuda")
        W0_copy = W0.clone()
        out = h.empty_field()
        mlbm.mlbm_step_states(h, W0, out, states, n, nstates=nstates)
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
        assert torch.equal(W0, W0_copy)          # src is read only
        if nstates >= n:
            for j in range(n):
                after = W0.clone()
                mlbm.mlbm_step(h, after, h.empty_field(), j + 1)
                streamed = h.empty_field()
                mlbm.mlbm_stream(h, states[j], streamed)
                assert torch.equal(streamed, after), j


@pytest.mark.parametrize("shape,n", [((37, 70), 7), ((13, 9, 11), 4), ((16, 16), 1)])
def test_adjoint_sweep_equals_segment(shape, n):
    """mlbm_adjoint_sweep on states kept by mlbm_step_states == mlbm_adjoint_segment (which recomputes them)."""
    f = fields(shape, 43)
    h = make_handle(shape, tau=0.7)
    W0 = gpu_init(h, f)
    rng = np.random.default_rng(7)
    lamN = from_pauli(h, rng.standard_normal((4, h.Q) + tuple(shape)))
    states = torch.empty((max(n, 2),) + tuple(W0.shape), dtype=W0.dtype, device="cuda")
    mlbm.mlbm_step_states(h, W0, h.empty_field(), states, n, nstates=n)
    lam_a = lamN.clone()
    dom_a = torch.zeros(1, dtype=torch.float64, device="cuda")
    mlbm.mlbm_adjoint_sweep(h, W0, states if n > 1 else None, n, lam_a, h.empty_field(), dom_a)
    lam_b = lamN.clone()
    dom_b = torch.zeros(1, dtype=torch.float64, device="cuda")
    buf = torch.empty((max(n - 1, 1),) + tuple(W0.shape), dtype=W0.dtype, device="cuda")
    mlbm.mlbm_adjoint_segment(h, W0, buf if n > 1 else None, n, lam_b, h.empty_field(), dom_b)
    assert torch.equal(lam_a, lam_b)
    assert dom_a.item() == dom_b.item()


@pytest.mark.parametrize("steps,K", [(10, 1), (7, 3), (0, 4)])
def test_rollout_segmentations_match_oracle(steps, K):
    """Every segment length, including one-step segments and no steps at all."""
    shape, tau = (16, 16), 0.8
    f = fields(shape, synthetic.BASE_SEED + 5)
    rt_np = synthetic.target_bloch_field(shape, synthetic.BASE_SEED + 105)
    h = make_handle(shape, tau=tau)
    W0 = gpu_init(h, f)
    L, gW, gtau = _loss_and_grad(h, W0, tau, steps, K, torch.from_numpy(rt_np).cuda())
    lat, Wo = oracle_init(shape, f)
    Lo, Lam0, dtau_o = adjoint.rollout_grad(lat, Wo, tau, steps, rt_np)
    assert abs(L / Lo - 1) < 1e-12
    assert normwise_rel_err(to_pauli_np(h, gW), pauli.pauli_from_matrix(Lam0) / 2.0) < 1e-11
    if steps > 0:
        assert abs(gtau / dtau_o - 1) < 1e-11
    else:
        assert gtau == 0.0


def test_rollout_backward_twice():
    """A second backward over the same graph (retain_graph) recomputes the last segment and agrees."""
    shape, tau, steps, K = (16, 16), 0.8, 10, 4
    f = fields(shape, synthetic.BASE_SEED + 5)
    rt = torch.from_numpy(synthetic.target_bloch_field(shape, synthetic.BASE_SEED + 105)).cuda()
    h = make_handle(shape, tau=tau)
    W0 = gpu_init(h, f).requires_grad_(True)
    tau_t = torch.tensor(tau, dtype=torch.float64, requires_grad=True)
    loss = MLBMRollout.apply(W0, tau_t, h, steps, K, rt)
    loss.backward(retain_graph=True)
    g1, t1 = W0.grad.clone(), tau_t.grad.clone()
    W0.grad, tau_t.grad = None, None
    loss.backward()
    assert torch.equal(W0.grad, g1)
    assert tau_t.grad.item() == t1.item()


@pytest.mark.parametrize("shape", [(37, 70), (13, 9, 11)])
@pytest.mark.parametrize("n,m", [(1, 1), (2, 3), (5, 4)])
def test_step_post_equals_step(shape, n, m):
    """mlbm_step_post keeps the same post-collision states as mlbm_step_states bit for bit; streaming its
    last state gives mlbm_step's result; continuing from that post-collision state (src_post) for m more
    steps gives the state after n + m steps."""
    print(f"step_post {shape} n={n} m={m}", flush=True)
    f = fields(shape, 47)
    h = make_handle(shape, tau=0.7)
    W0 = gpu_init(h, f)
    ref_states = torch.empty((max(n, 2),) + tuple(W0.shape), dtype=W0.dtype, device="cuda")
    mlbm.mlbm_step_states(h, W0, h.empty_field(), ref_states, n, nstates=n)
    states = torch.empty((max(n - 1, 1),) + tuple(W0.shape), dtype=W0.dtype, device="cuda")
    last = h.empty_field()
    mlbm.mlbm_step_post(h, W0, n, states=states if n > 1 else None, dst=last, nstates=max(n - 1, 1))
    for j in range(n - 1):
        assert torch.equal(states[j], ref_states[j]), j
    assert torch.equal(last, ref_states[n - 1])
    after_n = W0.clone()
    mlbm.mlbm_step(h, after_n, h.empty_field(), n)
    streamed = h.empty_field()
    mlbm.mlbm_stream(h, last, streamed)
    assert torch.equal(streamed, after_n)
    # continue from the post-collision state, all states into a ring of two
    ring = torch.empty((2,) + tuple(W0.shape), dtype=W0.dtype, device="cuda")
    last2 = h.empty_field()
    mlbm.mlbm_step_post(h, last, m, states=ring, dst=last2, src_post=True, nstates=2)
    after_nm = W0.clone()
    mlbm.mlbm_step(h, after_nm, h.empty_field(), n + m)
    mlbm.mlbm_stream(h, last2, streamed)
    assert torch.equal(streamed, after_nm)


@pytest.mark.parametrize("shape,n", [((37, 70), 5), ((13, 9, 11), 4), ((16, 16), 1)])
def test_adjoint_sweep_post_equals_sweep(shape, n):
    """A segment started from the post-collision state before it (mlbm_adjoint_sweep_post) equals the same
    segment started from its pre-collision state (mlbm_adjoint_sweep), bit for bit."""
    f = fields(shape, 53)
    h = make_handle(shape, tau=0.7)
    W0 = gpu_init(h, f)
    S_prev = h.empty_field()
    mlbm.mlbm_step_post(h, W0, 3, states=torch.empty((2,) + tuple(W0.shape), dtype=W0.dtype, device="cuda"),
                        dst=S_prev, nstates=2)
    Wa = h.empty_field()
    mlbm.mlbm_stream(h, S_prev, Wa)                  # pre-collision state at the segment start
    states = torch.empty((max(n - 1, 1),) + tuple(W0.shape), dtype=W0.dtype, device="cuda")
    if n > 1:
        mlbm.mlbm_step_post(h, S_prev, n - 1, states=states, src_post=True, nstates=n - 1)
    rng = np.random.default_rng(8)
    lamN = from_pauli(h, rng.standard_normal((4, h.Q) + tuple(shape)))
    lam_a, lam_b = lamN.clone(), lamN.clone()
    dom_a = torch.zeros(1, dtype=torch.float64, device="cuda")
    dom_b = torch.zeros(1, dtype=torch.float64, device="cuda")
    mlbm.mlbm_adjoint_sweep(h, Wa, states if n > 1 else None, n, lam_a, h.empty_field(), dom_a)
    mlbm.mlbm_adjoint_sweep_post(h, S_prev, states if n > 1 else None, n, lam_b, h.empty_field(), dom_b)
    assert torch.equal(lam_a, lam_b)
    assert dom_a.item() == dom_b.item()


@pytest.mark.parametrize("shape", [(37, 70), (13, 9, 130)])
@pytest.mark.parametrize("storage", [mlbm.MLBM_STORE_F64, mlbm.MLBM_STORE_F32])
def test_adjoint_launch_shapes_give_identical_results(shape, storage):
    """A 4-step reverse sweep on pulled post-collision states (as in a rollout) under every channel-form
    shape: block width, XCD order, occupancy cap and store policy only reorder independent cells, so lam is
    the same bit for bit; dL/domega is summed over other block partials (bounded on the scale of its terms)."""
    print(f"adjoint launch shapes {shape} storage={storage}", flush=True)
    f = fields(shape, 59)
    h = make_handle(shape, tau=0.7, storage=storage)
    W0 = gpu_init(h, f)
    S_prev = h.empty_field()
    mlbm.mlbm_step_post(h, W0, 2, states=torch.empty((2,) + tuple(W0.shape), dtype=W0.dtype, device="cuda"),
                        dst=S_prev, nstates=2)
    n = 4
    states = torch.empty((n - 1,) + tuple(W0.shape), dtype=W0.dtype, device="cuda")
    mlbm.mlbm_step_post(h, S_prev, n - 1, states=states, src_post=True, nstates=n - 1)
    lamN = from_pauli(h, np.random.default_rng(10).standard_normal((4, h.Q) + tuple(shape)))
    scale = n * float(lamN.abs().sum()) * float(S_prev.abs().max())
    ref = dref = None
    for stores in (0, 1):
        for bx in (64, 128):
            for order in (mlbm.MLBM_ORDER_NATURAL, mlbm.MLBM_ORDER_XCD_RANGE, mlbm.MLBM_ORDER_INTERLEAVE8):
                for cap in (0, 2):
                    mlbm.mlbm_set_adjoint_launch(h, mlbm.MLBM_ADJ_CHANNEL, bx, order, cap, stores)
                    lam = lamN.clone()
                    dom = torch.zeros(1, dtype=torch.float64, device="cuda")
                    mlbm.mlbm_adjoint_sweep_post(h, S_prev, states, n, lam, h.empty_field(), dom)
                    torch.cuda.synchronize()
                    if ref is None:
                        ref, dref = lam, dom.item()
                    else:
                        assert torch.equal(lam, ref), (stores, bx, order, cap)
                        assert abs(dom.item() - dref) <= 1e-13 * scale, (stores, bx, order, cap, dom.item(), dref)
    mlbm.mlbm_set_adjoint_launch(h)
