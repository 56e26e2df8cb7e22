"""Differentiable rollout: torch.autograd.Function over the library's step and
its hand-written adjoint, with checkpoints every K steps.

Loss: L = (1/N) sum_x |r(x, n) - r_target(x)|^2, r the Bloch vector of
rho(x) = sum_i W_i(x) after n steps (mlbm_spin_loss).

Forward: one mlbm_step_states call per K-step segment writes the segment's
final pre-collision state straight into the next checkpoint (no copies, one
collide-only and one stream-only pass per segment besides the fused ones).
The last segment keeps all its post-collision states.

Backward, newest segment first: the last segment runs mlbm_adjoint_sweep on
the kept states; every earlier one runs mlbm_adjoint_segment, which
recomputes its states from the checkpoint (one fused pass each) into the same
buffer.  dL/domega accumulates on the device; dL/dtau = -dL/domega / tau^2.
Memory: one field per segment (checkpoints) plus K for the states.
"""
import torch

from . import mlbm


class MLBMRollout(torch.autograd.Function):
    """loss = MLBMRollout.apply(W0, tau, handle, nsteps, K, r_target).

    W0: field of the handle's storage type (F64 or F32; read, never written,
    and it must not change before backward); tau: scalar float64 tensor;
    r_target: [3, *grid] float64 device tensor.  Gradients flow to W0 (dL/da of
    every Pauli coefficient) and tau.
    """

    @staticmethod
    def forward(ctx, W0, tau, handle, nsteps, K, r_target):
        if K < 1 or nsteps < 0:
            raise ValueError("need K >= 1 and nsteps >= 0")
        mlbm.mlbm_set_tau(handle, float(tau))
        W = W0.detach()
        fshape = tuple(W.shape)
        nseg = -(-nsteps // K)
        ckpts = [W]                   # pre-collision state at the start of every segment (0: W0 itself)
        states = None
        final = W
        if nseg > 0:
            pair = torch.empty((2,) + fshape, dtype=W.dtype, device=W.device) if nseg > 1 else None
            states = torch.empty((max(K, 2),) + fshape, dtype=W.dtype, device=W.device)
            for s in range(nseg):
                n = min(K, nsteps - s * K)
                out = torch.empty_like(W)
                if s < nseg - 1:
                    mlbm.mlbm_step_states(handle, ckpts[-1], out, pair, n, nstates=2)
                    ckpts.append(out)
                else:
                    mlbm.mlbm_step_states(handle, ckpts[-1], out, states, n, nstates=n)
                    final = out
            del pair
        loss = torch.zeros(1, dtype=torch.float64, device=W.device)
        mlbm.mlbm_spin_loss(handle, final, r_target, loss=loss)
        ctx.handle, ctx.nsteps, ctx.K = handle, nsteps, K
        ctx.ckpts, ctx.final, ctx.r_target, ctx.states = ckpts, final, r_target, states
        ctx.states_kept = states is not None      # the last segment's states are in `states`
        ctx.save_for_backward(W0)                  # checkpoint 0 (autograd checks it was not modified)
        ctx.tau = float(tau)
        ctx.tau_device = tau.device if torch.is_tensor(tau) else torch.device("cpu")
        return loss[0].clone()

    @staticmethod
    def backward(ctx, gL):
        h, K, nsteps = ctx.handle, ctx.K, ctx.nsteps
        (W0,) = ctx.saved_tensors
        ckpts = [W0.detach()] + ctx.ckpts[1:]
        mlbm.mlbm_set_tau(h, ctx.tau)
        lam = torch.empty_like(ctx.final)
        mlbm.mlbm_spin_loss(h, ctx.final, ctx.r_target, lam=lam)
        lam_tmp = torch.empty_like(lam)
        domega = torch.zeros(1, dtype=torch.float64, device=lam.device)
        nseg = -(-nsteps // K)
        for s in range(nseg - 1, -1, -1):
            n = min(K, nsteps - s * K)
            if s == nseg - 1 and ctx.states_kept:
                mlbm.mlbm_adjoint_sweep(h, ckpts[s], ctx.states if n > 1 else None, n, lam, lam_tmp, domega)
                ctx.states_kept = False           # the recomputations below overwrite them
            else:
                mlbm.mlbm_adjoint_segment(h, ckpts[s], ctx.states if n > 1 else None, n, lam, lam_tmp,
                                          domega)
        grad_W0 = lam * gL.to(lam.dtype) if ctx.needs_input_grad[0] else None
        grad_tau = None
        if ctx.needs_input_grad[1]:
            grad_tau = (-domega[0] / ctx.tau ** 2 * gL).to(device=ctx.tau_device, dtype=torch.float64)
        return grad_W0, grad_tau, None, None, None, None


def rollout_loss(W0, tau, handle, nsteps, K, r_target):
    return MLBMRollout.apply(W0, tau, handle, nsteps, K, r_target)
