"""Differentiable rollout: torch.autograd.Function over the library's step and
its hand-written adjoint, with checkpoints every K steps.

Loss: L = (1/N) sum_x |r(x, n) - r_target(x)|^2, r the Bloch vector of
rho(x) = sum_i W_i(x) after n steps (mlbm_spin_loss).  Backward: for each
K-step segment, newest first, one mlbm_adjoint_segment call recomputes the
segment's states from its checkpoint (one fused pass each) and runs the
adjoint steps in reverse, accumulating dL/domega on the device; dL/dtau =
-dL/domega / tau^2.  Memory: one checkpoint per segment plus K - 1 states.
"""
import torch

from . import mlbm


class MLBMRollout(torch.autograd.Function):
    """loss = MLBMRollout.apply(W0, tau, handle, nsteps, K, r_target).

    W0: field of the handle's storage type (F64 or F32); tau: scalar float64
    tensor; r_target: [3, *grid] float64 device tensor.  Gradients flow to W0
    (dL/da of every Pauli coefficient) and tau.
    """

    @staticmethod
    def forward(ctx, W0, tau, handle, nsteps, K, r_target):
        if K < 1 or nsteps < 0:
            raise ValueError("need K >= 1 and nsteps >= 0")
        mlbm.mlbm_set_tau(handle, float(tau))
        W = W0.detach().clone()
        scratch = torch.empty_like(W)
        ckpts = [W.clone()]
        done = 0
        while done < nsteps:
            n = min(K, nsteps - done)
            mlbm.mlbm_step(handle, W, scratch, n)
            done += n
            if done < nsteps:
                ckpts.append(W.clone())
        loss = torch.zeros(1, dtype=torch.float64, device=W.device)
        mlbm.mlbm_spin_loss(handle, W, r_target, loss=loss)
        ctx.handle, ctx.nsteps, ctx.K = handle, nsteps, K
        ctx.ckpts, ctx.final, ctx.r_target = ckpts, W, r_target
        ctx.tau = float(tau)
        ctx.tau_device = tau.device if torch.is_tensor(tau) else torch.device("cpu")
        return loss[0].clone()

    @staticmethod
    def backward(ctx, gL):
        h, K, nsteps = ctx.handle, ctx.K, ctx.nsteps
        mlbm.mlbm_set_tau(h, ctx.tau)
        lam = torch.empty_like(ctx.final)
        mlbm.mlbm_spin_loss(h, ctx.final, ctx.r_target, lam=lam)
        lam_tmp = torch.empty_like(lam)
        states = torch.empty((K - 1,) + tuple(lam.shape), dtype=lam.dtype, device=lam.device) if K > 1 else None
        domega = torch.zeros(1, dtype=torch.float64, device=lam.device)
        for s in range(len(ctx.ckpts) - 1, -1, -1):
            n = min(K, nsteps - s * K)
            mlbm.mlbm_adjoint_segment(h, ctx.ckpts[s], states, n, lam, lam_tmp, domega)
        grad_W0 = lam * gL.to(lam.dtype) if ctx.needs_input_grad[0] else None
        grad_tau = None
        if ctx.needs_input_grad[1]:
            grad_tau = (-domega[0] / ctx.tau ** 2 * gL).to(device=ctx.tau_device, dtype=torch.float64)
        return grad_W0, grad_tau, None, None, None, None


def rollout_loss(W0, tau, handle, nsteps, K, r_target):
    return MLBMRollout.apply(W0, tau, handle, nsteps, K, r_target)
