"""Differentiable rollout: torch.autograd.Function over the library's step and
its hand-written adjoint, with checkpoints every K steps.

Loss: L = (1/N) sum_x |r(x, n) - r_target(x)|^2, r the Bloch vector of
rho(x) = sum_i W_i(x) after n steps (mlbm_spin_loss).

Checkpoints are kept in post-collision form: the checkpoint of segment s >= 1
is the post-collision state of the step before it, from which the segment's
first pre-collision state is a pull away.  So the forward pass is one chain
of passes, one collide-only, n - 1 fused and one stream-only for the final
state, with the checkpoints written along the way (mlbm_step_post); the last
segment keeps all its post-collision states.

Backward, newest segment first: the last segment runs the adjoint sweep on
the kept states; every earlier one first recomputes its states from its
checkpoint (one pass each) into the same buffer.  Segment 0 starts from the
pre-collision W0 (mlbm_adjoint_sweep), the others from their post-collision
checkpoints (mlbm_adjoint_sweep_post).  dL/domega accumulates on the device;
dL/dtau = -dL/domega / tau^2.  Memory: one field per segment (checkpoints)
plus K for the states.
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
        ckpts = [None]                # post-collision checkpoint of every segment s >= 1
        states = None
        final = W
        if nseg > 0:
            pair = torch.empty((2,) + fshape, dtype=W.dtype, device=W.device) if nseg > 1 else None
            states = torch.empty((max(K, 2),) + fshape, dtype=W.dtype, device=W.device)
            last_post = torch.empty_like(W)
            for s in range(nseg):
                n = min(K, nsteps - s * K)
                src, post = (W, False) if s == 0 else (ckpts[s], True)
                if s < nseg - 1:
                    out = torch.empty_like(W)
                    mlbm.mlbm_step_post(handle, src, n, states=pair, dst=out, src_post=post, nstates=2)
                    ckpts.append(out)
                else:
                    mlbm.mlbm_step_post(handle, src, n, states=states if n > 1 else None, dst=last_post,
                                        src_post=post, nstates=max(n - 1, 1))
            del pair
            final = torch.empty_like(W)
            mlbm.mlbm_stream(handle, last_post, final)
            del last_post
        loss = torch.zeros(1, dtype=torch.float64, device=W.device)
        mlbm.mlbm_spin_loss(handle, final, r_target, loss=loss)
        ctx.handle, ctx.nsteps, ctx.K = handle, nsteps, K
        ctx.ckpts, ctx.final, ctx.r_target, ctx.states = ckpts, final, r_target, states
        ctx.states_kept = states is not None      # the last segment's states are in `states`
        ctx.save_for_backward(W0)                  # the first state (autograd checks it was not modified)
        ctx.tau = float(tau)
        ctx.tau_device = tau.device if torch.is_tensor(tau) else torch.device("cpu")
        return loss[0].clone()

    @staticmethod
    def backward(ctx, gL):
        h, K, nsteps = ctx.handle, ctx.K, ctx.nsteps
        (W0,) = ctx.saved_tensors
        W0 = W0.detach()
        mlbm.mlbm_set_tau(h, ctx.tau)
        lam = torch.empty_like(ctx.final)
        mlbm.mlbm_spin_loss(h, ctx.final, ctx.r_target, lam=lam)
        lam_tmp = torch.empty_like(lam)
        domega = torch.zeros(1, dtype=torch.float64, device=lam.device)
        nseg = -(-nsteps // K)
        for s in range(nseg - 1, -1, -1):
            n = min(K, nsteps - s * K)
            st = ctx.states if n > 1 else None
            if not (s == nseg - 1 and ctx.states_kept) and n > 1:
                # recompute the segment's post-collision states 0 .. n - 2 from its start
                src, post = (W0, False) if s == 0 else (ctx.ckpts[s], True)
                mlbm.mlbm_step_post(h, src, n - 1, states=ctx.states, src_post=post, nstates=n - 1)
            if s == nseg - 1:
                ctx.states_kept = False           # the recomputations below overwrite them
            if s == 0:
                mlbm.mlbm_adjoint_sweep(h, W0, st, n, lam, lam_tmp, domega)
            else:
                mlbm.mlbm_adjoint_sweep_post(h, ctx.ckpts[s], st, n, lam, lam_tmp, domega)
        grad_W0 = None
        if ctx.needs_input_grad[0]:
            # the usual cotangent of a scalar loss is exactly 1: then lam is the gradient itself
            grad_W0 = lam if float(gL) == 1.0 else lam * gL.to(lam.dtype)
        grad_tau = None
        if ctx.needs_input_grad[1]:
            grad_tau = (-domega[0] / ctx.tau ** 2 * gL).to(device=ctx.tau_device, dtype=torch.float64)
        return grad_W0, grad_tau, None, None, None, None


def rollout_loss(W0, tau, handle, nsteps, K, r_target):
    return MLBMRollout.apply(W0, tau, handle, nsteps, K, r_target)
