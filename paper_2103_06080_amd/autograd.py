"""torch.autograd.Function over the C ABI: forward = kzk_step, backward = kzk_adjoint.

The gradient of any loss of the final field with respect to the initial
field comes from the hand-written discrete adjoint of the whole march
(transposed FFTs, conjugate multipliers, WENO5 weight Jacobians and the
Lax-Friedrichs speed term), with checkpointed recomputation every `ckpt`
steps (0: the longest interval whose stored fields fit in half of the free
device memory, the whole march when it fits).  Only the loss itself is
differentiated by torch.
"""
from __future__ import annotations

import math

import torch


class KZKMarch(torch.autograd.Function):
    """u_end = march(u0) over steps first .. first + n_steps - 1 of `plan`."""

    @staticmethod
    def forward(ctx, u0, plan, first: int, n_steps: int, ckpt: int):
        u = u0.detach().contiguous().clone()
        plan.step(u, first, n_steps)
        ctx.save_for_backward(u0.detach().contiguous())
        ctx.plan, ctx.first, ctx.n_steps, ctx.ckpt = plan, first, n_steps, ckpt
        return u

    @staticmethod
    def backward(ctx, g):
        (u0,) = ctx.saved_tensors
        grad = ctx.plan.adjoint(u0, g.contiguous(), ctx.first, ctx.n_steps, ctx.ckpt)
        return grad, None, None, None, None


def march(u0, plan, first: int = 0, n_steps: int = 1, ckpt: int = 50):
    return KZKMarch.apply(u0, plan, first, n_steps, ckpt)


def ground_loss(u, problem, kappa: float = 20.0, window=(-2.0, 2.0)):
    """Ground-signature loss over the central y-window W = {y in [lo, hi)} x all tau:
    a softmax-smoothed peak overpressure plus the mean square,
        L = (1/kappa) log(mean_W exp(kappa u)) + mean_W u^2."""
    y = problem.y0 + (problem.L_y / problem.n_y) * torch.arange(problem.n_y, device=u.device, dtype=torch.float64)
    rows = torch.nonzero((y >= window[0]) & (y < window[1])).flatten()
    uw = u.view(problem.n_y, problem.n_tau).index_select(0, rows)
    n = uw.numel()
    return (torch.logsumexp(kappa * uw.flatten(), 0) - math.log(n)) / kappa + (uw * uw).sum() / n
