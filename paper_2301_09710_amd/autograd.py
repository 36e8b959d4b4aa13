"""Differentiable projector and unrolled EM on top of libspect.

The paper trains unrolled EM iterations end to end (Sec. II-B, Alg. 3), so
the projector has to be backpropagatable.  Because the back projector is the
exact adjoint of the forward projector (Eq. (2)), the gradient of either is
the other, and nothing has to be stored for the backward pass:

    project(x)      = A x,   d/dx <A x, g>  = A' g
    backproject(v)  = A' v,  d/dv <A' v, g> = A g

``em_step`` wraps one ML-EM update (Eq. (7)-(8) with beta -> 0) whose
backward is ``spect_em_step_vjp``: it recomputes the step's own projections
from the saved input iterate (four projector directions), so an unrolled
reconstruction keeps only its iterates x_k -- checkpointing across
iterations.  All arithmetic runs in the library's kernels; torch supplies
memory, streams and the autograd graph.
"""
from __future__ import annotations

import torch

from . import spect

__all__ = ["project", "backproject", "em_step", "unrolled_mlem"]


class _Project(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, plan):
        ctx.plan = plan
        return plan.forward(x.contiguous())

    @staticmethod
    def backward(ctx, g):
        return ctx.plan.back(g.contiguous()), None


class _BackProject(torch.autograd.Function):
    @staticmethod
    def forward(ctx, v, plan):
        ctx.plan = plan
        return plan.back(v.contiguous())

    @staticmethod
    def backward(ctx, g):
        return ctx.plan.forward(g.contiguous()), None


class _EMStep(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, y, plan, sens, r):
        x = x.contiguous()
        out = x.clone()
        plan.em_step(out, y, sens, r)
        ctx.plan, ctx.sens, ctx.r = plan, sens, r
        ctx.save_for_backward(x, y)
        return out

    @staticmethod
    def backward(ctx, g):
        x, y = ctx.saved_tensors
        gx, gy = ctx.plan.em_step_vjp(x, y, ctx.sens, g.contiguous(), ctx.r,
                                      need_gy=ctx.needs_input_grad[1])
        return gx, gy, None, None, None


def project(plan: "spect.Plan", x: torch.Tensor) -> torch.Tensor:
    """A x, differentiable in x (backward = A')."""
    return _Project.apply(x, plan)


def backproject(plan: "spect.Plan", v: torch.Tensor) -> torch.Tensor:
    """A' v, differentiable in v (backward = A)."""
    return _BackProject.apply(v, plan)


def em_step(plan: "spect.Plan", x: torch.Tensor, y: torch.Tensor, sens: torch.Tensor,
            r: torch.Tensor | None = None) -> torch.Tensor:
    """x * A'(y / (A x + r)) / sens, differentiable in x and y."""
    return _EMStep.apply(x, y, plan, sens, r)


def unrolled_mlem(plan: "spect.Plan", x0: torch.Tensor, y: torch.Tensor, sens: torch.Tensor,
                  r: torch.Tensor | None = None, iters: int = 10) -> torch.Tensor:
    """``iters`` ML-EM updates from x0, differentiable in x0 and y.  Autograd
    keeps one volume per iteration (the iterate); the backward pass of each
    step recomputes that step's projections."""
    x = x0
    for _ in range(iters):
        x = em_step(plan, x, y, sens, r)
    return x
