"""torch.autograd wrapper: total fluence as a differentiable function of the
per-voxel density scale.  Forward and backward both run in the library; the
backward call re-runs the forward solve and the adjoint solve, recomputing
every group's angular fluence instead of keeping it (checkpointing)."""
import torch

from .dsn import Problem


class DsnFluence(torch.autograd.Function):
    @staticmethod
    def forward(ctx, density, problem: Problem, source, solve_kw):
        problem.set_density(density.detach())
        out = problem.solve([source], **solve_kw)
        ctx.problem, ctx.source, ctx.solve_kw = problem, source, solve_kw
        ctx.save_for_backward(density.detach())
        return out["phi_total"][0]

    @staticmethod
    def backward(ctx, grad_phi):
        (density,) = ctx.saved_tensors
        problem = ctx.problem
        problem.set_density(density)
        kw = {k: v for k, v in ctx.solve_kw.items() if k in ("tol", "max_iters", "fixed_iters")}
        r = problem.adjoint(ctx.source, grad_phi.contiguous(), **kw)
        return r["grad"].to(density.dtype), None, None, None


def fluence(density, problem: Problem, source, **solve_kw):
    """phi_total [G][V] (cuda FP64) as a differentiable function of density [V]."""
    return DsnFluence.apply(density, problem, source, solve_kw)
