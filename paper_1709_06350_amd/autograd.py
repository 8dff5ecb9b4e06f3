"""torch.autograd.Function around the HIP solve and its adjoint (gradient with respect to delta).

forward: theta = solve(delta) by the FP64 (or mixed) multigrid of the given context.
backward: dL/ddelta from mr_adjoint_solve (transposed linearised multigrid, hierarchy rebuilt
from the saved theta and delta; no V-cycle state is stored between the two passes). Optionally
both passes use Anderson-accelerated cycles.
"""
from __future__ import annotations

import torch

from .mr import Context


class MongeAmpereSolve(torch.autograd.Function):
    @staticmethod
    def forward(fctx, delta: torch.Tensor, solver: Context, anderson_depth: int = 0):
        d = delta.detach().contiguous()
        if anderson_depth > 0:
            theta, info = solver.solve_anderson(d, depth=anderson_depth)
        else:
            theta, info = solver.solve(d)
        fctx.save_for_backward(d, theta)
        fctx.solver = solver
        fctx.info = info
        fctx.anderson_depth = anderson_depth
        return theta

    @staticmethod
    def backward(fctx, gtheta: torch.Tensor):
        delta, theta = fctx.saved_tensors
        grad, _ = fctx.solver.adjoint_solve(delta, theta, gtheta.contiguous().to(torch.float64),
                                            anderson_depth=fctx.anderson_depth)
        return grad, None, None


def solve(delta: torch.Tensor, solver: Context, anderson_depth: int = 0) -> torch.Tensor:
    """Differentiable solve: returns theta(delta) with <theta> = 0. anderson_depth > 0 runs both
    the solve and the adjoint with Anderson-accelerated cycles (same results, fewer cycles)."""
    return MongeAmpereSolve.apply(delta, solver, anderson_depth)
