"""torch.autograd.Function around the HIP solve and its adjoint (gradient with respect to delta).

forward: theta = solve(delta) by the FP64 (or mixed) multigrid of the given context.
backward: dL/ddelta from mr_adjoint_solve (transposed linearised multigrid, hierarchy rebuilt
from the saved theta and delta; no V-cycle state is stored between the two passes).
"""
from __future__ import annotations

import torch

from .mr import Context


class MongeAmpereSolve(torch.autograd.Function):
    @staticmethod
    def forward(fctx, delta: torch.Tensor, solver: Context):
        d = delta.detach().contiguous()
        theta, info = solver.solve(d)
        fctx.save_for_backward(d, theta)
        fctx.solver = solver
        fctx.info = info
        return theta

    @staticmethod
    def backward(fctx, gtheta: torch.Tensor):
        delta, theta = fctx.saved_tensors
        grad, _ = fctx.solver.adjoint_solve(delta, theta, gtheta.contiguous().to(torch.float64))
        return grad, None


def solve(delta: torch.Tensor, solver: Context) -> torch.Tensor:
    """Differentiable solve: returns theta(delta) with <theta> = 0."""
    return MongeAmpereSolve.apply(delta, solver)
