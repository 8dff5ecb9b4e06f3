"""Brute-force Newton on tiny meshes (oracle; test infrastructure only).

Unknowns (theta, m) with the equations nabla^2 theta - Sigma(theta) + m = 0 at every cell
(Sec. II.A.1, Eq. 15 with the uniform shift m of the mean-projection reading) and the gauge
sum(theta) = 0. The Jacobian is formed densely by central finite differences of the
residual, column by column, and Newton's method is iterated until the residual stops
decreasing. No multigrid, no relaxation, no shared code with ``multigrid``.
"""
from __future__ import annotations

import numpy as np

from .operator import laplacian, source

__all__ = ["bordered_residual", "newton_solve"]


def bordered_residual(x, delta):
    n = delta.shape[0]
    th = x[:-1].reshape(n, n, n)
    m = x[-1]
    F = laplacian(th, 1.0) - source(th, delta, 1.0) + m
    return np.concatenate([F.ravel(), [th.sum()]])


def newton_solve(delta, iters: int = 30, eps: float = 1e-6, theta0=None):
    """Returns (theta, m, final residual max-norm)."""
    delta = np.asarray(delta, dtype=np.float64)
    n = delta.shape[0]
    nn = n ** 3
    x = np.zeros(nn + 1)
    if theta0 is not None:
        x[:-1] = np.asarray(theta0).ravel()
    best = np.inf
    for _ in range(iters):
        F = bordered_residual(x, delta)
        res = np.max(np.abs(F))
        if res >= best and res < 1e-12:
            break
        best = min(best, res)
        Jm = np.empty((nn + 1, nn + 1))
        for j in range(nn + 1):
            xp = x.copy()
            xm = x.copy()
            xp[j] += eps
            xm[j] -= eps
            Jm[:, j] = (bordered_residual(xp, delta) - bordered_residual(xm, delta)) / (2 * eps)
        x = x - np.linalg.solve(Jm, F)
    F = bordered_residual(x, delta)
    return x[:-1].reshape(n, n, n), float(x[-1]), float(np.max(np.abs(F)))
