"""Nonlinear multigrid (FAS V-cycle, red-black Newton-Gauss-Seidel) -- oracle, test infrastructure only.

Follows Sec. II.A.2 (Gauss-Seidel relaxation, Eq. 17 with dL/dtheta = -6/h^2, red-black
chessboard ordering, initial guess theta = 0, periodic boundaries, residual epsilon) and
Sec. II.A.3 (restriction by averaging the 8 son cells, the coarse equation Eq. 19, the
correction Eq. 20, V-cycles down to a 4^3 mesh).

Readings where the paper is silent or garbled:
  * the level equation is the mean-projected operator = f (see ``operator.projected_operator``);
  * the coarse equation uses the coarse operator on the restricted solution,
    L^H[R theta_hat] - R d (the printed Eq. 19 writes L^h inside, a misprint), and the
    coarse density is R delta;
  * prolongation P is trilinear interpolation between cell centres (the paper only
    specifies R);
  * within one colour every cell is updated from the same snapshot (Jacobi within a
    colour), red ((i+j+k) even) first; the uniform shift <Sigma> is taken from the snapshot;
  * coarsening continues while the coarse mesh is even and at least 4 cells wide
    (4^3 for powers of two, 6^3 for 96^3); the coarsest mesh gets nu_c red-black sweeps;
  * convergence is tested on ||r|| / ||r(theta = 0)|| on the finest mesh (the paper uses
    the absolute rms residual < 1e-8 in code units); the gauge <theta> = 0 is fixed at the end.

A second ordering, ``ordering="4c"``, splits a sweep into 4 sub-sweeps (the paper suggests
this as a possible improvement in Sec. II.A.2 and does not pursue it). Its classes are
c = 2 ((j + k) mod 2) + ((i + k) mod 2): a face step changes one parity of i, j, k and an
edge step two, and in either case (j + k, i + k) mod 2 changes, so no cell of the 19-point
stencil shares the class of its centre. Within a sub-sweep the sources therefore stay fixed
and the snapshot update is an exact Gauss-Seidel sub-sweep in any cell order.
"""
from __future__ import annotations

import numpy as np

from .operator import defect, laplacian, projected_operator, residual_norm, source

__all__ = [
    "restrict",
    "prolong",
    "red_mask",
    "four_colour_classes",
    "class_sweep",
    "sweep",
    "level_sizes",
    "half_sweep",
    "rb_sweep",
    "vcycle",
    "solve",
]


def restrict(a: np.ndarray) -> np.ndarray:
    """R: coarse value = average of its 8 son cells (Sec. II.A.3)."""
    n = a.shape[0]
    m = n // 2
    return a.reshape(m, 2, m, 2, m, 2).mean(axis=(1, 3, 5))


def _prolong_1d(a: np.ndarray, axis: int) -> np.ndarray:
    # Fine cell 2I sits a quarter coarse cell below the centre of coarse cell I, fine cell
    # 2I+1 a quarter above: linear weights 3/4 on the own coarse cell, 1/4 on the neighbour.
    lo = 0.75 * a + 0.25 * np.roll(a, 1, axis=axis)
    hi = 0.75 * a + 0.25 * np.roll(a, -1, axis=axis)
    shape = list(a.shape)
    shape[axis] *= 2
    out = np.empty(shape, dtype=a.dtype)
    sl_lo = [slice(None)] * a.ndim
    sl_hi = [slice(None)] * a.ndim
    sl_lo[axis] = slice(0, None, 2)
    sl_hi[axis] = slice(1, None, 2)
    out[tuple(sl_lo)] = lo
    out[tuple(sl_hi)] = hi
    return out


def prolong(a: np.ndarray) -> np.ndarray:
    """P: trilinear cell-centred interpolation from the coarse to the fine mesh."""
    out = a
    for ax in range(3):
        out = _prolong_1d(out, ax)
    return out


def red_mask(n: int) -> np.ndarray:
    """Chessboard colouring: red cells have (i + j + k) even (Sec. II.A.2)."""
    i, j, k = np.indices((n, n, n))
    return (i + j + k) % 2 == 0


def four_colour_classes(n: int) -> np.ndarray:
    """Class index 2 ((j + k) mod 2) + ((i + k) mod 2) of every cell (n even)."""
    i, j, k = np.indices((n, n, n))
    return 2 * ((j + k) % 2) + (i + k) % 2


def level_sizes(n: int):
    """Mesh sizes from the finest down: halve while the coarse mesh stays even and >= 4."""
    sizes = [n]
    while sizes[-1] % 2 == 0 and sizes[-1] // 2 >= 4 and (sizes[-1] // 2) % 2 == 0:
        sizes.append(sizes[-1] // 2)
    return sizes


def class_sweep(theta, delta, f, h, mask, m=None):
    """Newton-Gauss-Seidel update of the cells in ``mask`` from a snapshot (Sec. II.A.2, Eq. 17).

    theta_new = theta - L/(dL/dtheta) with dL/dtheta = -6/h^2 on the masked cells, where
    L = nabla^2 theta - (Sigma - m) - f is evaluated on the snapshot. ``m`` defaults to
    <Sigma> of the snapshot; it may be given explicitly.
    """
    sig = source(theta, delta, h)
    if m is None:
        m = sig.mean()
    L = laplacian(theta, h) - (sig - m)
    if f is not None:
        L = L - f
    new = theta - L / (-6.0 / (h * h))
    return np.where(mask, new, theta)


def half_sweep(theta, delta, f, h, red: bool, m=None):
    """One colour's update (red: (i + j + k) even) from a snapshot; see ``class_sweep``."""
    mask = red_mask(theta.shape[0])
    return class_sweep(theta, delta, f, h, mask if red else ~mask, m)


def rb_sweep(theta, delta, f, h, m=None):
    """A sweep: red sub-sweep then black sub-sweep (Sec. II.A.2)."""
    theta = half_sweep(theta, delta, f, h, True, m)
    theta = half_sweep(theta, delta, f, h, False, m)
    return theta


def sweep(theta, delta, f, h, m=None, ordering: str = "rb"):
    """A sweep in the given ordering: "rb" (red then black) or "4c" (classes 0, 1, 2, 3)."""
    if ordering == "rb":
        return rb_sweep(theta, delta, f, h, m)
    if ordering != "4c":
        raise ValueError(f"unknown ordering {ordering!r}")
    cls = four_colour_classes(theta.shape[0])
    for c in range(4):
        theta = class_sweep(theta, delta, f, h, cls == c, m)
    return theta


def vcycle(thetas, deltas, fs, level, nu1=2, nu2=2, nu_c=20, ordering="rb"):
    """FAS V-cycle on ``level`` (Sec. II.A.3, Eqs. 18-20). Updates thetas[level] in place."""
    h = float(2 ** level)
    th = thetas[level]
    if level == len(deltas) - 1:
        for _ in range(nu_c):
            th = sweep(th, deltas[level], fs[level], h, ordering=ordering)
        thetas[level] = th
        return
    for _ in range(nu1):
        th = sweep(th, deltas[level], fs[level], h, ordering=ordering)
    d = defect(th, deltas[level], fs[level], h)               # Eq. 18
    th_c = restrict(th)
    H = 2.0 * h
    fs[level + 1] = projected_operator(th_c, deltas[level + 1], H) - restrict(d)   # Eq. 19
    thetas[level + 1] = th_c.copy()
    vcycle(thetas, deltas, fs, level + 1, nu1, nu2, nu_c, ordering)
    th = th + prolong(thetas[level + 1] - th_c)               # Eq. 20
    for _ in range(nu2):
        th = sweep(th, deltas[level], fs[level], h, ordering=ordering)
    thetas[level] = th


def solve(delta: np.ndarray, tol: float = 1e-10, max_cycles: int = 100, nu1: int = 2,
          nu2: int = 2, nu_c: int = 20, theta0=None, ordering: str = "rb"):
    """Solve the mean-projected reconstruction equation for theta with <theta> = 0.

    Starts from theta = 0 (Sec. II.A.2) unless ``theta0`` is given (warm start). Returns
    (theta, info) with info = dict(cycles, rel_residual, history, m_shift, converged).
    """
    delta = np.asarray(delta, dtype=np.float64)
    n = delta.shape[0]
    sizes = level_sizes(n)
    deltas = [delta]
    for _ in sizes[1:]:
        deltas.append(restrict(deltas[-1]))
    thetas = [np.zeros_like(delta) if theta0 is None else np.array(theta0, dtype=np.float64)]
    thetas += [None] * (len(sizes) - 1)
    fs = [None] * len(sizes)

    r0 = residual_norm(projected_operator(np.zeros_like(delta), delta, 1.0))
    if r0 == 0.0:  # uniform density: theta = 0 solves the equation exactly (Sec. II, Eq. 6)
        r0 = 1.0
    rel = residual_norm(projected_operator(thetas[0], delta, 1.0)) / r0
    history = [rel]
    cycles = 0
    while rel > tol and cycles < max_cycles:
        vcycle(thetas, deltas, fs, 0, nu1, nu2, nu_c, ordering)
        cycles += 1
        rel = residual_norm(projected_operator(thetas[0], delta, 1.0)) / r0
        history.append(rel)
    theta = thetas[0] - thetas[0].mean()
    m_shift = float(source(theta, delta, 1.0).mean())
    return theta, dict(cycles=cycles, rel_residual=rel, history=history, m_shift=m_shift,
                       converged=bool(rel <= tol))
