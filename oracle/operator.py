"""Discrete operator of the reconstruction equation (oracle; test infrastructure only).

Notation follows Sec. II of the paper: theta is the displacement potential with
Theta = x^2/2 + theta (Eq. 6-8), h the cell size of the mesh, delta the overdensity.
All fields are float64 [n][n][n] arrays, periodic, k fastest. Grid units: h = 1 on the
finest mesh and h = 2^l on level l, theta in units of (finest cell)^2.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "nb",
    "hessian",
    "laplacian",
    "traceless",
    "invariants",
    "cubic_coefficients",
    "largest_real_root",
    "source",
    "operator_L",
    "projected_operator",
    "defect",
    "residual_norm",
    "relative_residual",
    "relative_residual_slabs",
]


def nb(a: np.ndarray, di: int, dj: int, dk: int) -> np.ndarray:
    """Periodic neighbour field: nb(a, di, dj, dk)[i, j, k] = a[i+di, j+dj, k+dk]."""
    return np.roll(a, (-di, -dj, -dk), axis=(0, 1, 2))


def hessian(theta: np.ndarray, h: float) -> np.ndarray:
    """Second-order finite-difference Hessian, shape [..., 3, 3] (Sec. II.A.1, Eqs. 11-14).

    Diagonal entries are the 3-point second differences, the off-diagonal ones the
    4-point cross differences (theta(+,+) + theta(-,-) - theta(-,+) - theta(+,-)) / 4h^2.
    """
    c = theta
    h2 = h * h
    H = np.empty(theta.shape + (3, 3), dtype=np.float64)
    unit = ((1, 0, 0), (0, 1, 0), (0, 0, 1))
    for a in range(3):
        e = unit[a]
        H[..., a, a] = (nb(c, *e) + nb(c, *(-x for x in e)) - 2.0 * c) / h2
    for a in range(3):
        for b in range(a + 1, 3):
            ea, eb = np.array(unit[a]), np.array(unit[b])
            pp = nb(c, *(ea + eb))
            mm = nb(c, *(-ea - eb))
            mp = nb(c, *(-ea + eb))
            pm = nb(c, *(ea - eb))
            H[..., a, b] = (pp + mm - mp - pm) / (4.0 * h2)
            H[..., b, a] = H[..., a, b]
    return H


def laplacian(theta: np.ndarray, h: float) -> np.ndarray:
    """7-point Laplacian (Sec. II.A.1, Eq. 11)."""
    s = (nb(theta, 1, 0, 0) + nb(theta, -1, 0, 0) + nb(theta, 0, 1, 0) + nb(theta, 0, -1, 0)
         + nb(theta, 0, 0, 1) + nb(theta, 0, 0, -1))
    return (s - 6.0 * theta) / (h * h)


def traceless(H: np.ndarray) -> np.ndarray:
    """Barred (traceless) part of a Hessian: H = (1/3) I tr H + Hbar (Sec. II, Eq. 4)."""
    tr = np.trace(H, axis1=-2, axis2=-1)
    out = H.copy()
    for a in range(3):
        out[..., a, a] -= tr / 3.0
    return out


def invariants(theta: np.ndarray, h: float):
    """T2 = tr(Mbar^2) and T3 = tr(Mbar^3) of the barred Hessian (Sec. II, Eq. 9; Appendix A).

    Computed from the assembled 3x3 matrix rather than from the appendix's expanded
    stencils (the printed expansion of T3 has a misprinted cross term).
    """
    M = traceless(hessian(theta, h))
    T2 = np.einsum("...ij,...ji->...", M, M)
    T3 = np.einsum("...ij,...jk,...ki->...", M, M, M)
    return T2, T3


def cubic_coefficients(T2, T3, delta):
    """p = -(9/2) T2 and q = 9 T3 - 27 (1 + delta) of the cubic s^3 + p s + q = 0 (Sec. II, Eqs. 8-9)."""
    p = -4.5 * T2
    q = 9.0 * T3 - 27.0 * (1.0 + delta)
    return p, q


def largest_real_root(p, q):
    """Physical root s = nabla^2 theta + 3 of s^3 + p s + q = 0 (Sec. II, discriminant and Eq. 10).

    With Delta = q^2/4 + p^3/27: for Delta >= 0 the single real root (Cardano), written
    with the two cube roots' product fixed to -p/3 so that no cancellation occurs; for
    Delta < 0 the largest of the three real roots, 2 sqrt(-p/3) cos(sigma/3) with the
    paper's cos(sigma) = (3q/2p) sqrt(-3/p). Reading: the printed Delta < 0 branch is not a
    root of the cubic; the largest real root is the branch that is continuous across
    Delta = 0, equals 3 at p = 0, q = -27 (delta = 0, theta = 0) and is the only root for
    which the Jacobian of the mapping is positive definite (no shell crossing, Sec. II).
    """
    p = np.asarray(p, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    p, q = np.broadcast_arrays(p, q)
    disc = 0.25 * q * q + p * p * p / 27.0
    s = np.empty(p.shape, dtype=np.float64)

    one = disc >= 0.0
    if np.any(one):
        qq = q[one]
        pp = p[one]
        sq = np.sqrt(disc[one])
        sgn = np.where(qq > 0.0, -1.0, 1.0)  # sign of -q (use +1 at q = 0)
        A = np.cbrt(-0.5 * qq + sgn * sq)
        with np.errstate(divide="ignore", invalid="ignore"):
            B = np.where(A != 0.0, -pp / (3.0 * np.where(A != 0.0, A, 1.0)), 0.0)
        s[one] = A + B

    three = ~one
    if np.any(three):
        pp = p[three]
        qq = q[three]
        cos_sigma = (3.0 * qq / (2.0 * pp)) * np.sqrt(-3.0 / pp)
        sigma = np.arccos(np.clip(cos_sigma, -1.0, 1.0))
        s[three] = 2.0 * np.sqrt(-pp / 3.0) * np.cos(sigma / 3.0)
    return s


def source(theta: np.ndarray, delta: np.ndarray, h: float) -> np.ndarray:
    """Sigma = (physical root) - 3, the right-hand side of nabla^2 theta = ... (Sec. II, Eqs. 10, 15)."""
    T2, T3 = invariants(theta, h)
    p, q = cubic_coefficients(T2, T3, delta)
    return largest_real_root(p, q) - 3.0


def operator_L(theta: np.ndarray, delta: np.ndarray, h: float) -> np.ndarray:
    """The paper's discrete operator L^h[theta] = nabla^2 theta - Sigma (Sec. II.A.1, Eq. 15)."""
    return laplacian(theta, h) - source(theta, delta, h)


def projected_operator(theta: np.ndarray, delta: np.ndarray, h: float) -> np.ndarray:
    """Mean-projected operator nabla^2 theta - (Sigma - <Sigma>).

    Reading (discrete compatibility): on a periodic mesh the sum of the discrete Laplacian
    vanishes while the sum of Sigma does not, so the literal Eq. 15 has no exact periodic
    solution. The uniform part of the source is projected out; <Sigma> is an unknown
    uniform shift that the solve reports. Every closed-form case has <Sigma> = 0 at the
    solution, where this operator equals L^h.
    """
    sig = source(theta, delta, h)
    return laplacian(theta, h) - (sig - sig.mean())


def defect(theta, delta, f, h):
    """d = L[theta] - f for the level equation L[theta] = f (Sec. II.A.3, Eq. 18)."""
    d = projected_operator(theta, delta, h)
    if f is not None:
        d = d - f
    return d


def residual_norm(r: np.ndarray) -> float:
    """Euclidean norm sqrt(sum r^2) (the paper's rms epsilon times sqrt(N^3), Sec. II.A.2)."""
    return float(np.sqrt(np.sum(r * r)))


def relative_residual(theta: np.ndarray, delta: np.ndarray) -> float:
    """||r(theta)|| / ||r(0)|| on the finest mesh (h = 1), r the mean-projected residual."""
    r = projected_operator(theta, delta, 1.0)
    r0 = projected_operator(np.zeros_like(delta), delta, 1.0)
    return residual_norm(r) / residual_norm(r0)


def _source_slabs(theta, delta, h, slab, workers=1):
    n = theta.shape[0]
    out = np.empty_like(theta)

    def one(i0):
        i1 = min(n, i0 + slab)
        idx = np.arange(i0 - 1, i1 + 1)
        t = np.take(theta, idx, axis=0, mode="wrap")
        d = np.take(delta, idx, axis=0, mode="wrap")
        out[i0:i1] = source(t, d, h)[1:-1]

    starts = list(range(0, n, slab))
    if workers > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(workers) as ex:
            list(ex.map(one, starts))
    else:
        for i0 in starts:
            one(i0)
    return out


def relative_residual_slabs(theta: np.ndarray, delta: np.ndarray, slab: int = 16, workers: int = 1):
    """Same quantity as ``relative_residual`` evaluated slab by slab to bound memory on large meshes.

    Each slab of planes is padded with one periodic plane on either side; the padded
    planes are discarded after evaluation, so every kept cell sees its true neighbours.
    Slabs may be evaluated by several threads. Returns (relative residual, <Sigma(theta)>).
    """
    sig = _source_slabs(theta, delta, 1.0, slab, workers)
    lap = laplacian(theta, 1.0)
    r = lap - (sig - sig.mean())
    sig0 = _source_slabs(np.zeros_like(delta), delta, 1.0, slab, workers)
    r0 = -(sig0 - sig0.mean())
    return residual_norm(r) / residual_norm(r0), float(sig.mean())
