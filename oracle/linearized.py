"""Linearised operator, its transpose and the adjoint gradient (oracle; test infrastructure only).

Differentiating the physical root of the cubic s^3 + p s + q = 0 (Sec. II, Eqs. 8-10)
implicitly gives ds = -(s dp + dq) / (3 s^2 + p). With p = -(9/2) tr(Mbar^2),
q = 9 tr(Mbar^3) - 27 (1 + delta) and Mbar the barred Hessian (Eq. 4):

    dSigma = tr(W dMbar) + D d(delta),   W = (9 s Mbar - 27 Mbar^2) / (3 s^2 + p),
                                         D = 27 / (3 s^2 + p).

dMbar(e) is the barred discrete Hessian of the perturbation e (Eqs. 11-14), so the Jacobian
of the mean-projected operator nabla^2 theta - (Sigma - <Sigma>) is

    J_p e = nabla^2 e - dSigma(e) + <dSigma(e)>,

a 19-point stencil (centre, 6 faces, 12 edges) plus a rank-one mean term. J_p annihilates
constants and maps onto mean-free fields, so J_p^T annihilates constants too.

Adjoint of the solve theta(delta) (gauge <theta> = 0) for a loss with gradient g = dL/dtheta:
solve J_p^T lambda = g - <g>, then dL/d(delta) = D * (lambda - <lambda>).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .operator import (cubic_coefficients, hessian, laplacian, largest_real_root, nb,
                       traceless)

__all__ = [
    "linearisation",
    "jacobian_apply",
    "stencil",
    "apply_stencil",
    "apply_stencil_T",
    "sparse_jacobian",
    "adjoint_gradient",
    "spectral_loss",
    "spectral_loss_grad",
]


def linearisation(theta, delta, h):
    """Per-cell W (shape [..., 3, 3]), D = dSigma/d(delta), and the root s."""
    M = traceless(hessian(theta, h))
    M2 = np.einsum("...ij,...jk->...ik", M, M)
    T2 = np.trace(M2, axis1=-2, axis2=-1)
    T3 = np.einsum("...ij,...ji->...", M2, M)
    p, q = cubic_coefficients(T2, T3, delta)
    s = largest_real_root(p, q)
    den = 3.0 * s * s + p
    W = (9.0 * s[..., None, None] * M - 27.0 * M2) / den[..., None, None]
    D = 27.0 / den
    return W, D, s


def jacobian_apply(theta, delta, e, h=1.0):
    """J_p e for the mean-projected operator."""
    W, _, _ = linearisation(theta, delta, h)
    dM = traceless(hessian(e, h))
    dS = np.einsum("...ij,...ji->...", W, dM)
    return laplacian(e, h) - dS + dS.mean()


def stencil(theta, delta, h=1.0):
    """Unprojected J as {offset: coefficient field}: (J e)_c = sum_o a_o(c) e(c + o)."""
    W, _, _ = linearisation(theta, delta, h)
    Wb = traceless(W)
    h2 = h * h
    st = {(0, 0, 0): np.full(theta.shape, -6.0 / h2)}
    unit = np.eye(3, dtype=int)
    for a in range(3):
        c = (1.0 - Wb[..., a, a]) / h2
        st[tuple(unit[a])] = c
        st[tuple(-unit[a])] = c
    for a in range(3):
        for b in range(a + 1, 3):
            w = W[..., a, b] / (2.0 * h2)
            st[tuple(unit[a] + unit[b])] = -w
            st[tuple(-unit[a] - unit[b])] = -w
            st[tuple(unit[a] - unit[b])] = w
            st[tuple(-unit[a] + unit[b])] = w
    return st


def apply_stencil(st, e):
    out = np.zeros_like(e)
    for o, a in st.items():
        out += a * nb(e, *o)
    return out


def apply_stencil_T(st, lam):
    """(J^T lambda)_c = sum_o a_o(c - o) lambda(c - o)."""
    out = np.zeros_like(lam)
    for o, a in st.items():
        out += nb(a * lam, *(-x for x in o))
    return out


def sparse_jacobian(st, n):
    """Assemble the unprojected J as a CSR matrix over the flattened C-order grid."""
    idx = np.arange(n ** 3).reshape(n, n, n)
    rows, cols, vals = [], [], []
    for o, a in st.items():
        rows.append(idx.ravel())
        cols.append(nb(idx, *o).ravel())
        vals.append(a.ravel())
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n ** 3, n ** 3))


def adjoint_gradient(theta, delta, g):
    """dL/d(delta) for dL/dtheta = g at the solution theta of delta (finest mesh, h = 1).

    The adjoint equation J_p^T lambda = g - <g> is solved directly: for mean-free lambda,
    J_p^T lambda = J^T lambda, so the bordered system [[J^T, 1], [1^T, 0]] is used.
    Returns (dL/ddelta, lambda).
    """
    n = theta.shape[0]
    st = stencil(theta, delta, 1.0)
    J = sparse_jacobian(st, n)
    ones = np.ones((n ** 3, 1))
    A = sp.bmat([[J.T, sp.csr_matrix(ones)], [sp.csr_matrix(ones.T), None]], format="csc")
    rhs = np.concatenate([(g - g.mean()).ravel(), [0.0]])
    sol = spla.spsolve(A, rhs)
    lam = sol[:-1].reshape(n, n, n)
    lam = lam - lam.mean()
    _, D, _ = linearisation(theta, delta, 1.0)
    return D * lam, lam


def spectral_loss(theta, theta_t, n_cells_smooth=4.0):
    """L = sum_k W(k) |phi_hat - phi_t_hat|^2, W = exp(-(k * 4 cells)^2), unnormalised FFT."""
    n = theta.shape[0]
    k1 = 2.0 * np.pi * np.fft.fftfreq(n)
    k2 = k1[:, None, None] ** 2 + k1[None, :, None] ** 2 + k1[None, None, :] ** 2
    Wk = np.exp(-k2 * n_cells_smooth ** 2)
    d = np.fft.fftn(theta - theta_t)
    return float(np.sum(Wk * (d.real ** 2 + d.imag ** 2)))


def spectral_loss_grad(theta, theta_t, n_cells_smooth=4.0):
    """dL/dtheta = 2 N^3 Re ifftn(W * fftn(theta - theta_t))."""
    n = theta.shape[0]
    k1 = 2.0 * np.pi * np.fft.fftfreq(n)
    k2 = k1[:, None, None] ** 2 + k1[None, :, None] ** 2 + k1[None, None, :] ** 2
    Wk = np.exp(-k2 * n_cells_smooth ** 2)
    return 2.0 * n ** 3 * np.fft.ifftn(Wk * np.fft.fftn(theta - theta_t)).real
