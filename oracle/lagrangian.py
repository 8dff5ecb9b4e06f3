"""Lagrangian mapping (oracle; test infrastructure only).

With Theta = Theta_0 + theta and Theta_0 = |x|^2 / 2 (Sec. II, the homogeneous solution), the
Lagrangian coordinate of an Eulerian point is q = grad Theta = x + grad theta, so the displacement
is psi = q - x = grad theta (equivalently x - q = -grad theta, Sec. III). On the mesh the
gradient is the second-order central difference of the discretisation section,
(theta(i+1) - theta(i-1)) / (2h) per axis, periodic; at a particle position the mesh field is
interpolated with the cloud-in-cell weights of the density assignment (mesh points at integer
coordinates, weight 1 - f at floor(x) and f at floor(x) + 1 per axis, f = x - floor(x)), i.e. the
transpose of the CIC deposit. Everything is in cell units (h = 1 unless given).
"""
from __future__ import annotations

import itertools

import numpy as np

__all__ = ["displacement_mesh", "gather_cic_loop", "gather_cic", "lagrangian_map"]


def displacement_mesh(theta: np.ndarray, h: float = 1.0) -> np.ndarray:
    """psi[i, j, k, a] = (theta(c + e_a) - theta(c - e_a)) / (2h), periodic."""
    theta = np.asarray(theta, dtype=np.float64)
    out = np.empty(theta.shape + (3,), dtype=np.float64)
    for a in range(3):
        out[..., a] = (np.roll(theta, -1, axis=a) - np.roll(theta, 1, axis=a)) / (2.0 * h)
    return out


def _base_frac(x: float, n: int):
    b = int(np.floor(x))
    return b % n, float(x) - b


def gather_cic_loop(field: np.ndarray, pos) -> np.ndarray:
    """Brute-force per-particle CIC interpolation of field[n, n, n, c] (tiny inputs only)."""
    n = field.shape[0]
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    out = np.zeros((pos.shape[0],) + field.shape[3:], dtype=np.float64)
    for p, x in enumerate(pos):
        bf = [_base_frac(c, n) for c in x]
        for corner in itertools.product((0, 1), repeat=3):
            w = 1.0
            idx = []
            for d in range(3):
                base, frac = bf[d]
                w *= frac if corner[d] else (1.0 - frac)
                idx.append((base + corner[d]) % n)
            out[p] += w * field[idx[0], idx[1], idx[2]]
    return out


def gather_cic(field: np.ndarray, pos) -> np.ndarray:
    """Vectorised CIC interpolation (same definition as ``gather_cic_loop``)."""
    n = field.shape[0]
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    base = np.floor(pos)
    frac = pos - base
    base = base.astype(np.int64)
    out = np.zeros((pos.shape[0],) + field.shape[3:], dtype=np.float64)
    for corner in itertools.product((0, 1), repeat=3):
        w = np.ones(pos.shape[0], dtype=np.float64)
        idx = []
        for d in range(3):
            w = w * (frac[:, d] if corner[d] else (1.0 - frac[:, d]))
            idx.append(np.mod(base[:, d] + corner[d], n))
        vals = field[idx[0], idx[1], idx[2]]
        out += w.reshape((-1,) + (1,) * (vals.ndim - 1)) * vals
    return out


def lagrangian_map(theta: np.ndarray, pos, h: float = 1.0):
    """Per-particle displacement psi(x_p) (q_p = x_p + psi(x_p)) and the mesh field psi."""
    psi = displacement_mesh(theta, h)
    return gather_cic(psi, pos), psi
