"""Density assignment (oracle; test infrastructure only).

The paper assigns particles to the mesh with a standard scheme (NGP, CIC or TSC; footnote
in Sec. I) and does not smooth further. Convention used here: mesh points sit at integer
coordinates in cell units and indices wrap periodically; a particle contributes
mass * prod_d w_d to the mesh points around it. Per axis, with b = floor(x) and f = x - b:

* NGP: weight 1 at the nearest point, b if f < 1/2 else b + 1 (a tie goes up);
* CIC: w = 1 - f at b and w = f at b + 1 (8 points);
* TSC: with i the NGP point and d = x - i in [-1/2, 1/2), weights (1/2 - d)^2 / 2, 3/4 - d^2,
  (1/2 + d)^2 / 2 at i - 1, i, i + 1 (27 points): the quadratic B-spline, which reproduces the
  particle's position as the weighted mean of the points and has variance 1/4.

delta = rho / <rho> - 1 (the paper's 1 + delta = rho/rho_bar).
"""
from __future__ import annotations

import itertools

import numpy as np

__all__ = ["axis_weights", "deposit_loop", "deposit", "deposit_cic_loop", "deposit_cic", "overdensity",
           "SCHEMES"]

SCHEMES = ("ngp", "cic", "tsc")


def deposit_cic_loop(pos, n: int, mass: float = 1.0) -> np.ndarray:
    """Brute-force per-particle loop (tiny inputs only)."""
    rho = np.zeros((n, n, n), dtype=np.float64)
    for x in np.asarray(pos, dtype=np.float64):
        base = [int(np.floor(c)) for c in x]
        frac = [float(c) - b for c, b in zip(x, base)]
        for corner in itertools.product((0, 1), repeat=3):
            w = mass
            idx = []
            for d in range(3):
                w *= frac[d] if corner[d] else (1.0 - frac[d])
                idx.append((base[d] + corner[d]) % n)
            rho[idx[0], idx[1], idx[2]] += w
    return rho


def deposit_cic(pos, n: int, mass: float = 1.0) -> np.ndarray:
    """Vectorised CIC (same definition as ``deposit_cic_loop``), accumulation by np.add.at."""
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    base = np.floor(pos)
    frac = pos - base
    base = base.astype(np.int64)
    rho = np.zeros(n * n * n, dtype=np.float64)
    for corner in itertools.product((0, 1), repeat=3):
        w = np.full(pos.shape[0], mass, dtype=np.float64)
        flat = np.zeros(pos.shape[0], dtype=np.int64)
        for d in range(3):
            w = w * (frac[:, d] if corner[d] else (1.0 - frac[:, d]))
            flat = flat * n + np.mod(base[:, d] + corner[d], n)
        np.add.at(rho, flat, w)
    return rho.reshape(n, n, n)


def axis_weights(x, scheme: str):
    """Per-axis assignment of coordinates x (any shape): (first point, weights[..., S]) with
    S = 1, 2, 3 points starting at the returned integer index (not yet wrapped)."""
    x = np.asarray(x, dtype=np.float64)
    b = np.floor(x)
    f = x - b                                # exact
    if scheme == "cic":
        return b.astype(np.int64), np.stack([1.0 - f, f], axis=-1)
    up = f >= 0.5
    i = b + up                               # nearest point, ties up
    if scheme == "ngp":
        return i.astype(np.int64), np.ones(x.shape + (1,))
    if scheme == "tsc":
        d = f - up                           # x - i, exact
        w = np.stack([0.5 * (0.5 - d) ** 2, 0.75 - d * d, 0.5 * (0.5 + d) ** 2], axis=-1)
        return (i - 1).astype(np.int64), w
    raise ValueError(f"unknown scheme {scheme!r}")


def deposit_loop(pos, n: int, mass: float = 1.0, scheme: str = "cic") -> np.ndarray:
    """Brute-force per-particle loop for any scheme (tiny inputs only)."""
    rho = np.zeros((n, n, n), dtype=np.float64)
    for x in np.asarray(pos, dtype=np.float64).reshape(-1, 3):
        first, w = zip(*(axis_weights(c, scheme) for c in x))
        npt = w[0].shape[-1]
        for off in itertools.product(range(npt), repeat=3):
            rho[(first[0] + off[0]) % n, (first[1] + off[1]) % n, (first[2] + off[2]) % n] += (
                mass * w[0][off[0]] * w[1][off[1]] * w[2][off[2]])
    return rho


def deposit(pos, n: int, mass: float = 1.0, scheme: str = "cic") -> np.ndarray:
    """Vectorised deposit (same definition as ``deposit_loop``), accumulation by np.add.at."""
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    first, w = axis_weights(pos, scheme)      # [np, 3], [np, 3, S]
    npt = w.shape[-1]
    rho = np.zeros(n * n * n, dtype=np.float64)
    for off in itertools.product(range(npt), repeat=3):
        ww = np.full(pos.shape[0], mass, dtype=np.float64)
        flat = np.zeros(pos.shape[0], dtype=np.int64)
        for d in range(3):
            ww = ww * w[:, d, off[d]]
            flat = flat * n + np.mod(first[:, d] + off[d], n)
        np.add.at(rho, flat, ww)
    return rho.reshape(n, n, n)


def overdensity(rho: np.ndarray) -> np.ndarray:
    """delta = rho / <rho> - 1."""
    return rho / rho.mean() - 1.0
