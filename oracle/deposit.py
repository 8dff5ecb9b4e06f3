"""Cloud-in-cell density assignment (oracle; test infrastructure only).

The paper assigns particles to the mesh with a standard scheme (NGP, CIC or TSC; footnote
in Sec. I) and does not smooth further. Convention used here: mesh points sit at integer
coordinates in cell units; a particle at x contributes mass * prod_d w_d to the 8 mesh
points around it, with w = 1 - f at floor(x) and w = f at floor(x) + 1, f = x - floor(x),
indices wrapped periodically. delta = rho / <rho> - 1 (the paper's 1 + delta = rho/rho_bar).
"""
from __future__ import annotations

import itertools

import numpy as np

__all__ = ["deposit_cic_loop", "deposit_cic", "overdensity"]


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


def overdensity(rho: np.ndarray) -> np.ndarray:
    """delta = rho / <rho> - 1."""
    return rho / rho.mean() - 1.0
