"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only synthesises input fields and particle sets. It contains none of the
reconstruction arithmetic (no stencil, no cubic root, no multigrid); both the CPU oracle
and the HIP path receive the same host arrays produced here.

Stand-ins for the paper's workloads (Sec. III uses N-body snapshots that are not
available here):
  * ``lognormal``   -- a smooth lognormal overdensity with the power-law-times-Gaussian
                       spectrum P(k) ~ k^-1.5 exp(-(k R_c)^2) (k in radians per cell);
  * ``zeldovich_particles`` -- one particle per cell on the integer lattice, displaced by
                       the Zel'dovich field psi = -grad inv-laplacian(delta_L) of a Gaussian
                       random field, rescaled to a chosen rms displacement;
  * ``gaussian_smooth`` -- multiplication by exp(-k^2 R^2 / 2) in Fourier space (the paper
                       smooths its density fields with a 2 Mpc/h Gaussian, Sec. III.C).
All arrays are float64, C-order [i][j][k] with k fastest, periodic.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "kgrid",
    "grf",
    "lognormal",
    "zeldovich_particles",
    "gaussian_smooth",
    "normalise_density",
    "batched_boxes",
    "config0_delta",
    "config2_delta",
]


def kgrid(n: int):
    """Wavenumber components (radians per cell) broadcastable over an n^3 grid."""
    k1 = 2.0 * np.pi * np.fft.fftfreq(n)
    kx = k1[:, None, None]
    ky = k1[None, :, None]
    kz = k1[None, None, :]
    return kx, ky, kz


def grf(n: int, r_c: float, seed: int, slope: float = -1.5) -> np.ndarray:
    """Zero-mean Gaussian random field with P(k) = |k|^slope * exp(-(|k| r_c)^2), P(0) = 0."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n, n, n))
    kx, ky, kz = kgrid(n)
    k = np.sqrt(kx * kx + ky * ky + kz * kz)
    with np.errstate(divide="ignore"):
        pk = np.where(k > 0, k ** slope * np.exp(-((k * r_c) ** 2)), 0.0)
    g = np.fft.ifftn(np.fft.fftn(w) * np.sqrt(pk)).real
    g -= g.mean()
    return np.ascontiguousarray(g)


def lognormal(n: int, sigma_g: float, r_c: float, seed: int) -> np.ndarray:
    """delta with 1+delta = exp(g - sigma_g^2/2), g a GRF with std sigma_g; <1+delta> = 1 exactly."""
    g = grf(n, r_c, seed)
    g *= sigma_g / g.std()
    one_plus = np.exp(g - 0.5 * sigma_g * sigma_g)
    one_plus /= one_plus.mean()
    return np.ascontiguousarray(one_plus - 1.0)


def zeldovich_particles(n: int, r_c: float, seed: int, rms_disp: float = 2.0) -> np.ndarray:
    """n^3 particle positions (cell units, in [0, n)) shaped [n^3, 3].

    Lattice points q sit at integer coordinates. The displacement is the Zel'dovich field
    psi_hat = i k delta_hat / k^2 of a GRF delta_L, rescaled so that rms |psi| = rms_disp.
    """
    d = grf(n, r_c, seed)
    dk = np.fft.fftn(d)
    kx, ky, kz = kgrid(n)
    k2 = kx * kx + ky * ky + kz * kz
    k2[0, 0, 0] = 1.0
    psi = []
    for kc in (kx, ky, kz):
        pk = 1j * kc * dk / k2
        pk[0, 0, 0] = 0.0
        psi.append(np.fft.ifftn(pk).real)
    psi = np.stack(psi, axis=-1)
    rms = np.sqrt((psi * psi).sum(axis=-1).mean())
    psi *= rms_disp / rms
    q = np.indices((n, n, n), dtype=np.float64).transpose(1, 2, 3, 0)
    x = np.mod(q + psi, float(n))
    return np.ascontiguousarray(x.reshape(-1, 3))


def gaussian_smooth(field: np.ndarray, radius: float) -> np.ndarray:
    """Multiply by exp(-k^2 radius^2 / 2) in Fourier space (k in radians per cell)."""
    n = field.shape[0]
    kx, ky, kz = kgrid(n)
    k2 = kx * kx + ky * ky + kz * kz
    out = np.fft.ifftn(np.fft.fftn(field) * np.exp(-0.5 * k2 * radius * radius)).real
    return np.ascontiguousarray(out)


def normalise_density(rho: np.ndarray) -> np.ndarray:
    """delta = rho / <rho> - 1 (plain normalisation used by the input recipes)."""
    return np.ascontiguousarray(rho / rho.mean() - 1.0)


def config0_delta() -> np.ndarray:
    """32^3 lognormal, sigma_g = 0.5, R_c = 4 cells, seed 1000."""
    return lognormal(32, 0.5, 4.0, 1000)


def config2_delta(n: int = 512) -> np.ndarray:
    """Lognormal with sigma_g = 1.0 and R_c = 2 cells, seed 1002 (512^3 by default)."""
    return lognormal(n, 1.0, 2.0, 1002)


def batched_boxes(nbox: int = 64, seed: int = 1003, sizes=(64, 96, 128), r_c: float = 4.0):
    """Box list for the batched workload: sizes drawn uniformly from ``sizes``, sigma_g ~ U[0.5, 1.2].

    Returns a list of (n, sigma_g, field_seed); fields come from ``lognormal(n, sigma_g, r_c, field_seed)``.
    """
    rng = np.random.default_rng(seed)
    out = []
    for b in range(nbox):
        n = int(sizes[int(rng.integers(0, len(sizes)))])
        s = float(rng.uniform(0.5, 1.2))
        out.append((n, s, seed * 1000 + b))
    return out
