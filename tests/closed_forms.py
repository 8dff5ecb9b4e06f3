"""Exact discrete solutions used to pin the oracle and the HIP path (test helpers).

Separable density (the smoothed form of the paper's cubic test, Sec. III.A): if
1 + delta = rx(i) ry(j) rz(k), each 1D factor of mean 1, then theta = gx(i) + gy(j) + gz(k)
with the 1D periodic second difference g(i+1) - 2 g(i) + g(i-1) = r(i) - 1 solves the
discrete equation exactly: every cross difference vanishes, the discrete Hessian is
diag(gx'', gy'', gz''), and det(I + H) = prod(1 + g'') = 1 + delta (Sec. II, Eq. 2).
The 1D Poisson problems are solved here with a dense periodic solve plus the gauge row.
"""
import numpy as np


def poisson_1d(rhs):
    """Mean-zero g with g(i+1) - 2 g(i) + g(i-1) = rhs(i) (periodic); rhs must have mean 0."""
    n = rhs.shape[0]
    A = np.zeros((n + 1, n + 1))
    for i in range(n):
        A[i, i] = -2.0
        A[i, (i + 1) % n] += 1.0
        A[i, (i - 1) % n] += 1.0
        A[i, n] = 1.0
        A[n, i] = 1.0
    sol = np.linalg.solve(A, np.concatenate([rhs, [0.0]]))
    return sol[:n]


def factor_1d(n, amp, seed, modes=3):
    """A smooth positive 1D density factor exp(sum of cosines), normalised to mean exactly 1."""
    rng = np.random.default_rng(seed)
    x = np.arange(n) * 2.0 * np.pi / n
    g = np.zeros(n)
    for m in range(1, modes + 1):
        g += amp / m * np.cos(m * x + rng.uniform(0, 2 * np.pi))
    r = np.exp(g)
    return r / r.mean()


def separable_case(n, amp=0.9, seed=7):
    """(delta, theta_exact) for a separable density."""
    rx, ry, rz = (factor_1d(n, amp, seed + a) for a in range(3))
    gx, gy, gz = (poisson_1d(r - 1.0) for r in (rx, ry, rz))
    one_plus = rx[:, None, None] * ry[None, :, None] * rz[None, None, :]
    theta = gx[:, None, None] + gy[None, :, None] + gz[None, None, :]
    return one_plus - 1.0, theta - theta.mean()


def plane_wave_case(n, amp=0.6, seed=3, axis=0):
    """(delta, theta_exact) for a density varying along one axis only."""
    r = factor_1d(n, amp, seed)
    g = poisson_1d(r - 1.0)
    shape = [1, 1, 1]
    shape[axis] = n
    one_plus = np.broadcast_to(r.reshape(shape), (n, n, n)).copy()
    theta = np.broadcast_to(g.reshape(shape), (n, n, n)).copy()
    return one_plus - 1.0, theta - theta.mean()


def manufactured_case(n, amp=0.12, seed=11):
    """(delta, theta_exact): smooth theta*, delta* = det(I + H_h theta*) - 1 by np.linalg.det."""
    rng = np.random.default_rng(seed)
    i, j, k = np.indices((n, n, n)) * (2.0 * np.pi / n)
    th = np.zeros((n, n, n))
    for _ in range(4):
        a, b, c = rng.integers(-2, 3, size=3)
        ph = rng.uniform(0, 2 * np.pi)
        th += np.cos(a * i + b * j + c * k + ph)
    th *= amp * (n / (2.0 * np.pi)) ** 2 / 8.0
    # discrete Hessian written out directly (independent of oracle.operator.hessian)
    def at(di, dj, dk):
        return np.roll(th, (-di, -dj, -dk), axis=(0, 1, 2))
    H = np.empty((n, n, n, 3, 3))
    H[..., 0, 0] = at(1, 0, 0) + at(-1, 0, 0) - 2 * th
    H[..., 1, 1] = at(0, 1, 0) + at(0, -1, 0) - 2 * th
    H[..., 2, 2] = at(0, 0, 1) + at(0, 0, -1) - 2 * th
    H[..., 0, 1] = H[..., 1, 0] = (at(1, 1, 0) + at(-1, -1, 0) - at(-1, 1, 0) - at(1, -1, 0)) / 4
    H[..., 0, 2] = H[..., 2, 0] = (at(1, 0, 1) + at(-1, 0, -1) - at(-1, 0, 1) - at(1, 0, -1)) / 4
    H[..., 1, 2] = H[..., 2, 1] = (at(0, 1, 1) + at(0, -1, -1) - at(0, -1, 1) - at(0, 1, -1)) / 4
    A = np.eye(3) + H
    evals = np.linalg.eigvalsh(A)
    assert evals.min() > 0.05, "manufactured theta must keep I + H positive definite"
    delta = np.linalg.det(A) - 1.0
    return delta, th - th.mean()


def poisson_fft(rhs):
    """Mean-zero solution of the 7-point discrete Laplacian = rhs - <rhs> (periodic, FFT)."""
    n = rhs.shape[0]
    k = 2.0 * np.pi * np.fft.fftfreq(n)
    eig = (2 * np.cos(k)[:, None, None] + 2 * np.cos(k)[None, :, None]
           + 2 * np.cos(k)[None, None, :] - 6.0)
    eig[0, 0, 0] = 1.0
    r = np.fft.fftn(rhs - rhs.mean()) / eig
    r[0, 0, 0] = 0.0
    return np.fft.ifftn(r).real
