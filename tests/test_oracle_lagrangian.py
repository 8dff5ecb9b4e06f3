"""Oracle Lagrangian mapping pinned to the mathematics.

- Closed form: for theta = A cos(2 pi m x / n) the central difference is exactly
  -A sin(2 pi m / n) sin(2 pi m i / n) along x (sum-to-product identity) and zero along y and z.
- Separable reduction: for a field that depends on x only, the 3D CIC interpolation reduces to
  1D linear interpolation (the y and z weights sum to one), and the other components vanish.
- Transpose identity: sum_p gather(f)(x_p) = sum_c f_c rho_c with rho the CIC deposit of the same
  particles (the deposit oracle, a separate implementation).
- Exactness: particles on mesh points return the mesh value; constant fields are reproduced;
  theta = 0 gives no displacement; a linear field along one axis is reproduced between points.
- The vectorised gather against the brute-force loop, including wrapped coordinates.
"""
import numpy as np
import pytest

from oracle import deposit as odep
from oracle import lagrangian as olag


def test_central_difference_closed_form():
    n, m, amp = 24, 3, 1.7
    i = np.arange(n)
    theta = np.broadcast_to(amp * np.cos(2 * np.pi * m * i / n)[:, None, None], (n, n, n)).copy()
    psi = olag.displacement_mesh(theta)
    ref = -amp * np.sin(2 * np.pi * m / n) * np.sin(2 * np.pi * m * i / n)
    np.testing.assert_allclose(psi[..., 0], np.broadcast_to(ref[:, None, None], (n, n, n)), rtol=0, atol=1e-14)
    assert np.abs(psi[..., 1]).max() == 0.0 and np.abs(psi[..., 2]).max() == 0.0
    # cell size h scales the gradient
    np.testing.assert_allclose(olag.displacement_mesh(theta, h=2.0), psi / 2.0, rtol=0, atol=1e-15)


def test_separable_field_reduces_to_linear_interpolation():
    n, m, amp = 16, 2, 0.9
    rng = np.random.default_rng(5)
    i = np.arange(n)
    theta = np.broadcast_to(amp * np.cos(2 * np.pi * m * i / n)[:, None, None], (n, n, n)).copy()
    grid = -amp * np.sin(2 * np.pi * m / n) * np.sin(2 * np.pi * m * i / n)   # closed form of psi_x
    pos = rng.uniform(-2 * n, 3 * n, size=(200, 3))
    disp, _ = olag.lagrangian_map(theta, pos)
    x0 = np.floor(pos[:, 0])
    f = pos[:, 0] - x0
    i0 = np.mod(x0.astype(np.int64), n)
    ref = (1 - f) * grid[i0] + f * grid[(i0 + 1) % n]
    np.testing.assert_allclose(disp[:, 0], ref, rtol=0, atol=1e-14)
    assert np.abs(disp[:, 1:]).max() <= 1e-15


def test_gather_is_the_transpose_of_the_deposit():
    n = 12
    rng = np.random.default_rng(7)
    f = rng.standard_normal((n, n, n))
    pos = rng.uniform(0, n, size=(300, 3))
    lhs = olag.gather_cic(f[..., None], pos)[:, 0].sum()
    rho = odep.deposit_cic(pos, n, 1.0)
    rhs = (f * rho).sum()
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_exact_cases():
    n = 10
    rng = np.random.default_rng(9)
    field = rng.standard_normal((n, n, n, 3))
    pts = rng.integers(-n, 2 * n, size=(50, 3)).astype(np.float64)
    out = olag.gather_cic(field, pts)
    idx = np.mod(pts.astype(np.int64), n)
    np.testing.assert_array_equal(out, field[idx[:, 0], idx[:, 1], idx[:, 2]])
    const = np.full((n, n, n, 3), 2.5)
    np.testing.assert_allclose(olag.gather_cic(const, rng.uniform(-5, 15, (40, 3))), 2.5, rtol=0, atol=1e-14)
    disp, psi = olag.lagrangian_map(np.zeros((n, n, n)), rng.uniform(0, n, (20, 3)))
    assert np.abs(disp).max() == 0.0 and np.abs(psi).max() == 0.0
    # linear along y between mesh points 3 and 4 (the field is linear there)
    lin = np.zeros((n, n, n, 1))
    lin[:, :, :, 0] = np.arange(n)[None, :, None].astype(np.float64)
    y = rng.uniform(3.0, 4.0, 30)
    p = np.stack([rng.uniform(0, n, 30), y, rng.uniform(0, n, 30)], axis=1)
    np.testing.assert_allclose(olag.gather_cic(lin, p)[:, 0], y, rtol=0, atol=1e-13)


def test_vectorised_gather_matches_loop():
    n = 6
    rng = np.random.default_rng(11)
    field = rng.standard_normal((n, n, n, 3))
    pos = np.concatenate([rng.uniform(-3 * n, 4 * n, (25, 3)), np.array([[0.0, n - 1e-12, 5.0], [-0.0, -1e-300, 2 * n]])])
    np.testing.assert_allclose(olag.gather_cic(field, pos), olag.gather_cic_loop(field, pos), rtol=0, atol=1e-14)
