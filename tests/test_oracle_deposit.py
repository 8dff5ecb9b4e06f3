"""Pins of the oracle CIC deposit."""
import itertools

import numpy as np
import pytest

import inputs
from oracle import deposit as dep


def test_single_particle_hand_weights():
    x = np.array([[1.25, 2.5, 3.75]])
    rho = dep.deposit_cic_loop(x, 6, mass=2.0)
    wx = {1: 0.75, 2: 0.25}
    wy = {2: 0.5, 3: 0.5}
    wz = {3: 0.25, 4: 0.75}
    for i, j, k in itertools.product(wx, wy, wz):
        assert rho[i, j, k] == pytest.approx(2.0 * wx[i] * wy[j] * wz[k], abs=1e-15)
    assert rho.sum() == pytest.approx(2.0)
    assert np.count_nonzero(rho) == 8


def test_periodic_wrap():
    rho = dep.deposit_cic_loop(np.array([[5.5, 0.0, 5.9]]), 6)
    assert rho[5, 0, 5] == pytest.approx(0.5 * 0.1)
    assert rho[0, 0, 0] == pytest.approx(0.5 * 0.9)


def test_vectorised_matches_loop_and_conserves_mass():
    rng = np.random.default_rng(0)
    pos = rng.uniform(-3.0, 11.0, size=(300, 3))
    a = dep.deposit_cic_loop(pos, 8, 0.7)
    b = dep.deposit_cic(pos, 8, 0.7)
    np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-14)
    assert b.sum() == pytest.approx(300 * 0.7, rel=1e-13)


def test_undisplaced_lattice_is_uniform():
    pos = np.indices((8, 8, 8)).reshape(3, -1).T.astype(float)
    rho = dep.deposit_cic(pos, 8)
    np.testing.assert_array_equal(rho, 1.0)
    np.testing.assert_array_equal(dep.overdensity(rho), 0.0)


def test_integer_shift_equivariance():
    pos = inputs.zeldovich_particles(8, 2.0, 4, rms_disp=1.5)
    rho = dep.deposit_cic(pos, 8)
    rho_s = dep.deposit_cic(pos + np.array([2.0, -3.0, 5.0]), 8)
    np.testing.assert_allclose(rho_s, np.roll(rho, (2, -3, 5), axis=(0, 1, 2)), atol=1e-13)


# ---- NGP and TSC (standard assignment schemes named in Sec. I's footnote) ----------------------


def test_ngp_and_tsc_hand_weights():
    # NGP: nearest point per axis, a tie (fraction exactly 1/2) goes up
    rho = dep.deposit_loop(np.array([[2.3, 5.5, 7.7]]), 10, mass=1.5, scheme="ngp")
    assert rho[2, 6, 8] == 1.5 and np.count_nonzero(rho) == 1
    # TSC at x = 3.25: nearest point 3, d = 1/4, weights 1/32, 11/16, 9/32 (written out by hand)
    rho = dep.deposit_loop(np.array([[3.25, 4.0, 5.5]]), 10, scheme="tsc")
    wx = {2: 1 / 32, 3: 11 / 16, 4: 9 / 32}
    wy = {3: 1 / 8, 4: 3 / 4, 5: 1 / 8}           # d = 0
    wz = {5: 1 / 2, 6: 1 / 2, 7: 0.0}             # x = 5.5 rounds up to 6, d = -1/2
    for i, j, k in itertools.product(wx, wy, wz):
        assert rho[i, j, k] == pytest.approx(wx[i] * wy[j] * wz[k], abs=1e-16)
    assert np.count_nonzero(rho) == 18


@pytest.mark.parametrize("scheme", dep.SCHEMES)
def test_weight_moments(scheme):
    """Zeroth, first and second moments of one particle's weights about its position: the schemes
    are the box, tent and quadratic B-spline, so sum w = 1; CIC and TSC reproduce the position
    (sum w i = x); the second moment is f(1 - f) for CIC and exactly 1/4 for TSC; NGP's single
    point lies within 1/2."""
    rng = np.random.default_rng(21)
    n = 16
    ax = np.arange(n, dtype=np.float64)
    for x in np.concatenate([rng.uniform(3.0, 12.0, (40, 3)), [[4.5, 7.0, 9.999999999999998]]]):
        rho = dep.deposit_loop(x[None, :], n, scheme=scheme)
        assert rho.sum() == pytest.approx(1.0, abs=1e-14)
        for a in range(3):
            m = rho.sum(axis=tuple(b for b in range(3) if b != a))   # marginal along axis a
            mean = (m * ax).sum()
            var = (m * (ax - x[a]) ** 2).sum()
            f = x[a] - np.floor(x[a])
            if scheme == "ngp":
                assert abs(mean - x[a]) <= 0.5
            else:
                assert mean == pytest.approx(x[a], abs=1e-12)
            if scheme == "cic":
                assert var == pytest.approx(f * (1 - f), abs=1e-12)
            if scheme == "tsc":
                assert var == pytest.approx(0.25, abs=1e-12)


@pytest.mark.parametrize("scheme", dep.SCHEMES)
def test_schemes_vectorised_match_loop_conserve_mass_and_wrap(scheme):
    rng = np.random.default_rng(22)
    pos = np.concatenate([rng.uniform(-9.0, 17.0, (250, 3)),
                          rng.integers(-8, 16, (20, 3)) + 0.5,               # NGP ties, TSC d = -1/2
                          [[0.0, -1e-300, 7.999999999999999]]])
    a = dep.deposit_loop(pos, 8, 0.7, scheme)
    b = dep.deposit(pos, 8, 0.7, scheme)
    np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-14)
    assert b.sum() == pytest.approx(pos.shape[0] * 0.7, rel=1e-13)
    # shifting every particle by whole periods changes nothing
    c = dep.deposit(pos + 8.0 * rng.integers(-3, 4, pos.shape), 8, 0.7, scheme)
    np.testing.assert_allclose(c, b, rtol=0, atol=1e-13)


def test_cic_entry_points_agree_with_general_deposit():
    pos = np.random.default_rng(23).uniform(-4, 12, (200, 3))
    np.testing.assert_allclose(dep.deposit(pos, 8, 1.3, "cic"), dep.deposit_cic(pos, 8, 1.3), rtol=0, atol=1e-14)


@pytest.mark.parametrize("scheme", dep.SCHEMES)
@pytest.mark.parametrize("offset", [0.0, 0.5, 0.25])
def test_shifted_lattices_are_uniform(scheme, offset):
    """A lattice of one particle per cell, shifted by the same offset on every axis, deposits
    exactly one particle mass per point for every scheme (the weights of the particles that reach
    a point are the weights of one particle at all its offsets, which sum to one)."""
    pos = np.indices((8, 8, 8)).reshape(3, -1).T.astype(float) + offset
    rho = dep.deposit(pos, 8, 1.0, scheme)
    np.testing.assert_allclose(rho, 1.0, rtol=0, atol=1e-14)
