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
