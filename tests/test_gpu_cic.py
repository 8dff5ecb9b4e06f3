"""CIC deposit parity: HIP fixed-point deposit against the oracle's CIC.

Tolerance derived from the arithmetic: each weight is rounded once to a multiple of 2^-40 of a
particle's mass (error <= 2^-41 per contribution), so a cell with c contributions differs from
the exact sum by <= c * 2^-41 particle masses plus FP64 rounding; in delta units this is scaled
by n^3 / np. The tests use atol = 64 * 2^-41 * n^3 / np (generous for <= 64 contributions).
"""
import numpy as np
import pytest

import inputs
from gpu_util import announce, dev, host, require_gpu
from oracle import deposit as odep

pytestmark = pytest.mark.gpu

from paper_1709_06350_amd import mr  # noqa: E402


def _gpu_cic(pos, n, mass=1.0):
    require_gpu()
    with mr.Context(n) as c:
        return host(c.deposit_cic(dev(pos), mass))


def _tol(n, npart):
    return 64 * 2.0 ** -41 * n ** 3 / npart


def _report(name, got, ref, n, npart):
    """Print the achieved error in delta units and in particle masses per cell (n^3 / np delta units)."""
    err = float(np.max(np.abs(got - ref)))
    announce(f"{name}: max |delta_gpu - delta_oracle| = {err:.3e} = {err * npart / n ** 3:.3e} particle masses "
             f"(tolerance {_tol(n, npart):.3e}; 1e-12 max rho would be {1e-12 * float(np.max(ref + 1.0)):.3e})")


def test_random_particles_match_oracle_loop():
    rng = np.random.default_rng(0)
    pos = rng.uniform(-5.0, 21.0, size=(500, 3))
    n = 16
    got = _gpu_cic(pos, n, mass=0.7)
    ref = odep.overdensity(odep.deposit_cic_loop(pos, n, 0.7))
    _report("cic random n=16", got, ref, n, 500)
    np.testing.assert_allclose(got, ref, atol=_tol(n, 500) + 1e-13)


def test_lattice_gives_exactly_zero_and_is_deterministic():
    n = 16
    pos = np.indices((n, n, n)).reshape(3, -1).T.astype(float)
    a = _gpu_cic(pos, n)
    assert np.all(a == 0.0)
    pz = inputs.zeldovich_particles(n, 2.0, 5, rms_disp=1.5)
    b1 = _gpu_cic(pz, n)
    b2 = _gpu_cic(pz, n)
    assert np.array_equal(b1, b2)


def test_zeldovich_matches_oracle_and_conserves_mass():
    n = 64
    announce("cic zeldovich n=64")
    pos = inputs.zeldovich_particles(n, 2.0, 1001, rms_disp=2.0)
    got = _gpu_cic(pos, n)
    ref = odep.overdensity(odep.deposit_cic(pos, n))
    _report("cic zeldovich n=64", got, ref, n, n ** 3)
    np.testing.assert_allclose(got, ref, atol=_tol(n, n ** 3) + 1e-13)
    assert abs(got.sum()) < 1e-9 * n ** 3


def test_error_paths():
    require_gpu()
    with mr.Context(8) as c:
        bad = np.zeros((4, 3))
        bad[1, 2] = np.nan
        with pytest.raises(mr.MRError):
            c.deposit_cic(dev(bad))
        with pytest.raises(mr.MRError):
            c.deposit_cic(dev(np.zeros((4, 3))), mass=-1.0)
