"""Lagrangian mapping on the GPU (mr_lagrangian) against the oracle.

The mesh displacement is compared bitwise (one subtraction and an exact halving per value on
both sides); per-particle displacements within 1e-13 of the field's scale (the 8-term CIC sums
may round in a different order). theta is a seeded synthetic field (the mapping is defined for
any potential), never a GPU solve, so no oracle input comes from the HIP path.
"""
import numpy as np
import pytest
import torch

import inputs
from gpu_util import announce, dev, host, require_gpu
from oracle import lagrangian as olag

pytestmark = pytest.mark.gpu

from paper_1709_06350_amd import mr  # noqa: E402


def _particles(n, count, seed):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(-1.5 * n, 2.5 * n, size=(count, 3))
    pos[:10] = rng.integers(-n, 2 * n, size=(10, 3))   # on mesh points (weights exactly 0 / 1)
    pos[10] = [0.0, n - 1e-12, -1e-300]               # at the periodic seam
    return pos


@pytest.mark.parametrize("n", [16, 32])
def test_lagrangian_matches_oracle(n):
    require_gpu()
    announce(f"lagrangian vs oracle n={n}")
    theta = np.random.default_rng(100 + n).standard_normal((n, n, n))
    pos = _particles(n, 5000, 200 + n)
    ref_disp, ref_psi = olag.lagrangian_map(theta, pos)
    with mr.Context(n) as c:
        disp, psi = c.lagrangian(dev(theta), dev(pos), want_psi=True)
        disp2, _ = c.lagrangian(dev(theta), dev(pos))           # without the mesh output
    np.testing.assert_array_equal(host(psi), ref_psi)
    scale = np.abs(ref_psi).max()
    np.testing.assert_allclose(host(disp), ref_disp, rtol=0, atol=1e-13 * scale)
    np.testing.assert_array_equal(host(disp2), host(disp))


def test_lagrangian_separable_closed_form():
    require_gpu()
    n, m, amp = 64, 3, 2.3
    announce("lagrangian separable closed form n=64")
    i = np.arange(n)
    theta = np.broadcast_to(amp * np.cos(2 * np.pi * m * i / n)[:, None, None], (n, n, n)).copy()
    grid = -amp * np.sin(2 * np.pi * m / n) * np.sin(2 * np.pi * m * i / n)
    pos = _particles(n, 4000, 7)
    with mr.Context(n) as c:
        disp, psi = c.lagrangian(dev(theta), dev(pos), want_psi=True)
    psi, disp = host(psi), host(disp)
    np.testing.assert_allclose(psi[..., 0], np.broadcast_to(grid[:, None, None], (n, n, n)), rtol=0, atol=1e-14)
    assert np.abs(psi[..., 1:]).max() == 0.0
    x0 = np.floor(pos[:, 0])
    f = pos[:, 0] - x0
    i0 = np.mod(x0.astype(np.int64), n)
    np.testing.assert_allclose(disp[:, 0], (1 - f) * grid[i0] + f * grid[(i0 + 1) % n], rtol=0, atol=1e-13)
    assert np.abs(disp[:, 1:]).max() <= 1e-14


@pytest.mark.timeout(600)
def test_lagrangian_256_zeldovich_particles_sampled():
    """The full-size workload: 256^3 Zel'dovich particles (one per cell) mapped through a smooth
    256^3 potential; the mesh field is compared in full, the particles on a random sample."""
    require_gpu()
    n = 256
    announce("lagrangian 256^3: inputs")
    theta = 40.0 * inputs.grf(n, 4.0, 1006)
    pos = inputs.zeldovich_particles(n, 2.0, 1001, rms_disp=2.0)
    with mr.Context(n) as c:
        announce("lagrangian 256^3: map")
        disp, psi = c.lagrangian(dev(theta), dev(pos), want_psi=True)
        disp, psi = host(disp), host(psi)
    announce("lagrangian 256^3: oracle")
    ref_psi = olag.displacement_mesh(theta)
    np.testing.assert_array_equal(psi, ref_psi)
    sample = np.random.default_rng(1007).choice(pos.shape[0], 20000, replace=False)
    ref = olag.gather_cic(ref_psi, pos[sample])
    np.testing.assert_allclose(disp[sample], ref, rtol=0, atol=1e-13 * np.abs(ref_psi).max())


def test_lagrangian_errors():
    require_gpu()
    n = 16
    theta = dev(np.zeros((n, n, n)))
    th = np.random.default_rng(3).standard_normal((n, n, n))
    theta = dev(th)
    with mr.Context(n) as c:
        bad = np.random.default_rng(4).uniform(0, n, (6, 3))
        bad[2, 1] = np.nan
        bad[4, 0] = np.inf
        out = torch.zeros((6, 3), dtype=torch.float64, device="cuda")
        with pytest.raises(mr.MRError):
            c.lagrangian(theta, dev(bad), out=out)
        # the finite particles are still mapped; the others receive NaN
        got = host(out)
        ok = [0, 1, 3, 5]
        ref, _ = olag.lagrangian_map(th, bad[ok])
        np.testing.assert_allclose(got[ok], ref, rtol=0, atol=1e-13 * 10)
        assert np.isnan(got[[2, 4]]).all()
        with pytest.raises(mr.MRError):
            c.lagrangian(theta, torch.zeros((0, 3), dtype=torch.float64, device="cuda"))


@pytest.mark.parametrize("n,count", [(48, 3000), (8, 1), (96, 1)])
def test_lagrangian_ragged_meshes_and_single_particle(n, count):
    """Non-power-of-two meshes (rows not a multiple of the block width) and a single particle."""
    require_gpu()
    announce(f"lagrangian n={n} particles={count}")
    theta = np.random.default_rng(500 + n).standard_normal((n, n, n))
    pos = _particles(n, max(count, 11), 600 + n)[:count] if count >= 11 else \
        np.random.default_rng(n).uniform(-n, 2 * n, (count, 3))
    ref_disp, ref_psi = olag.lagrangian_map(theta, pos)
    with mr.Context(n) as c:
        disp, psi = c.lagrangian(dev(theta), dev(pos), want_psi=True)
    np.testing.assert_array_equal(host(psi), ref_psi)
    np.testing.assert_allclose(host(disp), ref_disp, rtol=0, atol=1e-13 * np.abs(ref_psi).max())
