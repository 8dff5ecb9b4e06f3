"""Density assignment on the GPU (mr_deposit: NGP, CIC, TSC) against the oracle, and the
particles-per-cell convergence check (Sec. I footnote: 8N^3 particles on an N^3 mesh and N^3
particles on an 8N^3 mesh converge alike).

Tolerance derived from the arithmetic: each weight is rounded once to a multiple of 2^-40 of a
particle's mass (error <= 2^-41 per contribution), so a cell with c contributions differs from
the exact sum by <= c * 2^-41 particle masses; in delta units this is scaled by n^3 / np. The
tests use atol = 64 * 2^-41 * n^3 / np (no cell here receives 64 contributions).
"""
import numpy as np
import pytest
import torch

import inputs
from gpu_util import announce, dev, host, require_gpu
from oracle import deposit as odep

pytestmark = pytest.mark.gpu

from paper_1709_06350_amd import mr  # noqa: E402

SCHEMES = ("ngp", "cic", "tsc")


def _tol(n, npart):
    return 64 * 2.0 ** -41 * n ** 3 / npart


@pytest.mark.parametrize("scheme", SCHEMES)
def test_random_particles_match_oracle_loop(scheme):
    require_gpu()
    n = 16
    rng = np.random.default_rng(30)
    pos = np.concatenate([rng.uniform(-5.0, 21.0, (600, 3)),
                          rng.integers(-16, 32, (40, 3)) + 0.5,          # NGP ties, TSC at d = -1/2
                          rng.integers(-16, 32, (40, 3)).astype(float),  # on mesh points
                          [[0.0, -1e-300, n - 1e-12]]])
    announce(f"deposit {scheme} random n={n}")
    with mr.Context(n) as c:
        got = host(c.deposit(dev(pos), 0.7, scheme))
    ref = odep.overdensity(odep.deposit_loop(pos, n, 0.7, scheme))
    np.testing.assert_allclose(got, ref, rtol=0, atol=_tol(n, pos.shape[0]) + 1e-13)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_zeldovich_64_matches_oracle_and_is_deterministic(scheme):
    require_gpu()
    n = 64
    announce(f"deposit {scheme} zeldovich n={n}")
    pos = inputs.zeldovich_particles(n, 2.0, 1001, rms_disp=2.0)
    with mr.Context(n) as c:
        d = dev(pos)
        a = host(c.deposit(d, 1.0, scheme))
        b = host(c.deposit(d, 1.0, scheme))
    np.testing.assert_array_equal(a, b)
    ref = odep.overdensity(odep.deposit(pos, n, 1.0, scheme))
    np.testing.assert_allclose(a, ref, rtol=0, atol=_tol(n, n ** 3) + 1e-13)
    assert abs(a.sum()) < 1e-9 * n ** 3


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("offset", [0.0, 0.25, 0.5])
def test_shifted_lattice_gives_exactly_zero(scheme, offset):
    """Every weight of these lattices is a multiple of 2^-15, so the fixed-point sums are exact."""
    require_gpu()
    n = 16
    pos = np.indices((n, n, n)).reshape(3, -1).T.astype(float) + offset
    with mr.Context(n) as c:
        got = host(c.deposit(dev(pos), 1.0, scheme))
    assert np.all(got == 0.0)


def test_cic_entry_point_equals_general_deposit():
    require_gpu()
    n = 32
    pos = inputs.zeldovich_particles(n, 2.0, 31, rms_disp=1.5)
    with mr.Context(n) as c:
        d = dev(pos)
        np.testing.assert_array_equal(host(c.deposit_cic(d, 1.3)), host(c.deposit(d, 1.3, "cic")))


def test_error_paths_leave_the_output_unchanged():
    require_gpu()
    n = 8
    with mr.Context(n) as c:
        bad = np.random.default_rng(32).uniform(0, n, (5, 3))
        bad[3, 1] = np.inf
        out = torch.full((n, n, n), 7.0, dtype=torch.float64, device="cuda")
        for scheme in SCHEMES:
            with pytest.raises(mr.MRError):
                c.deposit(dev(bad), 1.0, scheme, out=out)
        assert torch.all(out == 7.0)
        good = dev(np.zeros((4, 3)))
        assert c.lib.mr_deposit(c.h, good.data_ptr(), 4, 1.0, 7, out.data_ptr()) == mr.MR_EINVAL
        assert c.lib.mr_deposit(c.h, good.data_ptr(), 0, 1.0, mr.MR_DEPOSIT_TSC, out.data_ptr()) == mr.MR_EINVAL
        assert c.lib.mr_deposit(c.h, good.data_ptr(), 4, 0.0, mr.MR_DEPOSIT_NGP, out.data_ptr()) == mr.MR_EINVAL
        # a valid deposit after the failures works
        np.testing.assert_allclose(host(c.deposit(dev(np.indices((n, n, n)).reshape(3, -1).T.astype(float)),
                                                  1.0, "tsc")), 0.0, atol=0)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("scheme", ["cic", "tsc"])
def test_particles_per_cell_convergence(scheme):
    """The same 64^3 Zel'dovich particles deposited on 32^3, 64^3 and 128^3 meshes (8, 1 and 1/8
    particles per cell), smoothed with the same physical Gaussian radius and solved to 1e-8: the
    V-cycle counts stay close (the paper reports similar convergence for 8N^3 particles on N^3
    and N^3 on 8N^3). Parity unpinned: cycle counts have no independent value; the bound checked
    here (within a factor 1.5) is this test's reading of 'similar'."""
    require_gpu()
    npart = 64
    pos64 = inputs.zeldovich_particles(npart, 4.0, 1010, rms_disp=2.0)
    cycles = {}
    for m in (32, 64, 128):
        announce(f"particles per cell: {scheme} mesh {m}")
        pos = pos64 * (m / npart)
        with mr.Context(m, tol=1e-8) as c:
            d = host(c.deposit(dev(pos), 1.0, scheme))
            delta = inputs.normalise_density(inputs.gaussian_smooth(d + 1.0, 3.0 * m / npart))
            assert delta.min() > -1.0
            _, info = c.solve(dev(delta))
        assert info.status == 0 and info.rel_residual <= 1e-8
        cycles[m] = info.cycles
    print(f"{scheme}: V-cycles to 1e-8 by mesh (8, 1, 1/8 particles per cell): {cycles}")
    assert max(cycles.values()) <= 1.5 * min(cycles.values())


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("n,count", [(48, 2000), (8, 1), (96, 1), (32, 1), (64, 5), (256, 1)])
def test_ragged_meshes_and_single_particle(scheme, n, count):
    """Ragged meshes (scatter kernels) and a handful of particles, also on meshes of the tile-sorted
    form (n a multiple of 32: one block of the sort, almost every tile empty)."""
    require_gpu()
    announce(f"deposit {scheme} n={n} particles={count}")
    pos = np.random.default_rng(700 + n + count).uniform(-n, 2 * n, (count, 3))
    with mr.Context(n) as c:
        got = host(c.deposit(dev(pos), 2.5, scheme))
    ref = odep.overdensity(odep.deposit_loop(pos, n, 2.5, scheme) if count < 50 else odep.deposit(pos, n, 2.5, scheme))
    np.testing.assert_allclose(got, ref, rtol=0, atol=_tol(n, count) + 1e-13 * np.abs(ref).max())


def test_binding_rejects_mismatched_buffers_before_any_launch():
    """The kernels index the buffers by the mesh and particle counts; the binding checks them."""
    require_gpu()
    n = 8
    with mr.Context(n) as c:
        pos = dev(np.random.default_rng(1).uniform(0, n, (10, 3)))
        small = torch.zeros(n ** 3 - 1, dtype=torch.float64, device="cuda")
        with pytest.raises(ValueError):
            c.deposit(pos, 1.0, "cic", out=small)
        with pytest.raises(ValueError):
            c.deposit(dev(np.zeros(7)), 1.0, "ngp")
        theta = dev(np.zeros((n, n, n)))
        with pytest.raises(ValueError):
            c.lagrangian(theta, pos, out=torch.zeros((9, 3), dtype=torch.float64, device="cuda"))
        with pytest.raises(ValueError):
            c.lagrangian(dev(np.zeros((n, n, n - 2))), pos)
        with pytest.raises(ValueError):
            c.solve(dev(np.zeros((n, n, n + 2))))


@pytest.mark.parametrize("scheme", SCHEMES)
def test_deposit_is_independent_of_particle_order(scheme):
    """Lattice order sends most waves through the LDS-binned path, a random permutation sends them
    all to direct atomics; the fixed-point sums are order-independent, so both give the same delta
    bitwise (also with particles on the periodic seam and a few far outside the box)."""
    require_gpu()
    n = 64
    announce(f"deposit order independence {scheme}")
    pos = inputs.zeldovich_particles(n, 2.0, 1011, rms_disp=2.0)
    rng = np.random.default_rng(1012)
    pos[::997] = rng.uniform(-3 * n, 4 * n, pos[::997].shape)
    pos[5:9, 2] = [n - 1e-9, 0.0, -1e-12, n - 0.5]
    perm = rng.permutation(pos.shape[0])
    with mr.Context(n) as c:
        a = host(c.deposit(dev(pos), 1.0, scheme))
        b = host(c.deposit(dev(np.ascontiguousarray(pos[perm])), 1.0, scheme))
    assert np.array_equal(a, b)
    ref = odep.overdensity(odep.deposit(pos, n, 1.0, scheme))
    np.testing.assert_allclose(a, ref, rtol=0, atol=_tol(n, n ** 3) + 1e-13)


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("m,n", [(8, 8), (24, 32), (40, 48)])
def test_displaced_lattice_catalogues(scheme, m, n):
    """Catalogues of m^3 particles in lattice order (k fastest), displaced by up to a few cells and
    across the periodic seam, on meshes of the same and of other sizes: the binned deposit takes
    them in 2 x 4 x 8 lattice blocks per wave. Against the oracle, and bitwise against the same particles shuffled
    (whose waves reach boxes too large to bin and add directly)."""
    require_gpu()
    announce(f"deposit {scheme} lattice m={m} on n={n}")
    rng = np.random.default_rng(900 + m)
    pos = (np.indices((m, m, m)).reshape(3, -1).T + 0.5) * (n / m) + rng.normal(0.0, 0.7, (m ** 3, 3))
    perm = rng.permutation(m ** 3)
    with mr.Context(n) as c:
        a = host(c.deposit(dev(pos), 1.5, scheme))
        b = host(c.deposit(dev(np.ascontiguousarray(pos[perm])), 1.5, scheme))
    assert np.array_equal(a, b)
    ref = odep.overdensity(odep.deposit(pos, n, 1.5, scheme))
    np.testing.assert_allclose(a, ref, rtol=0, atol=_tol(n, m ** 3) + 1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("scheme", ["cic", "tsc"])
@pytest.mark.parametrize("n", [32, 128, 256])
def test_tile_sorted_deposit_equals_scatter_bitwise(scheme, n):
    """The tile-sorted deposit (counting sort by 16 x 16 x 32 mesh tile, LDS accumulation, no global
    atomics) against the atomic scatter kernels (MR_FLAG_DEPOSIT_SCATTER): the same rounded
    contribution per particle and point, summed exactly, so the same delta bit for bit; for a
    Zel'dovich catalogue in lattice order and shuffled, with particles on the seam and far outside."""
    require_gpu()
    announce(f"tile-sorted deposit {scheme} n={n}")
    m = n if n <= 128 else n // 2
    pos = inputs.zeldovich_particles(m, 2.0, 1300 + n, rms_disp=1.5) * (n / m)
    rng = np.random.default_rng(1400 + n)
    pos[::4999] = rng.uniform(-2 * n, 3 * n, pos[::4999].shape)
    pos[1:5, 0] = [n - 1e-9, 0.0, -1e-12, n - 0.5]
    shuffled = np.ascontiguousarray(pos[rng.permutation(pos.shape[0])])
    with mr.Context(n) as c:
        a = host(c.deposit(dev(pos), 1.0, scheme))
        b = host(c.deposit(dev(shuffled), 1.0, scheme))
        c.set_opts(flags=mr.MR_FLAG_DEPOSIT_SCATTER)
        s = host(c.deposit(dev(shuffled), 1.0, scheme))
    assert np.array_equal(a, b)
    assert np.array_equal(a, s)
    if n <= 128:
        ref = odep.overdensity(odep.deposit(pos, n, 1.0, scheme))
        np.testing.assert_allclose(a, ref, rtol=0, atol=_tol(n, pos.shape[0]) * 8 + 1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("scheme", ["cic", "tsc"])
def test_tile_sorted_deposit_clustered_and_empty_tiles(scheme):
    """Most particles in one tile (a tight clump across the seam of x), the rest in a few cells:
    one tile block takes a large share, most tiles are empty; against the scatter kernels and the
    oracle."""
    require_gpu()
    n = 64
    announce(f"tile-sorted deposit clustered {scheme}")
    rng = np.random.default_rng(77)
    clump = rng.normal(0.0, 1.2, (200000, 3)) + np.array([0.3, 20.0, 40.0])
    few = rng.uniform(0, n, (40, 3))
    pos = np.ascontiguousarray(np.concatenate([clump, few]))
    with mr.Context(n) as c:
        a = host(c.deposit(dev(pos), 2.0, scheme))
        c.set_opts(flags=mr.MR_FLAG_DEPOSIT_SCATTER)
        s = host(c.deposit(dev(pos), 2.0, scheme))
    assert np.array_equal(a, s)
    ref = odep.overdensity(odep.deposit(pos, n, 2.0, scheme))
    # every contribution is rounded by at most 2^-41 particle masses; at most all np particles
    # with 27 points each reach one cell
    np.testing.assert_allclose(a, ref, rtol=0, atol=27 * 2.0 ** -41 * pos.shape[0] * n ** 3 / pos.shape[0])
