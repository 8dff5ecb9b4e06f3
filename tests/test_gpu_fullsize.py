"""Full-size cases: the 256^3 particle -> CIC -> smoothing -> solve chain and the 512^3 lognormal
solve (FP64 and mixed precision), each checked by the oracle on properties computable at any
size: the oracle-evaluated relative residual of the GPU potential (the binding check) and the
oracle CIC on the same particles.
"""
import os

import numpy as np
import pytest

import inputs
from gpu_util import announce, dev, host, require_gpu
from oracle import deposit as odep
from oracle import operator as oop

pytestmark = pytest.mark.gpu

from paper_1709_06350_amd import mr  # noqa: E402

WORKERS = min(16, os.cpu_count() or 1)


@pytest.mark.timeout(900)
def test_zeldovich_256_cic_smooth_solve():
    require_gpu()
    n = 256
    announce("full-size 256^3: zeldovich particles")
    pos = inputs.zeldovich_particles(n, 2.0, 1001, rms_disp=2.0)
    with mr.Context(n) as c:
        d_gpu = host(c.deposit_cic(dev(pos)))
        announce("full-size 256^3: oracle CIC on sampled planes")
        # oracle CIC restricted to particles near 3 sampled planes (computable piecewise)
        for plane in (0, 97, 255):
            sel = np.abs(((pos[:, 0] - plane + n / 2) % n) - n / 2) < 1.0
            ref = odep.deposit_cic(pos[sel], n)[plane]
            ref_d = ref * n ** 3 / pos.shape[0] - 1.0
            np.testing.assert_allclose(d_gpu[plane], ref_d, atol=64 * 2.0 ** -41 + 1e-12)
        delta = inputs.normalise_density(inputs.gaussian_smooth(d_gpu + 1.0, 2.0))
        assert delta.min() > -1.0
        announce("full-size 256^3: solve")
        theta, info = c.solve(dev(delta))
    th = host(theta)
    assert info.status == 0 and info.rel_residual <= 1e-10
    rel, _ = oop.relative_residual_slabs(th, delta, slab=16, workers=WORKERS)
    print(f"256^3 chain: cycles={info.cycles} gpu_rel={info.rel_residual:.3e} oracle_rel={rel:.3e}")
    assert rel <= 1e-10


@pytest.mark.timeout(900)
def test_lognormal_512_fp64_and_mixed():
    require_gpu()
    n = 512
    announce("full-size 512^3: input")
    delta = inputs.config2_delta(n)
    d = dev(delta)
    with mr.Context(n) as c:
        t64, i64 = c.solve(d)
        h64 = host(t64)
        del t64
        c.set_opts(precision=mr.PREC_MIXED)
        tm, im = c.solve(d)
        hm = host(tm)
    assert i64.status == 0 and im.status == 0
    announce("full-size 512^3: oracle residuals")
    r64, _ = oop.relative_residual_slabs(h64, delta, slab=16, workers=WORKERS)
    rm, _ = oop.relative_residual_slabs(hm, delta, slab=16, workers=WORKERS)
    err = np.linalg.norm(hm - h64) / np.linalg.norm(h64)
    print(f"512^3: fp64 cycles={i64.cycles} oracle_rel={r64:.3e}; mixed outer={im.cycles} oracle_rel={rm:.3e}; "
          f"mixed vs fp64 rel L2 {err:.3e}")
    assert r64 <= 1e-10 and rm <= 1e-10 and err <= 1e-8


@pytest.mark.timeout(900)
def test_largest_mesh_1024_tiled_periodic_field():
    """The largest supported mesh, 1024^3, on a 256^3 lognormal field tiled 4 x 4 x 4. The field has
    period 256, and so must the solution: every cell's update depends only on its neighbourhood
    and the mesh-wide sums are shared. Checked: the oracle's relative residual of one 256^3 tile on
    its own periodic mesh (the same quantity as on the whole mesh) for the FP64 and the mixed solve;
    the other tiles equal the first; the 1024^3 adjoint of a tiled dL/dtheta equals, tile by tile, the
    256^3 adjoint (also on the GPU, whose parity is pinned by the oracle and finite-difference tests)."""
    require_gpu()
    n, t = 1024, 256
    announce("largest mesh 1024^3: input")
    d256 = inputs.lognormal(t, 1.0, 2.0, 1010)
    delta = np.tile(d256, (4, 4, 4))
    d = dev(delta)
    del delta
    g256 = np.random.default_rng(1011).standard_normal((t, t, t))
    g256 -= g256.mean()
    with mr.Context(n, tol=1e-10) as c:
        announce("largest mesh 1024^3: FP64 solve")
        th, i64 = c.solve(d)
        assert i64.status == 0 and i64.rel_residual <= 1e-10
        announce("largest mesh 1024^3: adjoint")
        c.set_opts(tol=1e-8)
        gd = dev(np.tile(g256, (4, 4, 4)))
        grad, ia = c.adjoint_solve(d, th, gd)
        assert ia.status == 0
        del gd
        tiles = [(0, 0, 0), (1, 2, 3), (3, 3, 3)]
        th_t = [host(th[a * t:(a + 1) * t, b * t:(b + 1) * t, e * t:(e + 1) * t]) for a, b, e in tiles]
        gr_t = [host(grad[a * t:(a + 1) * t, b * t:(b + 1) * t, e * t:(e + 1) * t]) for a, b, e in tiles]
        announce("largest mesh 1024^3: mixed solve")
        c.set_opts(tol=1e-10, precision=mr.PREC_MIXED)
        thm, im = c.solve(d)
        assert im.status == 0 and im.rel_residual <= 1e-10
        thm_t = host(thm[:t, :t, :t])
        del th, grad, thm
    announce("largest mesh: 256^3 adjoint reference")
    with mr.Context(t, tol=1e-10) as c:
        th256, _ = c.solve(dev(d256))
        c.set_opts(tol=1e-8)
        ref_grad, _ = c.adjoint_solve(dev(d256), th256, dev(g256))
        ref_grad = host(ref_grad)
    for k in range(1, len(tiles)):
        np.testing.assert_allclose(th_t[k], th_t[0], rtol=0, atol=1e-12 * np.abs(th_t[0]).max())
        np.testing.assert_allclose(gr_t[k], gr_t[0], rtol=0, atol=1e-12 * np.abs(gr_t[0]).max())
    announce("largest mesh: oracle residual of a tile")
    r64, _ = oop.relative_residual_slabs(th_t[0], d256, slab=16, workers=WORKERS)
    rm, _ = oop.relative_residual_slabs(thm_t, d256, slab=16, workers=WORKERS)
    gerr = np.linalg.norm(gr_t[0] - ref_grad) / np.linalg.norm(ref_grad)
    print(f"1024^3 tiled: fp64 cycles={i64.cycles} oracle_rel={r64:.3e}; mixed outer={im.cycles} oracle_rel={rm:.3e}; "
          f"adjoint cycles={ia.cycles} vs 256^3 adjoint rel L2 {gerr:.3e}")
    assert r64 <= 1e-10 and rm <= 1e-10 and gerr <= 1e-6


@pytest.mark.timeout(900)
def test_largest_mesh_1024_anderson():
    """The accelerated FP64 solve on the largest mesh (the same tiled field): it converges and each
    checked tile equals the first tile and the plain solve's tile."""
    require_gpu()
    import torch
    torch.cuda.empty_cache()
    n, t = 1024, 256
    announce("largest mesh 1024^3: Anderson solve")
    d256 = inputs.lognormal(t, 1.0, 2.0, 1010)
    d = dev(np.tile(d256, (4, 4, 4)))
    with mr.Context(n, tol=1e-10) as c:
        th, ip = c.solve(d)
        ref = host(th[:t, :t, :t])
        del th
        tha, ia = c.solve_anderson(d, depth=2)
        assert ip.status == 0 and ia.status == 0 and ia.rel_residual <= 1e-10
        tiles = [(0, 0, 0), (2, 1, 3)]
        got = [host(tha[a * t:(a + 1) * t, b * t:(b + 1) * t, e * t:(e + 1) * t]) for a, b, e in tiles]
        del tha
    del d
    torch.cuda.empty_cache()
    scale = np.abs(ref).max()
    np.testing.assert_allclose(got[1], got[0], rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(got[0], ref, rtol=0, atol=1e-8 * scale)
    print(f"1024^3 Anderson: {ia.cycles} cycles (plain {ip.cycles})")
