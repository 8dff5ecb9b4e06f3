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
