"""Mixed-precision form: FP32 linearised multigrid inside an FP64 defect-correction loop.

Binding check (same as FP64): the oracle-evaluated relative residual of the returned theta is
<= 1e-10. Reported error against the FP64 result: ||theta_mixed - theta_fp64|| / ||theta_fp64||,
bounded here by 1e-8 (both satisfy the same residual bound on a well-conditioned operator).
"""
import numpy as np
import pytest

import closed_forms as cf
import inputs
from gpu_util import announce, dev, host, require_gpu
from oracle import operator as oop

pytestmark = pytest.mark.gpu

from paper_1709_06350_amd import mr  # noqa: E402


def _solve(delta, **opts):
    require_gpu()
    with mr.Context(delta.shape[0], **opts) as c:
        theta, info = c.solve(dev(delta))
    return host(theta), info


@pytest.mark.parametrize("n,sigma,rc,seed", [(32, 0.5, 4.0, 1000), (48, 0.8, 3.0, 31), (64, 1.0, 2.0, 32)])
def test_mixed_matches_fp64_and_oracle(n, sigma, rc, seed):
    announce(f"mixed n={n} sigma={sigma}")
    delta = inputs.lognormal(n, sigma, rc, seed)
    tm, im = _solve(delta, precision=mr.PREC_MIXED)
    t64, i64 = _solve(delta)
    assert im.status == 0 and im.rel_residual <= 1e-10
    assert oop.relative_residual(tm, delta) <= 1e-10
    err = np.linalg.norm(tm - t64) / np.linalg.norm(t64)
    print(f"mixed vs fp64: rel L2 diff {err:.3e}, outer iterations {im.cycles}, fp64 cycles {i64.cycles}")
    assert err <= 1e-8
    assert im.m_shift == pytest.approx(i64.m_shift, abs=1e-10)


def test_mixed_separable_closed_form():
    delta, exact = cf.separable_case(32)
    theta, info = _solve(delta, precision=mr.PREC_MIXED, tol=1e-12, max_cycles=80)
    assert np.max(np.abs(theta - exact)) <= 1e-9 * np.abs(exact).max()


def test_mixed_two_inner_cycles_converge_in_fewer_outer_steps():
    delta = inputs.lognormal(32, 0.8, 3.0, 33)
    _, i1 = _solve(delta, precision=mr.PREC_MIXED, inner_cycles=1)
    _, i2 = _solve(delta, precision=mr.PREC_MIXED, inner_cycles=2)
    assert i1.status == 0 and i2.status == 0 and i2.cycles < i1.cycles
