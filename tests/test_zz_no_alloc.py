"""The allocation-free residual entry point against mr_residual, through the C ABI.

mr_residual_noalloc computes the mean-projected residual (Sec. II.A.1, Eq. 15 with the uniform
shift) on natural-order arrays with a fixed device scratch array and no allocation. Two calls in a
row on one device, the second on a smaller mesh (the scratch keeps the first call's sums, so the
second checks that what must start at zero is cleared), each compared with mr_residual of a
context of that size: r element-wise to 1e-12 of its scale (both evaluate the same FP64 expressions;
the uniform shift is summed in a different order), the relative norm and <Sigma> to 1e-12.
"""
import numpy as np
import pytest
import torch

import inputs
from gpu_util import announce, dev, host, require_gpu

pytestmark = pytest.mark.gpu

from paper_1709_06350_amd import mr  # noqa: E402


def _state(n, seed):
    delta = inputs.lognormal(n, 0.8, 2.0, seed)
    theta = inputs.grf(n, 1.5, seed + 1)
    theta *= 0.3 / theta.std()
    return delta, theta


def test_noalloc_residual_matches_mr_residual_on_two_calls():
    require_gpu()
    for n, seed in ((64, 31), (24, 32)):
        announce(f"noalloc residual n={n}")
        delta, theta = _state(n, seed)
        d, t = dev(delta), dev(theta)
        r_na = torch.full_like(d, np.nan)
        _, rel_na, ms_na = mr.residual_noalloc(d, t, r_na)
        with mr.Context(n) as c:
            r, rel, ms = c.residual(d, t)
        ref = host(r)
        got = host(r_na)
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.abs(ref).max()
        assert rel_na == pytest.approx(rel, rel=1e-12)
        assert ms_na == pytest.approx(ms, rel=1e-12, abs=1e-15)
    # without an output array: only the scalars
    _, rel2, ms2 = mr.residual_noalloc(d, t)
    assert rel2 == rel_na and ms2 == ms_na


def test_noalloc_rejects_sizes_beyond_the_maximum():
    require_gpu()
    d = torch.zeros(8, dtype=torch.float64, device="cuda")
    lib = mr.load()
    assert lib.mr_residual_noalloc(2, mr._ptr(d), mr._ptr(d), None, None, None, None) == mr.MR_EINVAL
    assert lib.mr_residual_noalloc(1026, mr._ptr(d), mr._ptr(d), None, None, None, None) == mr.MR_EINVAL
    assert b"outside" in lib.mr_last_error()
