"""The 4-class ordering of the FP64 smoother (MR_FLAG_ORDER4) against the oracle.

One sweep (four class sub-sweeps with an explicit shift) is compared element by element with the
oracle's sweep in the same ordering, to 1e-12 of the field's scale (both sides evaluate the same
expressions in FP64; they differ by rounding order only). Solves are compared on the fixed point,
which does not depend on the ordering (parity of the result, not of the cycle count).
"""
import numpy as np
import pytest

import inputs
from gpu_util import announce, dev, host, require_gpu
from oracle import multigrid as omg
from oracle import operator as oop

pytestmark = pytest.mark.gpu

from paper_1709_06350_amd import mr  # noqa: E402


def _state(n, seed, amp=0.3):
    delta = inputs.lognormal(n, 0.8, 2.0, seed)
    rng = np.random.default_rng(seed)
    theta = amp * inputs.grf(n, 1.5, seed + 1) / inputs.grf(n, 1.5, seed + 1).std()
    theta += 0.02 * rng.standard_normal(theta.shape)
    return delta, theta


@pytest.fixture(scope="module")
def ctx4():
    require_gpu()
    with mr.Context(64, flags=mr.MR_FLAG_ORDER4) as c:
        yield c


@pytest.mark.parametrize("n,h,with_f", [(8, 8.0, True), (16, 1.0, False), (32, 1.0, False), (48, 1.0, False),
                                        (32, 2.0, True), (64, 4.0, True), (128, 1.0, False)])
def test_order4_sweep_matches_oracle(ctx4, n, h, with_f):
    announce(f"order4 sweep n={n} h={h} f={with_f}")
    delta, theta = _state(n, 300 + n)
    f = 0.05 * np.random.default_rng(n + 7).standard_normal(theta.shape) if with_f else None
    C = 0.0117
    out, s = ctx4.sweep(dev(delta), dev(theta), h=h, f=None if f is None else dev(f), cshift=C)
    got = host(out)
    ref = omg.sweep(theta, delta, f, h, m=C, ordering="4c")
    scale = np.abs(ref).max()
    err = np.abs(got - ref).max()
    assert err <= 1e-12 * scale, f"max abs diff {err:.3e}"
    # the reported sum is that of the last sub-sweep: colour 0 from the state before it, colour 1
    # after its colour-0 cells were updated
    cls = omg.four_colour_classes(n)
    red = omg.red_mask(n)
    th = theta
    for c in range(3):
        th = omg.class_sweep(th, delta, f, h, cls == c, C)
    ff = 0.0 if f is None else f
    s_red = (oop.source(th, delta, h) + ff)[red].sum()
    mid = omg.class_sweep(th, delta, f, h, (cls == 3) & red, C)
    s_black = (oop.source(mid, delta, h) + ff)[~red].sum()
    assert abs(s - (s_red + s_black)) <= 1e-11 * (np.abs(oop.source(theta, delta, h)).sum() + 1)


def test_order4_sweep_is_deterministic(ctx4):
    delta, theta = _state(32, 6)
    a, s1 = ctx4.sweep(dev(delta), dev(theta), cshift=0.01)
    b, s2 = ctx4.sweep(dev(delta), dev(theta), cshift=0.01)
    assert np.array_equal(host(a), host(b)) and s1 == s2


@pytest.mark.parametrize("n,sigma,rc", [(32, 0.5, 4.0), (64, 1.0, 2.0)])
def test_order4_solve_reaches_the_red_black_fixed_point(n, sigma, rc):
    require_gpu()
    announce(f"order4 solve n={n}")
    delta = inputs.lognormal(n, sigma, rc, 1002)
    d = dev(delta)
    with mr.Context(n, tol=1e-10) as c:
        t_rb, i_rb = c.solve(d)
    with mr.Context(n, tol=1e-10, flags=mr.MR_FLAG_ORDER4) as c:
        t_4, i_4 = c.solve(d)
    assert i_rb.status == 0 and i_4.status == 0
    a, b = host(t_rb), host(t_4)
    rel = oop.residual_norm(oop.projected_operator(b, delta, 1.0)) / oop.residual_norm(
        oop.projected_operator(np.zeros_like(delta), delta, 1.0))
    assert rel <= 2e-10
    np.testing.assert_allclose(b, a, rtol=0, atol=1e-8 * np.abs(a).max())
    print(f"n={n} sigma_g={sigma}: V-cycles to 1e-10, red-black {i_rb.cycles}, 4 classes {i_4.cycles}")
