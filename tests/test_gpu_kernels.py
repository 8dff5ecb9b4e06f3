"""Per-kernel parity: each building block of the HIP cycle against the oracle, element by element.

Sizes span several tiles and a ragged tile layout (48 = 3 x 16); h = 2 exercises the coarse-level
scaling and the FAS right-hand side f. Tolerance 1e-12 relative to the field's scale: both sides
evaluate the same closed-form expressions in FP64, so they differ by rounding order only (the
GPU's root is Newton-polished to ~1e-15 of the oracle's closed form).
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
    # a partially relaxed potential: a smooth field plus cell-level noise
    theta = amp * inputs.grf(n, 1.5, seed + 1) / inputs.grf(n, 1.5, seed + 1).std()
    theta += 0.02 * rng.standard_normal(theta.shape)
    return delta, theta


@pytest.fixture(scope="module")
def ctx():
    require_gpu()
    with mr.Context(64) as c:
        yield c


@pytest.fixture(scope="module")
def ctx2():
    """Context whose sweeps use one launch per colour instead of the fused red-black launch."""
    require_gpu()
    with mr.Context(64, flags=mr.MR_FLAG_TWO_PASS) as c:
        yield c


def _close(a, b, scale, tol=1e-12):
    err = np.max(np.abs(a - b))
    assert err <= tol * scale, f"max abs diff {err:.3e} > {tol:.0e} * {scale:.3e}"


@pytest.mark.parametrize("two_pass", [False, True])
@pytest.mark.parametrize("n,h,with_f", [(16, 1.0, False), (32, 1.0, False), (48, 1.0, False),
                                        (32, 2.0, True), (64, 4.0, True), (8, 8.0, True), (128, 1.0, False),
                                        (128, 2.0, True)])
def test_sweep_matches_oracle(ctx, ctx2, two_pass, n, h, with_f):
    announce(f"sweep n={n} h={h} f={with_f} two_pass={two_pass}")
    if two_pass:
        ctx = ctx2
    delta, theta = _state(n, 100 + n)
    f = 0.05 * np.random.default_rng(n).standard_normal(theta.shape) if with_f else None
    C = 0.0123
    out, s = ctx.sweep(dev(delta), dev(theta), h=h, f=None if f is None else dev(f), cshift=C)
    got = host(out)
    ref = omg.rb_sweep(theta, delta, f, h, m=C)
    _close(got, ref, np.abs(ref).max())
    # accounted sum: red cells from the snapshot, black cells after the red update
    red = omg.red_mask(n)
    ff = 0.0 if f is None else f
    s_red = (oop.source(theta, delta, h) + ff)[red].sum()
    mid = omg.half_sweep(theta, delta, f, h, True, m=C)
    s_black = (oop.source(mid, delta, h) + ff)[~red].sum()
    assert abs(s - (s_red + s_black)) <= 1e-11 * (np.abs(oop.source(theta, delta, h)).sum() + 1)


def test_sweep_is_deterministic(ctx):
    delta, theta = _state(32, 5)
    a, s1 = ctx.sweep(dev(delta), dev(theta), cshift=0.01)
    b, s2 = ctx.sweep(dev(delta), dev(theta), cshift=0.01)
    assert np.array_equal(host(a), host(b)) and s1 == s2


def test_fused_and_two_pass_sweeps_agree(ctx, ctx2):
    """Same update, two schedules: the fused launch recomputes the halo red values of every tile in
    the neighbouring blocks (the root iteration depends on the cell only), so both agree to
    rounding (the compiler may contract a product into an FMA differently in the two kernels)."""
    delta, theta = _state(64, 9)
    a, s1 = ctx.sweep(dev(delta), dev(theta), cshift=0.004)
    b, s2 = ctx2.sweep(dev(delta), dev(theta), cshift=0.004)
    ha, hb = host(a), host(b)
    _close(ha, hb, np.abs(hb).max(), tol=1e-14)
    assert abs(s1 - s2) <= 1e-12 * (abs(s1) + 1.0)


@pytest.mark.parametrize("n,h,with_f", [(16, 1.0, False), (48, 2.0, True), (128, 1.0, False), (64, 2.0, True)])
def test_defect_restrict_matches_oracle(ctx, n, h, with_f):
    announce(f"defect_restrict n={n}")
    delta, theta = _state(n, 200 + n)
    f = 0.05 * np.random.default_rng(n).standard_normal(theta.shape) if with_f else None
    C = -0.021
    tc, dr = ctx.defect_restrict(dev(delta), dev(theta), h=h, f=None if f is None else dev(f), cshift=C)
    sig = oop.source(theta, delta, h)
    d = oop.laplacian(theta, h) - sig + C - (0.0 if f is None else f)
    _close(host(dr), omg.restrict(d), np.abs(d).max())
    _close(host(tc), omg.restrict(theta), np.abs(theta).max())


@pytest.mark.parametrize("n,h", [(8, 2.0), (24, 4.0), (64, 2.0), (128, 2.0)])
def test_tau_rhs_matches_oracle(ctx, n, h):
    announce(f"tau n={n}")
    delta, theta = _state(n, 300 + n)
    rd = 0.1 * np.random.default_rng(n).standard_normal(theta.shape)
    f, s = ctx.tau_rhs(dev(delta), dev(theta), dev(rd), h)
    sig = oop.source(theta, delta, h)
    ref = oop.laplacian(theta, h) - sig - rd
    _close(host(f), ref, np.abs(ref).max())
    assert abs(s - (sig + ref).sum()) <= 1e-11 * (np.abs(sig).sum() + 1)


# 8 and 48: one coarse cell per thread (coarse size does not divide 256); 32 ... 512: coarse rows
# staged in LDS (32: 16 rows per block, 512: one row segment per block, the 512^3 solve's finest)
@pytest.mark.parametrize("n", [8, 32, 48, 64, 128, 512])
def test_prolong_correct_and_restrict_match_oracle(ctx, n):
    announce(f"prolong/restrict n={n}")
    rng = np.random.default_rng(n)
    tc, that, th = rng.standard_normal((n // 2,) * 3), rng.standard_normal((n // 2,) * 3), rng.standard_normal((n,) * 3)
    out = host(ctx.prolong_correct(dev(tc), dev(that), dev(th)))
    _close(out, th + omg.prolong(tc - that), 10.0)
    _close(host(ctx.restrict(dev(th))), omg.restrict(th), 1.0)


def test_residual_matches_oracle():
    require_gpu()
    n = 32
    delta, theta = _state(n, 400)
    with mr.Context(n) as c:
        r, rel, ms = c.residual(dev(delta), dev(theta))
    ref = oop.projected_operator(theta, delta, 1.0)
    _close(host(r), ref, np.abs(ref).max())
    assert rel == pytest.approx(oop.relative_residual(theta, delta), rel=1e-12)
    assert ms == pytest.approx(oop.source(theta, delta, 1.0).mean(), rel=1e-12, abs=1e-15)
