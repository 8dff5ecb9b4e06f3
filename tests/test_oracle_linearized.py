"""Pins of the oracle Jacobian, its transpose and the adjoint gradient."""
import numpy as np
import pytest

import closed_forms as cf
import inputs
from oracle import linearized as lin
from oracle import multigrid as mg
from oracle import operator as op


def _state(n=8, seed=3):
    delta = inputs.lognormal(n, 0.6, 1.5, seed)
    theta = mg.solve(delta, tol=1e-13, max_cycles=80)[0]
    return delta, theta


@pytest.mark.parametrize("h", [1.0, 2.0])
def test_jacobian_matches_central_differences(h):
    delta, theta = _state()
    e = np.random.default_rng(1).standard_normal(theta.shape)
    eps = 1e-5
    fd = (op.projected_operator(theta + eps * e, delta, h)
          - op.projected_operator(theta - eps * e, delta, h)) / (2 * eps)
    J = lin.jacobian_apply(theta, delta, e, h)
    assert np.max(np.abs(J - fd)) < 1e-8 * np.max(np.abs(fd))


def test_stencil_form_equals_jacobian_and_transpose_is_adjoint():
    delta, theta = _state()
    rng = np.random.default_rng(2)
    e, u = rng.standard_normal((2,) + theta.shape)
    st = lin.stencil(theta, delta)
    Je = lin.apply_stencil(st, e)
    dS = op.laplacian(e, 1.0) - Je           # the unprojected dSigma(e)
    np.testing.assert_allclose(Je + dS.mean(), lin.jacobian_apply(theta, delta, e), atol=1e-12)
    np.testing.assert_allclose(np.vdot(u, Je), np.vdot(lin.apply_stencil_T(st, u), e), rtol=1e-12)
    Jm = lin.sparse_jacobian(st, theta.shape[0])
    np.testing.assert_allclose(Jm @ e.ravel(), Je.ravel(), atol=1e-12)


def test_projected_jacobian_annihilates_constants_both_sides():
    delta, theta = _state()
    one = np.ones_like(theta)
    assert np.max(np.abs(lin.jacobian_apply(theta, delta, one))) < 1e-12
    # J_p^T 1 = 0: every column of J_p sums to zero
    rng = np.random.default_rng(4)
    for _ in range(5):
        e = rng.standard_normal(theta.shape)
        assert abs(lin.jacobian_apply(theta, delta, e).sum()) < 1e-10


def test_adjoint_gradient_matches_finite_differences():
    n = 8
    delta, theta = _state(n, seed=5)
    theta_t = 0.5 * mg.solve(inputs.lognormal(n, 0.6, 1.5, 6), tol=1e-13)[0]
    g = lin.spectral_loss_grad(theta, theta_t)
    grad, _ = lin.adjoint_gradient(theta, delta, g)
    rng = np.random.default_rng(7)
    cells = rng.choice(n ** 3, 6, replace=False)
    eps = 1e-5
    for c in cells:
        dp = delta.copy().ravel()
        dm = delta.copy().ravel()
        dp[c] += eps
        dm[c] -= eps
        tp = mg.solve(dp.reshape(delta.shape), tol=1e-14, max_cycles=80, theta0=theta)[0]
        tm = mg.solve(dm.reshape(delta.shape), tol=1e-14, max_cycles=80, theta0=theta)[0]
        fd = (lin.spectral_loss(tp, theta_t) - lin.spectral_loss(tm, theta_t)) / (2 * eps)
        assert grad.ravel()[c] == pytest.approx(fd, rel=2e-5, abs=1e-7 * np.abs(grad).max())


def test_spectral_loss_gradient_matches_finite_differences():
    rng = np.random.default_rng(8)
    a, b = rng.standard_normal((2, 6, 6, 6))
    g = lin.spectral_loss_grad(a, b)
    e = rng.standard_normal(a.shape)
    eps = 1e-6
    fd = (lin.spectral_loss(a + eps * e, b) - lin.spectral_loss(a - eps * e, b)) / (2 * eps)
    assert np.vdot(g, e) == pytest.approx(fd, rel=1e-7)


def test_adjoint_poisson_limit():
    # Small delta: J -> discrete Laplacian, dSigma/ddelta -> 1, so dL/ddelta -> inv-Laplacian(g - <g>).
    n = 8
    delta = 1e-4 * inputs.lognormal(n, 0.5, 1.5, 9)
    theta = mg.solve(delta, tol=1e-13)[0]
    g = np.random.default_rng(10).standard_normal(delta.shape)
    grad, _ = lin.adjoint_gradient(theta, delta, g)
    expect = cf.poisson_fft(g)
    assert np.max(np.abs(grad - expect)) < 2e-3 * np.max(np.abs(expect))
