"""Pins of the oracle multigrid solve: closed forms, limits, invariants and brute force."""
import numpy as np
import pytest

import closed_forms as cf
import inputs
from oracle import multigrid as mg
from oracle import newton
from oracle import operator as op


def test_level_sizes():
    assert mg.level_sizes(32) == [32, 16, 8, 4]
    assert mg.level_sizes(96) == [96, 48, 24, 12, 6]
    assert mg.level_sizes(512)[-1] == 4 and len(mg.level_sizes(512)) == 8
    assert mg.level_sizes(20) == [20, 10]


def test_restriction_and_prolongation_basics():
    rng = np.random.default_rng(0)
    a = rng.standard_normal((8, 8, 8))
    np.testing.assert_allclose(mg.restrict(a)[1, 2, 3], a[2:4, 4:6, 6:8].mean(), rtol=1e-14)
    np.testing.assert_allclose(mg.prolong(np.full((4, 4, 4), 2.5)), 2.5, rtol=1e-15)
    # P reproduces a field linear in the coarse index away from the periodic seam:
    # coarse I has centre at fine coordinate 2I + 1/2, so fine cell i gets 0.5 * i - 0.25 + c.
    ci = np.indices((8, 8, 8))[0].astype(float)
    f = mg.prolong(ci)
    fi = np.indices((16, 16, 16))[0].astype(float)
    np.testing.assert_allclose(f[2:14], (0.5 * fi - 0.25)[2:14], atol=1e-14)
    # the 1D weights: fine cell 2I takes 3/4 of coarse I and 1/4 of coarse I-1
    e = np.zeros((4, 4, 4))
    e[1, 1, 1] = 1.0
    p = mg.prolong(e)
    assert p[2, 2, 2] == pytest.approx(27 / 64)
    assert p[1, 2, 2] == pytest.approx(9 / 64)
    assert p[1, 1, 2] == pytest.approx(3 / 64)
    assert p[1, 1, 1] == pytest.approx(1 / 64)
    assert p.sum() == pytest.approx(8.0)


def test_uniform_density_gives_zero_potential():
    theta, info = mg.solve(np.zeros((8, 8, 8)))
    assert np.all(theta == 0.0) and info["cycles"] == 0


@pytest.mark.parametrize("n", [16, 32])
def test_separable_closed_form(n):
    delta, exact = cf.separable_case(n)
    theta, info = mg.solve(delta, tol=1e-13, max_cycles=60)
    assert info["converged"]
    np.testing.assert_allclose(theta, exact, atol=1e-10 * np.abs(exact).max())
    assert abs(info["m_shift"]) < 1e-12
    # both branches of the root are exercised by this case
    T2, T3 = op.invariants(exact, 1.0)
    p, q = op.cubic_coefficients(T2, T3, delta)
    disc = q * q / 4 + p ** 3 / 27
    assert (disc < 0).mean() > 0.05 and (disc >= 0).mean() > 0.05


def test_separable_iso_q_lines():
    # Sec. III.A: iso-q lines are uniform / q_x depends only on x for a separable density.
    delta, _ = cf.separable_case(16)
    theta, _ = mg.solve(delta, tol=1e-13, max_cycles=60)
    gx = (np.roll(theta, -1, 0) - np.roll(theta, 1, 0)) / 2.0
    assert np.max(np.abs(gx - gx[:, :1, :1])) < 1e-9


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_plane_wave_closed_form(axis):
    delta, exact = cf.plane_wave_case(16, axis=axis)
    theta, info = mg.solve(delta, tol=1e-13, max_cycles=60)
    np.testing.assert_allclose(theta, exact, atol=1e-10 * np.abs(exact).max())


def test_manufactured_solution():
    delta, exact = cf.manufactured_case(16)
    theta, info = mg.solve(delta, tol=1e-13, max_cycles=80)
    assert info["converged"]
    np.testing.assert_allclose(theta, exact, atol=1e-9 * np.abs(exact).max())
    assert abs(info["m_shift"]) < 1e-11


def test_poisson_limit():
    d1 = inputs.lognormal(16, 0.5, 2.0, 5)
    lin = cf.poisson_fft(d1)
    errs = []
    for eps in (1e-2, 1e-3):
        theta, _ = mg.solve(eps * d1, tol=1e-12, max_cycles=60)
        errs.append(np.abs(theta / eps - lin).max() / np.abs(lin).max())
    assert errs[0] < 0.05 and errs[1] < 0.005 and errs[1] < errs[0] / 5


def test_brute_force_newton_8cubed():
    delta = inputs.lognormal(8, 0.4, 1.5, 9)
    th_n, m_n, res = newton.newton_solve(delta)
    assert res < 1e-12
    th_mg, info = mg.solve(delta, tol=1e-14, max_cycles=80)
    np.testing.assert_allclose(th_mg, th_n - th_n.mean(), atol=1e-11 * np.abs(th_n).max())
    # m in the bordered system is the uniform shift, <Sigma> at the solution
    assert info["m_shift"] == pytest.approx(m_n, abs=1e-11)


def _solve16(delta):
    return mg.solve(delta, tol=1e-13, max_cycles=60)[0]


def test_equivariance_shift_permutation_reflection():
    delta = inputs.lognormal(16, 0.6, 2.0, 21)
    th = _solve16(delta)
    sh = _solve16(np.roll(delta, (3, -5, 2), axis=(0, 1, 2)))
    np.testing.assert_allclose(sh, np.roll(th, (3, -5, 2), axis=(0, 1, 2)), atol=1e-11)
    pm = _solve16(np.ascontiguousarray(np.transpose(delta, (2, 0, 1))))
    np.testing.assert_allclose(pm, np.transpose(th, (2, 0, 1)), atol=1e-11)
    rf = _solve16(np.ascontiguousarray(np.roll(delta[::-1], 1, axis=0)))
    np.testing.assert_allclose(rf, np.roll(th[::-1], 1, axis=0), atol=1e-11)


def test_solution_has_no_shell_crossing_and_zero_means():
    delta = inputs.config0_delta()
    theta, info = mg.solve(delta)
    assert info["converged"] and info["cycles"] <= 20
    assert abs(theta.mean()) < 1e-15
    r = op.projected_operator(theta, delta, 1.0)
    assert abs(r.mean()) < 1e-14
    A = np.eye(3) + op.hessian(theta, 1.0) + info["m_shift"] / 3.0 * np.eye(3)
    assert np.linalg.eigvalsh(A).min() > 0.0


def test_slab_residual_matches_full():
    delta = inputs.lognormal(16, 0.6, 2.0, 22)
    theta = 0.1 * np.random.default_rng(1).standard_normal(delta.shape)
    full = op.relative_residual(theta, delta)
    slab, m = op.relative_residual_slabs(theta, delta, slab=5)
    assert slab == pytest.approx(full, rel=1e-12)


@pytest.mark.parametrize("case", ["separable", "plane_wave", "manufactured"])
def test_literal_operator_vanishes_on_exact_solutions(case):
    """The paper's literal L^h = lap theta - Sigma (Sec. II.A.1, Eq. 15, no mean projection) is zero
    at every closed-form solution: there <Sigma> = 0, so it equals the projected operator."""
    make = {"separable": cf.separable_case, "plane_wave": cf.plane_wave_case,
            "manufactured": cf.manufactured_case}[case]
    delta, exact = make(16)
    L = op.operator_L(exact, delta, 1.0)
    assert np.abs(L).max() <= 1e-12 * max(1.0, np.abs(delta).max())


def test_literal_operator_differs_from_projected_by_the_uniform_shift():
    """On a generic field the literal operator at the projected solution is the constant -<Sigma>
    (reading: the literal periodic system has no exact solution), and its rms floors at |<Sigma>|."""
    delta = inputs.lognormal(16, 0.5, 2.0, 21)
    theta, info = mg.solve(delta, tol=1e-12)
    L = op.operator_L(theta, delta, 1.0)
    m = info["m_shift"]
    assert abs(m) > 1e-6
    np.testing.assert_allclose(L, -m, atol=1e-10)
    # pinned independently of the solve: sum of lap vanishes on a periodic mesh, so <L> = -<Sigma>
    assert abs(L.mean() + op.source(theta, delta, 1.0).mean()) < 1e-13
