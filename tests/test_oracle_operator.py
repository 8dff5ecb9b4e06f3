"""Pins of the oracle's discrete operator against facts fixed by the paper and by algebra.

Nothing here compares the oracle with itself: each test checks an independent computation
(eigenvalues, determinants, numpy.roots, the appendix's expanded stencils, closed forms).
"""
import numpy as np
import pytest

from oracle import operator as op


def _rand_theta(n=8, amp=0.3, seed=0):
    return amp * np.random.default_rng(seed).standard_normal((n, n, n))


def test_invariants_equal_eigenvalue_power_sums():
    th = _rand_theta()
    T2, T3 = op.invariants(th, 1.0)
    M = op.traceless(op.hessian(th, 1.0))
    mu = np.linalg.eigvalsh(M)
    np.testing.assert_allclose(T2, (mu ** 2).sum(-1), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(T3, (mu ** 3).sum(-1), rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(mu.sum(-1), 0.0, atol=1e-12)


def test_barred_terms_do_not_depend_on_centre_cell():
    # Sec. II: the barred derivatives of cell (i,j,k) do not involve theta_ijk.
    th = _rand_theta()
    M0 = op.traceless(op.hessian(th, 1.0))[3, 4, 5]
    th[3, 4, 5] += 0.77
    M1 = op.traceless(op.hessian(th, 1.0))[3, 4, 5]
    np.testing.assert_allclose(M0, M1, atol=1e-14)


def _raw(th):
    def t(di, dj, dk):
        return np.roll(th, (-di, -dj, -dk), axis=(0, 1, 2))
    Sx = t(1, 0, 0) + t(-1, 0, 0)
    Sy = t(0, 1, 0) + t(0, -1, 0)
    Sz = t(0, 0, 1) + t(0, 0, -1)
    Dxy = t(1, 1, 0) + t(-1, -1, 0) - t(1, -1, 0) - t(-1, 1, 0)
    Dxz = t(1, 0, 1) + t(-1, 0, -1) - t(1, 0, -1) - t(-1, 0, 1)
    Dyz = t(0, 1, 1) + t(0, -1, -1) - t(0, -1, 1) - t(0, 1, -1)
    return Sx, Sy, Sz, Dxy, Dxz, Dyz


def test_appendix_T2_expansion():
    # Appendix A, first expression (h = 1), typed from the paper's expanded stencil.
    th = _rand_theta(seed=1)
    Sx, Sy, Sz, Dxy, Dxz, Dyz = _raw(th)
    T2_app = ((Sx + Sy - 2 * Sz) ** 2 + (Sy + Sz - 2 * Sx) ** 2 + (Sz + Sx - 2 * Sy) ** 2) / 9.0 \
        + (Dxy ** 2 + Dxz ** 2 + Dyz ** 2) / 8.0
    T2, _ = op.invariants(th, 1.0)
    np.testing.assert_allclose(T2, T2_app, rtol=1e-12, atol=1e-13)


def _appendix_T3(Sx, Sy, Sz, Dxy, Dxz, Dyz, third_cross):
    t = (Sx * (2 * Sx ** 2 + Sy ** 2 + Sz ** 2) + Sy * (2 * Sy ** 2 + Sz ** 2 + Sx ** 2)
         + Sz * (2 * Sz ** 2 + Sx ** 2 + Sy ** 2)) / 9.0
    t -= 2.0 / 9.0 * (Sx ** 2 * (Sy + Sz) + Sy ** 2 * (Sz + Sx) + Sz ** 2 * (Sx + Sy))
    t -= 2.0 / 9.0 * (Sx * (Sy - Sz) ** 2 + Sy * (Sz - Sx) ** 2 + Sz * (Sx - Sy) ** 2)
    t += ((Sx + Sy - 2 * Sz) * Dxy ** 2 + (Sz + Sx - 2 * Sy) * Dxz ** 2
          + (Sy + Sz - 2 * Sx) * third_cross ** 2) / 16.0
    t += 3.0 / 32.0 * Dxy * Dxz * Dyz
    return t


def test_appendix_T3_expansion_with_corrected_cross_term():
    # Appendix A, second expression. As printed, the third cross term squares D_xy; with
    # D_yz in its place the expansion equals tr(Mbar^3) of the assembled matrix.
    th = _rand_theta(seed=2)
    raw = _raw(th)
    _, T3 = op.invariants(th, 1.0)
    corrected = _appendix_T3(*raw, third_cross=raw[5])
    np.testing.assert_allclose(T3, corrected, rtol=1e-11, atol=1e-12)
    printed = _appendix_T3(*raw, third_cross=raw[3])
    assert np.max(np.abs(printed - T3)) > 1e-3


def test_determinant_expansion_identity():
    # Sec. II, Eq. 3: det A = (trA)^3/6 - tr(A^2) trA / 2 + tr(A^3)/3 for symmetric A.
    rng = np.random.default_rng(3)
    A = rng.standard_normal((200, 3, 3))
    A = A + np.swapaxes(A, 1, 2)
    tr = np.trace(A, axis1=1, axis2=2)
    tr2 = np.einsum("nij,nji->n", A, A)
    tr3 = np.einsum("nij,njk,nki->n", A, A, A)
    np.testing.assert_allclose(tr ** 3 / 6 - tr2 * tr / 2 + tr3 / 3, np.linalg.det(A), rtol=1e-10, atol=1e-10)


def _random_pq(n=2000, seed=4):
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((n, 3, 3)) * rng.uniform(0.01, 1.5, size=(n, 1, 1))
    M = 0.5 * (M + np.swapaxes(M, 1, 2))
    M = M - np.trace(M, axis1=1, axis2=2)[:, None, None] * np.eye(3) / 3
    d = rng.uniform(-0.99, 4.0, size=n)
    T2 = np.einsum("nij,nji->n", M, M)
    T3 = np.einsum("nij,njk,nki->n", M, M, M)
    p, q = op.cubic_coefficients(T2, T3, d)
    return M, d, p, q


def test_root_is_largest_real_root_of_numpy_roots():
    _, _, p, q = _random_pq()
    s = op.largest_real_root(p, q)
    disc = q * q / 4 + p ** 3 / 27
    assert (disc < 0).sum() > 100 and (disc >= 0).sum() > 100  # both branches exercised
    for pi, qi, si in zip(p, q, s):
        r = np.roots([1.0, 0.0, pi, qi])
        real = r[np.abs(r.imag) <= 1e-7 * max(1.0, np.abs(r).max())].real
        assert abs(si - real.max()) <= 1e-9 * max(1.0, abs(si))
    scale = np.maximum(1.0, np.abs(q))
    assert np.max(np.abs(s ** 3 + p * s + q) / scale) < 1e-12


def test_root_reproduces_determinant_equation():
    # The physical root makes det(I s/3 + Mbar) = 1 + delta (Sec. II, Eqs. 2, 5, 8) with
    # I s/3 + Mbar positive definite (no shell crossing); np.linalg.det is independent.
    M, d, p, q = _random_pq(seed=5)
    s = op.largest_real_root(p, q)
    A = M + (s / 3.0)[:, None, None] * np.eye(3)
    np.testing.assert_allclose(np.linalg.det(A), 1.0 + d, rtol=1e-10, atol=1e-10)
    assert np.linalg.eigvalsh(A).min() > 0.0


def test_other_roots_are_not_positive_definite():
    M, d, p, q = _random_pq(seed=6)
    s = op.largest_real_root(p, q)
    for Mi, pi, qi, si in zip(M[:300], p[:300], q[:300], s[:300]):
        r = np.roots([1.0, 0.0, pi, qi])
        for ri in r:
            if abs(ri.imag) < 1e-9 and abs(ri.real - si) > 1e-6:
                assert np.linalg.eigvalsh(Mi + ri.real / 3 * np.eye(3)).min() <= 1e-9


def test_root_homogeneous_case():
    # delta = 0, theta = 0: p = 0, q = -27 and the Laplacian must vanish (s = 3; Sec. II).
    assert op.largest_real_root(0.0, -27.0) == pytest.approx(3.0, abs=1e-15)


def test_root_continuous_across_zero_discriminant():
    # Delta = 0 with q < 0: p = -3 a^2, q = -2 a^3 has roots 2a (simple) and -a (double).
    a = 1.7
    p0, q0 = -3 * a * a, -2 * a ** 3
    for eps in (1e-6, 1e-9, 0.0, -1e-9, -1e-6):
        s = op.largest_real_root(p0, q0 + eps)
        assert abs(s - 2 * a) < 1e-4


def test_source_at_theta_zero_closed_form():
    d = np.random.default_rng(7).uniform(-0.9, 3.0, size=(6, 6, 6))
    sig = op.source(np.zeros_like(d), d, 1.0)
    np.testing.assert_allclose(sig, 3.0 * (np.cbrt(1.0 + d) - 1.0), rtol=1e-13, atol=1e-14)


def test_laplacian_and_hessian_trace_agree_and_scale_with_h():
    th = _rand_theta(seed=8)
    H = op.hessian(th, 2.0)
    np.testing.assert_allclose(np.trace(H, axis1=-2, axis2=-1), op.laplacian(th, 2.0), atol=1e-13)
    np.testing.assert_allclose(op.laplacian(th, 2.0) * 4.0, op.laplacian(th, 1.0), atol=1e-13)


def test_quadratic_potential_has_exact_hessian():
    # theta = (a x^2 + b y^2 + c z^2)/2 + e x y restricted to a non-wrapping interior.
    n = 12
    x, y, z = np.indices((n, n, n)).astype(float)
    a, b, c, e = 0.3, -0.2, 0.1, 0.05
    th = 0.5 * (a * x * x + b * y * y + c * z * z) + e * x * y
    H = op.hessian(th, 1.0)[2:-2, 2:-2, 2:-2]
    np.testing.assert_allclose(H[..., 0, 0], a, atol=1e-12)
    np.testing.assert_allclose(H[..., 1, 1], b, atol=1e-12)
    np.testing.assert_allclose(H[..., 2, 2], c, atol=1e-12)
    np.testing.assert_allclose(H[..., 0, 1], e, atol=1e-12)
    np.testing.assert_allclose(H[..., 0, 2], 0.0, atol=1e-12)
