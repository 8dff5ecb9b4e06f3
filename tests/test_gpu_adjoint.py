"""Adjoint form: dL/ddelta through the solve, against the oracle's direct adjoint and central
finite differences of the GPU forward solve.

Tolerances: <= 1e-8 relative L2 against the oracle adjoint (both solve the same linear system
to ~1e-12); <= 1e-4 relative per cell against central differences (truncation O(eps^2) plus the
forward solves' residual floor).
"""
import functools

import numpy as np
import pytest
import torch

import inputs
from gpu_util import announce, dev, host, require_gpu
from oracle import linearized as olin
from oracle import multigrid as omg

pytestmark = pytest.mark.gpu

from paper_1709_06350_amd import autograd as mag  # noqa: E402
from paper_1709_06350_amd import mr  # noqa: E402


def spectral_loss_torch(theta, theta_t, cells=4.0):
    n = theta.shape[0]
    k1 = 2.0 * np.pi * torch.fft.fftfreq(n, dtype=torch.float64, device=theta.device)
    k2 = k1[:, None, None] ** 2 + k1[None, :, None] ** 2 + k1[None, None, :] ** 2
    W = torch.exp(-k2 * cells ** 2)
    d = torch.fft.fftn(theta - theta_t)
    return (W * (d.real ** 2 + d.imag ** 2)).sum()


@functools.lru_cache(maxsize=None)
def _oracle_case(n):
    delta = inputs.lognormal(n, 0.7, 2.0, 40 + n)
    theta = omg.solve(delta, tol=1e-14, max_cycles=100)[0]
    g = np.random.default_rng(n).standard_normal(delta.shape)
    ref, _ = olin.adjoint_gradient(theta, delta, g)
    return delta, theta, g, ref


# flags 0: the per-level timed kernel choice; ADJ_TILED: the tiled plane-marching kernel wherever a
# tile fits (both coefficient load schedules, alternating by level); ADJ_ROWS: the row kernel.
# 24^3 has a 4 x 8 tile on its finest level and a row-kernel coarse level (12^3).
@pytest.mark.parametrize("n,flags", [(8, 0), (16, 0), (16, mr.MR_FLAG_ADJ_TILED), (16, mr.MR_FLAG_ADJ_ROWS),
                                     (24, mr.MR_FLAG_ADJ_TILED)])
def test_adjoint_matches_oracle_direct(n, flags):
    require_gpu()
    announce(f"adjoint vs oracle n={n} flags={flags}")
    delta, theta, g, ref = _oracle_case(n)
    with mr.Context(n, tol=1e-13, flags=flags) as c:
        got, info = c.adjoint_solve(dev(delta), dev(theta), dev(g))
    got = host(got)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"adjoint n={n} flags={flags}: cycles={info.cycles} rel L2 err={err:.3e}")
    assert info.status == 0 and err <= 1e-8


@pytest.mark.parametrize("n", [64, 128])
def test_adjoint_tiled_matches_rows(n):
    """The tiled and the row half-sweeps on meshes with several tiles and chunks per level: both
    solve J^T l = g - <g> to 1e-12, so the gradients agree to that level (rounding order differs)."""
    require_gpu()
    announce(f"adjoint tiled vs rows n={n}")
    delta = dev(inputs.lognormal(n, 0.8, 3.0, 70 + n))
    with mr.Context(n, tol=1e-12) as c:
        theta = torch.zeros_like(delta)
        c.solve(delta, theta)
        g = torch.randn(delta.shape, dtype=torch.float64, generator=torch.Generator().manual_seed(n)).to(delta.device)
        out = {}
        for flags in (mr.MR_FLAG_ADJ_ROWS, mr.MR_FLAG_ADJ_TILED, 0):
            c.set_opts(flags=flags)
            got, info = c.adjoint_solve(delta, theta, g)
            assert info.status == 0, flags
            out[flags] = host(got)
    ref = out[mr.MR_FLAG_ADJ_ROWS]
    for flags in (mr.MR_FLAG_ADJ_TILED, 0):
        err = np.linalg.norm(out[flags] - ref) / np.linalg.norm(ref)
        print(f"n={n} flags={flags}: rel L2 vs rows {err:.3e}")
        assert err <= 1e-9, flags


def test_autograd_matches_oracle_gradient():
    require_gpu()
    n = 16
    delta = inputs.lognormal(n, 0.6, 2.0, 51)
    theta_t = 0.5 * omg.solve(inputs.lognormal(n, 0.6, 2.0, 52), tol=1e-13)[0]
    with mr.Context(n, tol=1e-13) as c:
        d = dev(delta).requires_grad_(True)
        th = mag.solve(d, c)
        L = spectral_loss_torch(th, dev(theta_t))
        L.backward()
        got = host(d.grad)
    theta = omg.solve(delta, tol=1e-14, max_cycles=100)[0]
    ref, _ = olin.adjoint_gradient(theta, delta, olin.spectral_loss_grad(theta, theta_t))
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-8
    assert float(L.detach()) == pytest.approx(olin.spectral_loss(theta, theta_t), rel=1e-10)


def _fd_gradient(c, delta, theta_star, theta_t, cells, eps):
    """Central differences of L(solve(delta)) with warm-started solves to the residual floor."""
    n = delta.shape[0]
    k1 = 2.0 * np.pi * torch.fft.fftfreq(n, dtype=torch.float64, device="cuda")
    W = torch.exp(-(k1[:, None, None] ** 2 + k1[None, :, None] ** 2 + k1[None, None, :] ** 2) * 16.0)
    pt = torch.fft.fftn(theta_t)
    out = []
    c.set_opts(warm_start=1, tol=1e-15, max_cycles=60)
    for cell in cells:
        sols = []
        for sgn in (1.0, -1.0):
            d = delta.clone().reshape(-1)
            d[cell] += sgn * eps
            th, _ = c.solve(d.reshape(delta.shape), theta=theta_star.clone(), check=False)
            sols.append(torch.fft.fftn(th))
        a, b = sols
        # |a - pt|^2 - |b - pt|^2 = Re[conj(a - b) (a + b - 2 pt)]
        diff = (W * (torch.conj(a - b) * (a + b - 2.0 * pt)).real).sum()
        out.append(float(diff) / (2.0 * eps))
    c.set_opts(warm_start=0, tol=1e-10, max_cycles=100)
    return np.array(out)


def test_adjoint_matches_finite_differences_32():
    require_gpu()
    n = 32
    delta = dev(inputs.lognormal(n, 0.8, 3.0, 61))
    theta_t = dev(0.5 * inputs.lognormal(n, 0.8, 3.0, 62))
    cells = np.random.default_rng(63).choice(n ** 3, 8, replace=False)
    with mr.Context(n, tol=1e-12) as c:
        d = delta.clone().requires_grad_(True)
        th = mag.solve(d, c)
        spectral_loss_torch(th, theta_t).backward()
        grad = host(d.grad).reshape(-1)[cells]
        fd = _fd_gradient(c, delta, th.detach(), theta_t, cells, 1e-6)
    scale = np.abs(grad).max()
    assert np.max(np.abs(grad - fd)) <= 1e-4 * scale, (grad, fd)


@pytest.mark.timeout(900)
def test_config_adjoint_256_fd_32_cells():
    """Forward FP64 solve on a CIC field (particles -> CIC -> 2-cell smoothing), spectral loss
    against a second seed's solution, gradient vs central differences on 32 random cells.

    Central differences at eps = 1e-6 are limited by the FP64 residual floor of the forward solves
    (theta ~ 1e2 gives an absolute floor of ~1e-10 in the residual, against ~eps * D ~ 1e-6 for the
    perturbation itself), i.e. ~1e-3 relative; they are checked at 2e-2 of the largest gradient.
    The per-cell 1e-4 check uses eps = 1e-4, where truncation (eps^2) and floor (floor / eps)
    errors are both below 1e-5.
    """
    require_gpu()
    n = 256

    def chain(c, seed):
        pos = inputs.zeldovich_particles(n, 2.0, seed, rms_disp=2.0)
        d = host(c.deposit_cic(dev(pos)))
        return dev(inputs.normalise_density(inputs.gaussian_smooth(d + 1.0, 2.0)))

    with mr.Context(n, tol=1e-10) as c:
        announce("adjoint 256^3: inputs")
        delta = chain(c, 1001)
        theta_t, _ = c.solve(chain(c, 1004))
        announce("adjoint 256^3: forward + backward")
        d = delta.clone().requires_grad_(True)
        th = mag.solve(d, c)
        spectral_loss_torch(th, theta_t).backward()
        cells = np.random.default_rng(1005).choice(n ** 3, 32, replace=False)
        grad = host(d.grad).reshape(-1)[cells]
        announce("adjoint 256^3: finite differences")
        fd6 = _fd_gradient(c, delta, th.detach(), theta_t, cells, 1e-6)
        fd4 = _fd_gradient(c, delta, th.detach(), theta_t, cells, 1e-4)
    scale = np.abs(grad).max()
    rel4 = np.abs(grad - fd4) / np.maximum(np.abs(fd4), 1e-3 * scale)
    err6 = np.max(np.abs(grad - fd6)) / scale
    print(f"adjoint 256^3: eps=1e-4 max per-cell rel err {rel4.max():.3e}; eps=1e-6 max err / max|g| {err6:.3e}")
    assert rel4.max() <= 1e-4
    assert err6 <= 2e-2


@pytest.mark.parametrize("n,depth", [(16, 2), (24, 4)])
def test_anderson_adjoint_matches_oracle_direct(n, depth):
    """mr_adjoint_solve_anderson: the same linear system, so the same gradient as the oracle's
    direct adjoint (<= 1e-8 relative L2)."""
    require_gpu()
    announce(f"anderson adjoint vs oracle n={n} depth={depth}")
    delta, theta, g, ref = _oracle_case(n)
    with mr.Context(n, tol=1e-13) as c:
        got, info = c.adjoint_solve(dev(delta), dev(theta), dev(g), anderson_depth=depth)
    err = np.linalg.norm(host(got) - ref) / np.linalg.norm(ref)
    print(f"anderson adjoint n={n}: cycles={info.cycles} rel L2 err={err:.3e}")
    assert info.status == 0 and err <= 1e-8


def test_anderson_adjoint_matches_plain_adjoint_128():
    require_gpu()
    n = 128
    announce("anderson adjoint vs plain n=128")
    delta = inputs.lognormal(n, 1.0, 2.0, 1002)
    with mr.Context(n, tol=1e-10) as c:
        theta, _ = c.solve(dev(delta))
        g = theta - theta.mean()
        c.set_opts(tol=1e-10)
        a, ia = c.adjoint_solve(dev(delta), theta, g)
        b, ib = c.adjoint_solve(dev(delta), theta, g, anderson_depth=2)
    ha, hb = host(a), host(b)
    err = np.linalg.norm(hb - ha) / np.linalg.norm(ha)
    print(f"adjoint 128^3: cycles plain {ia.cycles}, Anderson(2) {ib.cycles}; rel L2 diff {err:.2e}")
    assert ia.status == 0 and ib.status == 0 and err <= 1e-8
