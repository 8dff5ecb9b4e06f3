"""End-to-end pin of the oracle chain against an independent truth.

Particles are a lattice q displaced by a Zel'dovich (potential, curl-free) displacement
psi_true; the chain deposits them (CIC), smooths, solves the reconstruction equation and maps
the particles back: the reconstructed displacement x - q = -grad theta (Sec. III) must
reproduce psi_true. Without shell crossing the exact map is the gradient of a potential, so the
only differences are the smoothing and the discretisation. A flipped sign anywhere in the chain
(the mapping, the source, the root branch) turns the correlation negative or destroys it.
"""
import numpy as np

import inputs
from oracle import deposit as dep
from oracle import lagrangian as olag
from oracle import multigrid as mg


def test_reconstruction_recovers_the_zeldovich_displacement():
    n = 32
    pos = inputs.zeldovich_particles(n, 4.0, 1001, rms_disp=1.0)
    q = np.indices((n, n, n)).reshape(3, -1).T.astype(float)
    psi_true = (pos - q + n / 2) % n - n / 2
    rho = dep.deposit(pos, n, 1.0, "cic")
    delta = inputs.normalise_density(inputs.gaussian_smooth(rho / rho.mean(), 1.0))
    theta, info = mg.solve(delta, tol=1e-8)
    assert info["converged"]
    disp, _ = olag.lagrangian_map(theta, pos)
    psi_rec = -disp
    for a in range(3):
        assert np.corrcoef(psi_rec[:, a], psi_true[:, a])[0, 1] > 0.995
    err = np.sqrt(((psi_rec - psi_true) ** 2).sum(1).mean() / (psi_true ** 2).sum(1).mean())
    assert err < 0.12, err
