"""Plain, slow FP64 CPU oracle for the reconstruction solve (TEST INFRASTRUCTURE ONLY).

This package is the independent reference the HIP library is checked against. Only the
test-suite, the smoke entry point and the benchmark's CPU-baseline leg may import it; the
library and its Python binding never do, and it shares no code, tables or constants with
the HIP sources.

Every function follows the paper (Shi, Cautun & Li, "New method for initial density
reconstruction") and cites the section / equation it implements:

  * ``operator``   -- discrete derivatives, the traceless invariants, the cubic for the
                      Laplacian and its physical root, the operator L^h and its residual;
  * ``multigrid``  -- restriction, prolongation, red-black Newton-Gauss-Seidel relaxation,
                      the FAS V-cycle and the solve loop;
  * ``deposit``    -- cloud-in-cell density assignment;
  * ``linearized`` -- the Jacobian of the (mean-projected) operator, its transpose and the
                      adjoint gradient dL/d(delta);
  * ``newton``     -- brute-force bordered Newton on tiny grids (dense linear algebra).

Readings taken where the paper is silent or garbled are stated in the docstrings.
"""
from . import operator, multigrid, deposit, linearized, newton  # noqa: F401
