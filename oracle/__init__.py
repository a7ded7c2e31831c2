"""Oracle — TEST INFRASTRUCTURE ONLY.

A plain, slow, FP64 CPU implementation of the direct solve of the
second-order staggered Poisson equation by eigenfunction expansion
(Costa, "A FFT-based finite-difference solver for massively-parallel direct
numerical simulations of turbulent flows", Sec. 2.1, Tables 1 and 2, Sec. 3).

It exists to check the GPU path.  Only the tests, the package's ``smoke()``
entry and the CPU-baseline leg of the benchmark may import it.  The GPU
library never calls it, and the two share no code: the oracle evaluates the
printed transform sums as dense O(n)-per-output products, the GPU path uses
hand-written FFT-based kernels with its own host-built tables.

Modules:
  transforms   Table 2 sums (forward / backward) and Table 1 eigenvalues
  tridiagonal  the 1D operator rows, Gauss elimination, cyclic and pinned solves
  poisson      the seven-point operator (Eq. (poi)) and the three-step solve
  projection   the pressure-correction steps around the solve (Sec. 2):
               divergence, gradient, right-hand side and projection
  navier_stokes  one low-storage RK3 step with a pressure correction per
               substep (Sec. 2, Eq. (up)) on a tri-periodic grid: the
               divergence-form advection-diffusion term and the substeps

Every function is pinned by tests under ``tests/`` against things other than
itself (library transforms, LAPACK's tridiagonal routine, exact rational
elimination, dense solves, closed-form eigenfunctions).  Parity is not
unpinned for any function here.
"""
from . import transforms, tridiagonal, poisson, projection, navier_stokes  # noqa: F401
from .poisson import (solve, solve_corrected, apply_operator, residual, is_singular,  # noqa: F401
                      weighted_mean)
