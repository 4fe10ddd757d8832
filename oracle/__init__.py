"""CPU FP64 oracle for multipatch IgA Poisson and exact-local IETI-DP.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The GPU solver never
calls it, links it or reads anything it writes.

What it computes (Hofer, Langer, Takacs, "Inexact dual-primal isogeometric
tearing and interconnecting methods"):

* B-spline bases by the Cox-de Boor recursion (Sec. 2) -- ``bspline``;
* Galerkin stiffness, mass and load of one patch with pull-back basis
  functions (Sec. 1 eq. (1), Sec. 2) -- ``assembly``;
* the global conforming system and its sparse direct solution, the exact
  discrete solution every IETI-DP variant reproduces -- ``conforming``;
* IETI-DP with exact local solves, energy-minimising primal basis from the
  saddle-point systems (eq. (6)), local Neumann problems (eq. (7)), the dual
  problem F lambda = d (eq. (4)) and CG with the scaled Dirichlet
  preconditioner -- ``ietidp``.

Every function is pinned by tests that do not use the oracle itself as the
reference: closed-form B-spline values, partition of unity, Gauss exactness,
closed-form 1D stencils, the polynomial patch test, load-vector integrals,
convergence rates, FETI-DP spectral bounds and brute-force operators.
"""
from . import assembly, bspline, conforming, ietidp  # noqa: F401
