"""MI355X-native inexact IETI-DP solver for multipatch isogeometric Poisson problems.

The solver lives in the HIP library ``libieti.so`` (C ABI in include/ieti.h);
this package is its thin Python binding.  Importing it loads nothing; the
library is opened on first use and a missing build raises.
"""
from .solver import Plan, Server, Solver, default_options, options_for, quadrature_points  # noqa: F401
