"""FP64 CPU oracle for Gap-safe screening of box-constrained least squares.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call, link
or execute anything in this package: only the test suite, the smoke check and
the CPU-baseline leg of the benchmark use it.  It shares no code with the GPU
library (no kernels, headers, helpers or constants) and imports nothing from it.

Reference: C. F. Dantas, E. Soubies, C. Fevotte, "Accelerating Non-Negative and
Bounded-Variable Linear Regression Algorithms with Safe Screening",
arXiv:2202.07258.  Every function cites the section / equation / algorithm it
restates.  Arithmetic is IEEE FP64 throughout, with NumPy matrix products as
the only library primitive besides least-squares solves used for exact optima.

Modules
  boxls    primal/dual objectives, dual points, gap, safe sphere and rule,
           projected gradient, coordinate descent, the screening loop
           (Alg. 1 / Alg. 2), polishing and optimality checks
  brute    exhaustive enumeration of saturation patterns (tiny n)
  adjoint  implicit-differentiation gradient of the NNLS/BVLS solution map

Parity pins that hold for every function are in tests/test_oracle_*.py.  The
paper prints no worked numerical example, so no function is pinned against
printed values; each is pinned against definitions, closed forms, invariants
or brute force instead.
"""
from . import boxls, brute, adjoint  # noqa: F401
