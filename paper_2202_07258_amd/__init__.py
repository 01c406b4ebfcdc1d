"""boxscreen: Gap-safe screening for NNLS / BVLS on MI355X (gfx950).

The solvers live in the HIP shared library ``libboxscreen.so`` (C ABI in
include/boxscreen.h); this package only marshals PyTorch GPU tensors into it.
Importing the package does not load the library; the first solver call does,
and raises if it is missing (there is no CPU fallback).
"""
from .native import (  # noqa: F401
    BoxscreenError, colmajor, load, solve_bvls, solve_bvls_noalloc, solve_bvls_varbatch, solve_nnls,
    solve_nnls_batched_shared,
    nnls_adjoint, bvls_adjoint, version, LIBRARY_PATH, EXPORTED, MAX_ROWS,
)
from .layer import nnls_layer  # noqa: F401
from . import autotune  # noqa: F401
