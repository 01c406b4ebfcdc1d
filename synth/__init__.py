"""Seeded synthetic inputs for box-constrained least squares.

This package draws random problem instances (A, y, l, u) shaped like the
paper's synthetic workloads (Sec. 5.1, Tables 1-2) and the five benchmark
configurations of this project.  It holds none of the solver's arithmetic: no
gradient step, dual point, duality gap or screening test lives here.  Both the
FP64 CPU oracle tests and the GPU path consume exactly the arrays produced here.
"""
from .workloads import *  # noqa: F401,F403
