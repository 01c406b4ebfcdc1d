"""Implicit-differentiation gradient of the box-constrained LS solution map.

TEST INFRASTRUCTURE ONLY (see the package docstring).

At an optimum x* of min 1/2||Ax - y||^2 s.t. l <= x <= u with free set
F = {j : l_j < x*_j < u_j} and saturated set S, the optimality conditions
(Sec. 3.2, eq. optimality2: a_j^T theta* = 0 on F) give
    A_F^T (y - A_F x_F - A_S x_S) = 0,
so x_F = (A_F^T A_F)^{-1} A_F^T (y - A_S x_S) while x_S stays on its bound for
small perturbations when strict complementarity holds (a_j^T theta* != 0 on
S).  Differentiating this identity:

    v      = (A_F^T A_F)^{-1} dL/dx_F
    dL/dy  = A_F v
    dL/dA  = r v_bar^T - (dL/dy) x*^T,   r = y - A x*, v_bar = v on F, 0 on S
    dL/dl_j = dL/dx_j - a_j^T dL/dy  for j at its lower bound (same for u).

The paper does not differentiate the solution map; this is the adjoint used by
the differentiable layer, derived from the cited optimality conditions.
"""
from __future__ import annotations

import numpy as np


def free_set(x, l, u):
    return (x > l) & (x < u)


def solution_grad(A, y, l, u, x, dLdx):
    """Return (dL/dy, dL/dA, dL/dl, dL/du) at the optimum x (FP64)."""
    A = np.asarray(A, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    F = free_set(x, l, u)
    AF = A[:, F]
    M = AF.T @ AF
    v = np.linalg.solve(M, dLdx[F]) if np.any(F) else np.zeros(0)
    dy = AF @ v
    vbar = np.zeros(A.shape[1])
    vbar[F] = v
    r = y - A @ x
    dA = np.outer(r, vbar) - np.outer(dy, x)
    corr = dLdx - A.T @ dy
    dl = np.where(~F & (x <= l), corr, 0.0)
    du = np.where(~F & (x >= u), corr, 0.0)
    return dy, dA, dl, du


def exact_solution(A, y, l, u, x_approx):
    """Exact optimum with the saturation pattern of x_approx (free-set
    least squares, as in boxls.polish)."""
    from .boxls import polish
    return polish(A, y, l, u, x_approx)
