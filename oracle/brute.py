"""Exhaustive solution of tiny box-constrained least-squares problems.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Every optimum of min 1/2||Ax - y||^2 s.t. l <= x <= u has a saturation pattern
(each coordinate at l_j, at u_j, or free).  Given the pattern, the free part
solves an unconstrained least-squares problem with the saturated part folded
into y, and the pattern is optimal exactly when the free part lies in the box
and the correlations a_j^T (y - Ax) have the signs required by the first-order
conditions eqs. optimality1-2 (Sec. 3.2).  Enumerating all 3^n (BVLS) or 2^n
(NNLS) patterns therefore finds the optimum without any iterative solver.
"""
from __future__ import annotations

import itertools

import numpy as np


def solve_exhaustive(A, y, l, u, tol: float = 1e-9):
    """Return (x*, pattern) with pattern[j] in {-1 (at l), 0 (free), +1 (at u)}.

    Among all patterns whose least-squares completion is feasible (within tol)
    and satisfies the sign conditions (within tol), the one with the smallest
    objective is returned.  Intended for n <= 12."""
    A = np.asarray(A, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    l = np.asarray(l, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    m, n = A.shape
    if n > 14:
        raise ValueError("exhaustive search is for tiny problems only")
    best = None
    best_val = np.inf
    fin_u = np.isfinite(u)
    scale = 1.0 + float(np.max(np.abs(A.T @ y)))
    for free_mask in itertools.product((False, True), repeat=n):
        F = np.array(free_mask, dtype=bool)
        S = np.flatnonzero(~F)
        # saturated coordinates: each at l or (if finite) at u
        choices = [(-1, 1) if fin_u[j] else (-1,) for j in S]
        pinv = np.linalg.pinv(A[:, F]) if np.any(F) else None
        for side in itertools.product(*choices):
            x = np.empty(n)
            side = np.asarray(side, dtype=np.int64)
            if S.size:
                x[S] = np.where(side < 0, l[S], u[S])
            rhs = y - (A[:, S] @ x[S] if S.size else 0.0)
            if pinv is not None:
                x[F] = pinv @ rhs
                if np.any(x[F] < l[F] - tol) or np.any(x[F] > u[F] + tol):
                    continue
            g = A.T @ (y - A @ x)
            if S.size:
                gs = g[S]
                if np.any((side < 0) & (gs > tol * scale)) or np.any((side > 0) & (gs < -tol * scale)):
                    continue
            if np.any(F) and np.any(np.abs(g[F]) > 1e-7 * scale):
                continue
            val = 0.5 * float(np.sum((A @ x - y) ** 2))
            if val < best_val - 1e-14 * max(1.0, abs(val)):
                best_val = val
                pat = np.zeros(n, dtype=np.int8)
                if S.size:
                    pat[S] = np.where(side < 0, -1, 1)
                best = (x.copy(), pat)
    if best is None:
        raise RuntimeError("no optimal pattern found")
    return best
