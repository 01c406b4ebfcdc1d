"""Pins for the implicit-differentiation adjoint: FP64 central finite
differences of the exact solution map, and the one-dimensional closed form."""
import numpy as np
import pytest
from scipy.optimize import nnls

from oracle import adjoint as oa
from oracle import boxls as ob
from synth import workloads as W


def _exact_nnls(A, y, t):
    n = A.shape[1]
    res = ob.solve(A, y, np.zeros(n), np.full(n, np.inf), eps_gap=1e-11, max_iter=200000, K=10, t=t)
    if res.status != "ok":
        return None
    x, ok = ob.polish(A, y, np.zeros(n), np.full(n, np.inf), res.x)
    return x if ok else None


def _subproblem(rep):
    A, Y, T = W.c5_layer(rep)
    return A[:32, :64].copy(), Y[:32, 0].copy(), T[:64, 0].copy()


def _pick_rep():
    # need a non-degenerate, strictly complementary subproblem (|F| < m, full
    # rank) whose matrix admits a translation direction (Remark 4)
    for rep in range(40):
        A, y, tgt = _subproblem(rep)
        t = W.interior_direction(A)
        if t is None:
            continue
        x = _exact_nnls(A, y, t)
        if x is None:
            continue
        F = x > 0
        g = A.T @ (y - A @ x)
        if 0 < F.sum() < 32 and np.linalg.matrix_rank(A[:, F]) == F.sum() \
                and np.min(x[F]) > 1e-4 and np.max(g[~F]) < -1e-4:
            return A, y, tgt, x, t
    pytest.skip("no strictly complementary subproblem found")


def _nnls_exact(A, y):
    # SciPy's active-set NNLS (exact up to rounding): an independent solver
    return nnls(A, y, maxiter=10000)[0]


def test_adjoint_matches_finite_differences():
    A, y, tgt, x, t = _pick_rep()
    np.testing.assert_allclose(_nnls_exact(A, y), x, atol=1e-10)
    L = lambda xx: float(np.sum((xx - tgt) ** 2))
    dLdx = 2 * (x - tgt)
    dy, dA, dl, du = oa.solution_grad(A, y, np.zeros(64), np.full(64, np.inf), x, dLdx)
    h = 1e-6
    for i in range(32):
        e = np.zeros(32); e[i] = h
        fd = (L(_nnls_exact(A, y + e)) - L(_nnls_exact(A, y - e))) / (2 * h)
        assert fd == pytest.approx(dy[i], rel=1e-5, abs=1e-7)
    rng = np.random.default_rng(0)
    for _ in range(40):
        i, j = rng.integers(32), rng.integers(64)
        E = np.zeros_like(A); E[i, j] = h
        fd = (L(_nnls_exact(A + E, y)) - L(_nnls_exact(A - E, y))) / (2 * h)
        assert fd == pytest.approx(dA[i, j], rel=1e-5, abs=1e-7)


def test_adjoint_one_dimensional_closed_form():
    a, y, tt = 1.7, 2.3, 0.4
    x = np.array([y / a])
    dLdx = 2 * (x - tt)
    dy, dA, _, _ = oa.solution_grad(np.array([[a]]), np.array([y]), np.zeros(1), np.full(1, np.inf), x, dLdx)
    assert dy[0] == pytest.approx(dLdx[0] / a, rel=1e-14)
    assert dA[0, 0] == pytest.approx(-dLdx[0] * y / a ** 2, rel=1e-14)


def test_adjoint_bvls_bound_gradient():
    # dL/du for a coordinate at its upper bound: raising u_j moves x_j one-for-one
    rng = np.random.default_rng(4)
    A = rng.standard_normal((10, 4))
    l, u = -np.ones(4), 0.2 * np.ones(4)
    y = A @ np.array([0.5, 0.1, -0.3, 0.0]) + 0.01 * rng.standard_normal(10)
    res = ob.solve(A, y, l, u, eps_gap=1e-15, max_iter=10 ** 6)
    x, ok = ob.polish(A, y, l, u, res.x)
    assert ok and x[0] == u[0]
    tgt = rng.standard_normal(4)
    L = lambda xx: float(np.sum((xx - tgt) ** 2))
    _, _, dl, du = oa.solution_grad(A, y, l, u, x, 2 * (x - tgt))
    h = 1e-6
    def solve_u(uu):
        r = ob.solve(A, y, l, uu, eps_gap=1e-15, max_iter=10 ** 6)
        return ob.polish(A, y, l, uu, r.x)[0]
    e = np.zeros(4); e[0] = h
    fd = (L(solve_u(u + e)) - L(solve_u(u - e))) / (2 * h)
    assert fd == pytest.approx(du[0], rel=1e-5, abs=1e-8)
