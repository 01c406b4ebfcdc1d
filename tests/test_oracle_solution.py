"""Pins for the oracle's solutions: exhaustive enumeration pinned to closed
forms, then the iterative solvers (PG, CD; screened and unscreened) pinned to
the exhaustive optimum, SciPy's independent NNLS / BVLS routines, and planted
optima."""
import numpy as np
import pytest
from scipy.optimize import lsq_linear, nnls

from oracle import boxls as ob
from oracle.brute import solve_exhaustive
from synth import workloads as W


# --- exhaustive search pinned to closed forms ------------------------------
def test_exhaustive_matches_orthonormal_closed_form():
    # A^T A = I  =>  P(x) = 1/2||x - A^T y||^2 + const, so x* = Pi_[l,u](A^T y)
    for s in range(6):
        P = W.orthonormal_bvls(s, 9, 7)
        xs, pat = solve_exhaustive(P.A, P.y, P.l, P.u)
        np.testing.assert_allclose(xs, np.clip(P.A.T @ P.y, P.l, P.u), atol=1e-10)


def test_exhaustive_matches_diagonal_closed_form():
    rng = np.random.default_rng(5)
    d = 0.5 + rng.random(8)
    A = np.diag(d)
    y = 2 * rng.standard_normal(8)
    l, u = -rng.random(8), rng.random(8)
    xs, _ = solve_exhaustive(A, y, l, u)
    np.testing.assert_allclose(xs, np.clip(y / d, l, u), atol=1e-12)


@pytest.mark.parametrize("seed", range(6))
def test_exhaustive_matches_scipy_bvls(seed):
    P = W.tiny_bvls(seed, 12, 8)
    xs, _ = solve_exhaustive(P.A, P.y, P.l, P.u)
    ref = lsq_linear(P.A, P.y, bounds=(P.l, P.u), method="bvls", tol=1e-14)
    np.testing.assert_allclose(xs, ref.x, atol=1e-8)


@pytest.mark.parametrize("seed", range(6))
def test_exhaustive_matches_scipy_nnls(seed):
    P = W.tiny_nnls(seed, 12, 9)
    xs, _ = solve_exhaustive(P.A, P.y, P.l, P.u)
    ref, _ = nnls(P.A, P.y)
    np.testing.assert_allclose(xs, ref, atol=1e-9)


# --- iterative solvers pinned to the exhaustive optimum --------------------
@pytest.mark.parametrize("solver", ["pg", "cd"])
@pytest.mark.parametrize("screening", [True, False])
@pytest.mark.parametrize("kind", ["bvls", "nnls"])
def test_solver_reaches_exhaustive_optimum(solver, screening, kind):
    for seed in range(4):
        P = W.tiny_bvls(seed, 14, 9) if kind == "bvls" else W.tiny_nnls(seed, 14, 9)
        xs, pat = solve_exhaustive(P.A, P.y, P.l, P.u)
        res = ob.solve(P.A, P.y, P.l, P.u, solver=solver, K=5 if solver == "pg" else 1,
                       eps_gap=1e-14, max_iter=400000, screening=screening)
        assert res.status == "ok", (res.gap, res.iters)
        # Gap certificate: P(x) - P* <= Gap (weak duality)
        assert ob.primal(P.A, P.y, res.x) - ob.primal(P.A, P.y, xs) <= res.gap + 1e-13
        xp, ok = ob.polish(P.A, P.y, P.l, P.u, res.x)
        assert ok
        np.testing.assert_allclose(xp, xs, atol=1e-8)
        assert np.all((res.sat == 0) | (res.sat == pat))   # screened => saturated as brute force says


def test_exhaustive_n12_matches_pg():
    P = W.tiny_bvls(42, 16, 12)
    xs, pat = solve_exhaustive(P.A, P.y, P.l, P.u)
    res = ob.solve(P.A, P.y, P.l, P.u, eps_gap=1e-14, max_iter=10 ** 6)
    xp, ok = ob.polish(P.A, P.y, P.l, P.u, res.x)
    assert ok
    np.testing.assert_allclose(xp, xs, atol=1e-8)


def test_planted_bvls_recovered():
    rng = W.rng_for(97, 0)
    A = W.unit_columns(rng.standard_normal((60, 150)))
    l, u = -rng.random(150), rng.random(150)
    y, x_star, th, F = W.planted_bvls(A, l, u, 24, 0.05, rng)
    res = ob.solve(A, y, l, u, eps_gap=1e-13, max_iter=10 ** 6)
    assert res.status == "ok"
    xp, ok = ob.polish(A, y, l, u, res.x)
    assert ok
    np.testing.assert_allclose(xp, x_star, atol=1e-8)
    assert ob.kkt_violation(A, y, l, u, xp) < 1e-10


def test_kkt_small_at_termination():
    P = W.c1_companion(0, 40, 100)
    res = ob.solve(P.A, P.y, P.l, P.u, eps_gap=1e-10, max_iter=10 ** 6)
    assert res.status == "ok"
    # |a_j^T theta| = O(sqrt(gap)) on free coordinates
    assert ob.kkt_violation(P.A, P.y, P.l, P.u, res.x) < 1e-3


def test_step_default_is_inverse_lipschitz():
    P = W.tiny_bvls(1, 10, 20)
    L = ob.lipschitz(P.A)
    s = np.linalg.svd(P.A, compute_uv=False)
    assert L == pytest.approx(s[0] ** 2, rel=1e-12)
    assert ob.lipschitz_power(P.A, 500) == pytest.approx(L, rel=1e-6)


def test_maxiter_status():
    P = W.tiny_bvls(2, 10, 20)
    res = ob.solve(P.A, P.y, P.l, P.u, eps_gap=0.0, max_iter=23, K=10)
    assert res.status == "maxiter" and res.iters == 23 and res.passes == 3


def _hash_start(m):
    """The start vector of the library's Lanczos estimate: 1 +- 1/4 by the top
    bit of Knuth's multiplicative hash of the row index, i * 2654435761 mod
    2^32 (TAOCP Vol. 3, Sec. 6.4)."""
    h = (np.arange(m, dtype=np.uint64) * np.uint64(2654435761)) & np.uint64(0xFFFFFFFF)
    return np.where((h >> np.uint64(31)) != 0, 1.25, 0.75)


def test_lanczos_estimate_pins():
    rng = np.random.default_rng(7)
    # one step is the Rayleigh quotient u^T A A^T u of the unit start vector
    A = rng.standard_normal((9, 14))
    u = _hash_start(9)
    uu = u / np.linalg.norm(u)
    assert ob.lipschitz_lanczos(A, 1, u) == pytest.approx(float(np.sum((A.T @ uu) ** 2)), rel=1e-13)
    # a Krylov space that is invariant after two steps: exact largest eigenvalue
    # of the two coordinates the start vector touches
    s = np.array([3.0, 0.5, 7.0, 1.0])
    D = np.diag(s)
    assert ob.lipschitz_lanczos(D, 2, np.array([1.0, 1.0, 0.0, 0.0])) == pytest.approx(9.0, rel=1e-13)
    assert ob.lipschitz_lanczos(D, 3, np.array([1.0, 1.0, 1.0, 0.0])) == pytest.approx(49.0, rel=1e-13)
    # m steps span R^m: the exact ||A||_2^2
    L = ob.lipschitz(A)
    assert ob.lipschitz_lanczos(A, 9, u) == pytest.approx(L, rel=1e-10)
    # a Rayleigh-Ritz value: below L, nondecreasing in the number of steps,
    # and at least the Rayleigh quotient of the power iterate M^(k-1) u
    B = rng.standard_normal((60, 200))
    LB = ob.lipschitz(B)
    u = _hash_start(60)
    prev = 0.0
    v = u / np.linalg.norm(u)
    for k in range(1, 13):
        est = ob.lipschitz_lanczos(B, k, u)
        rq = float(np.sum((B.T @ v) ** 2))
        assert est <= LB * (1 + 1e-12)
        assert est >= prev * (1 - 1e-12)
        assert est >= rq * (1 - 1e-12)
        prev = est
        w = B @ (B.T @ v)
        v = w / np.linalg.norm(w)
    assert prev > 0.9 * LB
