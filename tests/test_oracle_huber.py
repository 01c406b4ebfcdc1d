"""Pins for the oracle's Huber fidelity (Sec. 3.3: eq. GAP_Safe_sph for a
fidelity whose gradient is 1-Lipschitz, alpha = 1; eq. Dual_obj with its
conjugate; Sec. 4.1's dual update -grad F).

The checks tie the oracle to facts outside it: the function's definition at
hand-computed points, its conjugate by brute-force maximisation, weak duality
and the per-coordinate gap identity on random pairs, and the optimum of an
independent bounded quasi-Newton solver (SciPy's L-BFGS-B) on small problems
whose optimum has residuals on both sides of delta and coordinates on both
bounds.
"""
import math

import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import boxls as ob
from synth import workloads as W


def test_huber_values_and_derivative():
    # h_1 at hand-computed points: s^2/2 inside, |s| - 1/2 outside
    s = np.array([-3.0, -1.0, 0.0, 0.5, 2.0])
    np.testing.assert_array_equal(ob.huber(s, 1.0), [2.5, 0.5, 0.0, 0.125, 1.5])
    np.testing.assert_array_equal(ob.huber_grad(s, 1.0), [-1.0, -1.0, 0.0, 0.5, 1.0])
    # psi = h' by central differences (h is C^1)
    rng = np.random.default_rng(1)
    z = 4.0 * rng.standard_normal(200)
    hstep = 1e-6
    fd = (ob.huber(z + hstep, 1.3) - ob.huber(z - hstep, 1.3)) / (2 * hstep)
    np.testing.assert_allclose(ob.huber_grad(z, 1.3), fd, rtol=0, atol=1e-6)
    # delta = +inf is the LS half-square
    np.testing.assert_array_equal(ob.huber(z), 0.5 * z * z)


def test_huber_conjugate_by_brute_force():
    # h*(v) = sup_z v z - h(z): v^2/2 for |v| <= delta, unbounded beyond
    delta = 0.8
    grid = np.linspace(-60.0, 60.0, 1_200_001)
    hg = ob.huber(grid, delta)
    for v in (-0.8, -0.3, 0.0, 0.55, 0.8):
        sup = float(np.max(v * grid - hg))
        assert sup == pytest.approx(float(ob.huber_conj(v, delta)), abs=1e-8)
    for v in (-0.9, 1.5):
        small = float(np.max(v * grid[np.abs(grid) <= 30.0] - hg[np.abs(grid) <= 30.0]))
        large = float(np.max(v * grid - hg))
        assert large > small + 1.0 and math.isinf(float(ob.huber_conj(v, delta)))
    # Fenchel-Young equality at theta = psi(rho)
    rng = np.random.default_rng(2)
    rho = 3.0 * rng.standard_normal(500)
    th = ob.huber_grad(rho, delta)
    np.testing.assert_allclose(ob.huber(rho, delta) + ob.huber_conj(th, delta), rho * th, rtol=0, atol=1e-12)


def _instance(seed, m=40, n=12, outliers=6, delta=0.5):
    rng = np.random.default_rng(seed)
    A = W.unit_columns(rng.standard_normal((m, n)))
    x0 = rng.uniform(-1.5, 1.5, n)
    y = A @ x0 + 0.05 * rng.standard_normal(m)
    y[rng.choice(m, outliers, replace=False)] += rng.choice([-1.0, 1.0], outliers) * rng.uniform(3.0, 6.0, outliers)
    l, u = -np.ones(n), np.ones(n)
    return A, y, l, u, delta


def test_weak_duality_and_per_coordinate_gap():
    # P(x) - D(theta) equals the per-coordinate form and is >= 0 for every
    # x in the box and |theta_i| <= delta (eq. Dual_obj with f* of the
    # Huber fidelity); theta outside that box has D = -inf
    A, y, l, u, delta = _instance(3)
    rng = np.random.default_rng(4)
    for _ in range(50):
        x = l + (u - l) * rng.random(l.size)
        th = rng.uniform(-delta, delta, y.size)
        pd = ob.duality_gap(A, y, l, u, x, th, delta)
        pc = ob.gap_per_coordinate(A, y, l, u, x, th, delta)
        assert pd >= -1e-12
        assert pc == pytest.approx(pd, rel=1e-10, abs=1e-12)
    th = np.full(y.size, 1.01 * delta)
    assert ob.dual(A, y, l, u, th, delta) == -math.inf
    assert ob.gap_per_coordinate(A, y, l, u, x, th, delta) == math.inf


def _lbfgsb(A, y, l, u, delta):
    def fg(x):
        r = y - A @ x
        return float(np.sum(ob.huber(r, delta))), -(A.T @ ob.huber_grad(r, delta))
    res = minimize(fg, np.zeros(A.shape[1]), jac=True, method="L-BFGS-B", bounds=list(zip(l, u)),
                   options={"maxiter": 100000, "ftol": 1e-16, "gtol": 1e-13, "maxcor": 50})
    return res.x


def _check_against_lbfgsb(seed, solver="pg"):
    A, y, l, u, delta = _instance(seed)
    xs = _lbfgsb(A, y, l, u, delta)
    rs = y - A @ xs
    # the optimum exercises both regimes and both bounds
    assert np.any(np.abs(rs) > 1.5 * delta) and np.any(np.abs(rs) < 0.5 * delta)
    assert np.any(xs <= l + 1e-9) and np.any(xs >= u - 1e-9)
    res = ob.solve(A, y, l, u, solver=solver, K=10, eps_gap=1e-12, max_iter=400000, huber_delta=delta)
    assert res.status == "ok"
    ps, po = ob.primal(A, y, xs, delta), ob.primal(A, y, res.x, delta)
    # the certified gap bounds the oracle's suboptimality; both solvers agree
    assert po - ps <= res.gap + 1e-12
    assert abs(po - ps) <= 1e-9
    np.testing.assert_allclose(res.x, xs, rtol=0, atol=1e-5)
    # screened coordinates sit at their bound in the independent optimum
    lo, hi = res.sat == -1, res.sat == 1
    assert np.count_nonzero(lo) + np.count_nonzero(hi) > 0
    np.testing.assert_allclose(xs[lo], l[lo], atol=1e-8)
    np.testing.assert_allclose(xs[hi], u[hi], atol=1e-8)
    # and the oracle's point satisfies the Huber optimality conditions, not the LS ones
    assert ob.kkt_violation(A, y, l, u, res.x, delta) < 1e-5
    assert ob.kkt_violation(A, y, l, u, res.x) > 1e-2


@pytest.mark.parametrize("seed", [5, 6, 7])
def test_huber_solve_matches_lbfgsb(seed):
    _check_against_lbfgsb(seed)


@pytest.mark.parametrize("seed", [5, 6])
def test_huber_chambolle_pock_matches_lbfgsb(seed):
    # the primal-dual solver with the clipped dual prox reaches the same optimum
    _check_against_lbfgsb(seed, solver="cp")


def test_planted_mistake_unclipped_dual_prox_is_caught(monkeypatch):
    """The Chambolle-Pock dual step without the clip to [-delta, delta] (the
    LS prox): the iterates solve the LS problem instead."""
    real = ob.cp_step
    monkeypatch.setattr(ob, "cp_step", lambda A, y, l, u, x, v, tau, sigma, delta=math.inf:
                        real(A, y, l, u, x, v, tau, sigma))
    with pytest.raises(AssertionError):
        _check_against_lbfgsb(5, solver="cp")


def test_planted_mistake_ls_gradient_is_caught(monkeypatch):
    """The Huber gradient replaced by the LS residual (psi not applied): the
    iterates go to the LS optimum, which the independent solver does not
    share."""
    real = ob.huber_grad
    monkeypatch.setattr(ob, "pg_step", lambda A, y, l, u, x, eta, delta=math.inf:
                        ob.project(x + eta * (np.asarray(A).T @ (y - np.asarray(A) @ x)), l, u))
    with pytest.raises(AssertionError):
        _check_against_lbfgsb(5)
    assert ob.huber_grad is real


def test_huber_with_huge_delta_is_ls():
    # no residual reaches delta: the Huber solve takes the LS iterates
    A, y, l, u, _ = _instance(8)
    a = ob.solve(A, y, l, u, solver="pg", K=10, eps_gap=1e-9, max_iter=20000)
    b = ob.solve(A, y, l, u, solver="pg", K=10, eps_gap=1e-9, max_iter=20000, huber_delta=1e300)
    np.testing.assert_array_equal(a.x, b.x)
    assert a.iters == b.iters and np.array_equal(a.sat, b.sat)
    assert b.gap == pytest.approx(a.gap, rel=1e-9, abs=1e-15)


def test_huber_with_unbounded_coordinates_uses_theta_zero():
    # a u_j = +inf column: no translation for the Huber fidelity, theta = 0,
    # so the gap is P(x) and nothing is screened (Sec. 4.2's fallback)
    A, y, l, u, delta = _instance(9)
    u = u.copy()
    u[0] = math.inf
    th, eps, ok = ob.dual_point(A, y, u, np.zeros(A.shape[1]), -np.ones(A.shape[0]), delta)
    assert not ok and eps == 0.0 and not np.any(th)
    res = ob.solve(A, y, l, u, solver="pg", K=10, eps_gap=1e-12, max_iter=200, huber_delta=delta)
    assert not np.any(res.sat) and res.gap == pytest.approx(res.primal, rel=1e-12)


def test_huber_rejects_coordinate_descent():
    # the exact coordinate step has no closed form for this fidelity
    A, y, l, u, delta = _instance(10)
    with pytest.raises(ValueError):
        ob.solve(A, y, l, u, solver="cd", huber_delta=delta)
