"""Pins for the oracle-dual experiment (Sec. 5.1, Fig. 3): the screening loop
informed with a known dual optimum theta* in place of the dual update.

With theta = theta* the dual objective is the optimal value, so the gap of
every pass must equal the primal suboptimality P(x) - P* of the current
iterate (strong duality, eq. Dual_Gap at theta*), a closed form that the
planted instances make exact; the usual dual update can only give a larger
gap.  Screening with theta* stays safe, and screens at least as early."""
import numpy as np
import pytest

from oracle import boxls as ob
from synth import workloads as W


def _planted_bvls(seed, m, n, nf, scale):
    rng = W.rng_for(61, seed, m, n)
    A = W.unit_columns(rng.standard_normal((m, n)))
    l, u = -rng.random(n), rng.random(n)
    y, x_star, theta, F = W.planted_bvls(A, l, u, nf, scale, rng)
    return A, y, l, u, x_star, theta


def _planted_nnls(seed, m, n, nf, scale):
    """NNLS instance with a known optimum (eqs. optimality1-2): nf free
    columns, theta* = -(I - P_F) 1 scaled to norm `scale` (orthogonal to the
    free columns, negative sum), every other column a non-negative unit
    column drawn until a_j^T theta* < 0, so it sits at 0 with a margin."""
    rng = W.rng_for(62, seed, m, n)
    AF = W.unit_columns(np.abs(rng.standard_normal((m, nf))))
    Q, _ = np.linalg.qr(AF)
    th = -(np.ones(m) - Q @ (Q.T @ np.ones(m)))
    th *= scale / np.linalg.norm(th)
    cols = []
    while len(cols) < n - nf:
        a = W.unit_columns(np.abs(rng.standard_normal((m, 1))))[:, 0]
        if a @ th < -1e-3 * scale:
            cols.append(a)
    A = np.concatenate([AF, np.stack(cols, axis=1)], axis=1)
    perm = rng.permutation(n)
    A = np.asfortranarray(A[:, perm])
    x = np.concatenate([np.abs(rng.standard_normal(nf)) + 0.1, np.zeros(n - nf)])[perm]
    y = A @ x + th
    return A, y, np.zeros(n), np.full(n, np.inf), x, th


@pytest.mark.parametrize("kind", ["bvls", "nnls"])
def test_gap_with_theta_star_is_the_primal_suboptimality(kind):
    gen = _planted_bvls if kind == "bvls" else _planted_nnls
    A, y, l, u, x_star, theta = gen(0, 40, 120, 12, 0.3)
    p_star = ob.primal(A, y, x_star)
    res = ob.solve(A, y, l, u, K=5, eps_gap=1e-12, max_iter=3000, theta_star=theta, keep_theta=True)
    assert res.passes > 3
    for h in res.history:
        sub = ob.primal(A, y, h["x"]) - p_star
        assert h["gap"] == pytest.approx(sub, rel=1e-7, abs=1e-12 * (1 + p_star))


def test_usual_dual_update_gap_is_larger():
    # the residual point is not the optimum before convergence: its gap
    # exceeds P(x) - P* (a solve that ignored theta_star fails the pin above)
    A, y, l, u, x_star, theta = _planted_bvls(1, 40, 120, 12, 0.3)
    p_star = ob.primal(A, y, x_star)
    res = ob.solve(A, y, l, u, K=5, eps_gap=1e-12, max_iter=200, keep_theta=True)
    excess = [h["gap"] - (ob.primal(A, y, h["x"]) - p_star) for h in res.history]
    assert min(excess) > 0 and max(excess) > 1e-6


@pytest.mark.parametrize("kind", ["bvls", "nnls"])
def test_theta_star_screening_is_safe_and_no_later(kind):
    gen = _planted_bvls if kind == "bvls" else _planted_nnls
    for seed in range(3):
        A, y, l, u, x_star, theta = gen(seed, 50, 160, 15, 0.3)
        step = 1.0 / (1.05 * ob.lipschitz(A))
        kw = dict(K=5, eps_gap=1e-10 if kind == "bvls" else 1e-7, max_iter=100000, step=step)
        ora = ob.solve(A, y, l, u, theta_star=theta, **kw)
        usual = ob.solve(A, y, l, u, **kw)
        assert ora.status == "ok" and usual.status == "ok"
        lo, hi = ora.sat == -1, ora.sat == 1
        assert np.all(x_star[lo] == l[lo]) and np.all(x_star[hi] == u[hi])
        # by the last pass the informed rule has screened at least as much
        assert np.count_nonzero(ora.sat) >= np.count_nonzero(usual.sat)
        assert np.max(np.abs(ora.x - x_star)) <= (1e-4 if kind == "bvls" else 1e-2)


def test_oracle_dual_point_translates_only_when_needed():
    A, y, l, u, x_star, theta = _planted_nnls(3, 30, 80, 10, 0.3)
    th, eps, ok = ob.oracle_dual_point(A, u, theta, -np.ones(30))
    assert ok and eps <= 1e-12 and np.max(np.abs(th - theta)) <= 1e-12
    # a point with some positive correlation is moved onto the feasible set
    z = theta + 0.1 * A[:, 0]
    th, eps, ok = ob.oracle_dual_point(A, u, z, -np.ones(30))
    assert ok and eps > 0 and np.max(A.T @ th) <= 1e-12
