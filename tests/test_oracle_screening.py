"""Pins for the screening loop (Alg. 1 / Alg. 2, eq. safe_rule, eq.
GAP_Safe_sph): safety against exact optima, the safe sphere containing theta*
at every pass, degenerate instances screening nothing, the reduced gap never
exceeding the full gap, and planted mistakes being caught."""
import numpy as np
import pytest

from oracle import boxls as ob
from oracle.brute import solve_exhaustive
from synth import workloads as W


def _planted(seed, m=80, n=240, nf=20, scale=0.05):
    rng = W.rng_for(96, seed)
    A = W.unit_columns(rng.standard_normal((m, n)))
    l, u = -rng.random(n), rng.random(n)
    y, x, th, F = W.planted_bvls(A, l, u, nf, scale, rng)
    return A, y, l, u, x, th


@pytest.mark.parametrize("solver", ["pg", "cd"])
def test_safe_sphere_contains_theta_star_every_pass(solver):
    for seed in range(3):
        A, y, l, u, xs, ths = _planted(seed)
        res = ob.solve(A, y, l, u, solver=solver, K=10 if solver == "pg" else 1,
                       eps_gap=1e-12, max_iter=200000, keep_theta=True)
        assert res.status == "ok"
        for h in res.history:
            assert np.linalg.norm(h["theta"] - ths) <= h["radius"] * (1 + 1e-9) + 1e-12


def test_screened_coordinates_are_saturated_at_optimum():
    for seed in range(3):
        A, y, l, u, xs, ths = _planted(seed)
        res = ob.solve(A, y, l, u, eps_gap=1e-10, max_iter=200000)
        S = res.sat != 0
        assert S.sum() > 0.5 * (A.shape[1] - 20)          # most saturated ones get screened
        assert np.all(xs[res.sat == -1] == l[res.sat == -1])
        assert np.all(xs[res.sat == 1] == u[res.sat == 1])


def test_nnls_screening_safe_vs_exhaustive():
    for seed in range(8):
        P = W.tiny_nnls(seed, 14, 10)
        xs, pat = solve_exhaustive(P.A, P.y, P.l, P.u)
        res = ob.solve(P.A, P.y, P.l, P.u, K=3, eps_gap=1e-12, max_iter=200000)
        assert np.all(pat[res.sat == -1] == -1)
        assert not np.any(res.sat == 1)                    # S_u is empty for NNLS (Alg. 2)


def test_c1_as_specified_screens_nothing():
    P = W.c1_nnls(0)
    res = ob.solve(P.A, P.y, P.l, P.u, K=10, eps_gap=1e-9, max_iter=3000)
    assert not res.t_valid
    assert not np.any(res.sat)
    assert res.status == "ok"
    assert res.gap == pytest.approx(res.primal)            # theta = 0 => D = 0


def test_degenerate_zero_residual_bvls_screens_nothing():
    # n > m with many free coordinates: y in range, theta* = 0, nothing screenable
    P = W.c2_bvls(0, m=60, n=240, dtype=np.float64)
    res = ob.solve(P.A, P.y, P.l, P.u, eps_gap=1e-9, max_iter=100000)
    assert res.status == "ok"
    assert not np.any(res.sat)


def test_reduced_gap_not_above_full_gap():
    A, y, l, u, xs, ths = _planted(5, m=50, n=150, nf=10)
    res = ob.solve(A, y, l, u, eps_gap=1e-10, max_iter=100000, keep_theta=True)
    for h in res.history:
        x = h["x"]
        full_theta = y - A @ x                             # BVLS: residual of the full problem
        full_gap = ob.duality_gap(A, y, l, u, x, full_theta)
        assert h["gap"] <= full_gap + 1e-10 * (1 + full_gap)


def test_gap_decreases_to_zero_and_screening_ratio_grows():
    A, y, l, u, xs, ths = _planted(6)
    res = ob.solve(A, y, l, u, eps_gap=1e-12, max_iter=200000)
    gaps = [h["gap"] for h in res.history]
    act = [h["n_active"] for h in res.history]
    assert gaps[-1] < 1e-12 and gaps[0] > 1e-3
    assert all(a >= b for a, b in zip(act, act[1:]))


def test_screening_same_solution_as_unscreened():
    A, y, l, u, xs, ths = _planted(7)
    eta = 1.0 / ob.lipschitz(A)
    r1 = ob.solve(A, y, l, u, eps_gap=1e-11, step=eta, screening=True, max_iter=10 ** 5)
    r0 = ob.solve(A, y, l, u, eps_gap=1e-11, step=eta, screening=False, max_iter=10 ** 5)
    np.testing.assert_allclose(r1.x, r0.x, atol=1e-6)
    assert r1.iters <= r0.iters + 10


# --- planted mistakes: each pin must fail when the oracle is wrong ----------
def test_planted_mistake_flipped_rule_is_caught(monkeypatch):
    orig = ob.safe_rule

    def flipped(A, theta, radius, u):
        lo, hi = orig(A, -theta, radius, u)     # wrong sign of the correlation
        return lo, hi
    monkeypatch.setattr(ob, "safe_rule", flipped)
    A, y, l, u, xs, ths = _planted(0)
    res = ob.solve(A, y, l, u, eps_gap=1e-10, max_iter=50000)
    bad = (res.sat == -1) & (xs != l) | (res.sat == 1) & (xs != u)
    assert np.any(bad)


def test_planted_mistake_dropped_dual_term_is_caught(monkeypatch):
    orig_dual = ob.dual

    def dual_no_upper(A, y, l, u, theta):      # forgets the u_j [A^T theta]^+ term
        return orig_dual(A, y, l, np.full_like(u, np.inf), theta)
    monkeypatch.setattr(ob, "dual", dual_no_upper)
    rng = W.rng_for(99, 0)
    A = W.unit_columns(rng.standard_normal((30, 60)))
    l, u = -rng.random(60), rng.random(60)
    y, x, th, F = W.planted_bvls(A, l, u, 12, 0.1, rng)
    assert abs(ob.primal(A, y, x) - ob.dual(A, y, l, u, th)) > 1e-6


def test_planted_mistake_min_translation_is_caught(monkeypatch):
    def translate_min(A, z, t, J):
        AJ = A[:, J]
        eps = float(np.min(np.maximum(AJ.T @ z, 0) / np.abs(AJ.T @ t)))
        return z + eps * t, eps
    monkeypatch.setattr(ob, "translate", translate_min)
    rng = np.random.default_rng(0)
    A = np.abs(rng.standard_normal((12, 25)))
    z = rng.standard_normal(12)
    th, _ = ob.translate(A, z, -np.ones(12), np.ones(25, bool))
    assert np.max(A.T @ th) > 1e-6                         # Prop. 1 pin fails
