"""Hand-worked fixtures (tests/golden/*.json): one pass of Alg. 1 (BVLS) and of
Alg. 2 (NNLS with the dual translation of Sec. 4.2) on 3x3 and 2x2 instances
with rational data, every quantity derived by hand in the fixture's
`derivation` field from eqs. Dual_obj, Dual_Gap, GAP_Safe_sph, safe_rule and
BVLR_dual_up / BVLR_dual_up2.  The matrices are not symmetric, so a transposed
operand changes every value; the data are chosen so that a correlation lies
strictly between the thresholds of the radius sqrt(2 Gap) (eq. GAP_Safe_sph)
and of sqrt(Gap): the rule's decision pins the factor 2.

The planted-mistake tests change the oracle and check that a fixture (or the
rounding-floor regression below) then fails."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import boxls as ob
from oracle.brute import solve_exhaustive
from synth import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _num(s):
    return math.inf if s == "inf" else float(Fraction(s))


def _vec(v):
    return np.array([_num(s) for s in v], dtype=np.float64)


def load(name):
    with open(os.path.join(GOLDEN, name + ".json")) as f:
        g = json.load(f)
    A = np.array([[_num(s) for s in row] for row in g["A_rows"]], dtype=np.float64)
    t = None if g["t"] is None else _vec(g["t"])
    return g, A, _vec(g["y"]), _vec(g["l"]), _vec(g["u"]), t


def check_pass1(name):
    """Run the oracle's building blocks and its screening loop on a fixture and
    compare every first-pass quantity with the hand derivation."""
    g, A, y, l, u, t = load(name)
    e = g["expected_pass1"]
    eta = float(Fraction(g["step"]))
    x0 = _vec(g["x0"])
    tt = -np.ones(A.shape[0]) if t is None else t
    rel = dict(rel=1e-14, abs=1e-15)

    # building blocks
    x1 = ob.pg_step(A, y, l, u, x0, eta)
    np.testing.assert_allclose(x1, _vec(e["x"]), rtol=1e-15, atol=1e-15)
    theta, eps, ok = ob.dual_point(A, y, u, x1, tt)
    assert ok
    np.testing.assert_allclose(theta, _vec(e["theta"]), rtol=1e-15, atol=1e-15)
    assert eps == pytest.approx(_num(e["eps"]), **rel)
    np.testing.assert_allclose(A.T @ theta, _vec(e["corr"]), rtol=1e-15, atol=1e-15)
    assert ob.primal(A, y, x1) == pytest.approx(_num(e["primal"]), **rel)
    assert ob.dual(A, y, l, u, theta) == pytest.approx(_num(e["dual"]), **rel)
    G = ob.gap_per_coordinate(A, y, l, u, x1, theta)
    assert G == pytest.approx(_num(e["gap"]), **rel)
    assert ob.duality_gap(A, y, l, u, x1, theta) == pytest.approx(_num(e["gap"]), **rel)
    r = ob.safe_radius(G)
    assert r * r == pytest.approx(_num(e["radius_squared"]), **rel)
    lo, hi = ob.safe_rule(A, theta, r, u)
    assert lo.tolist() == e["screen_lower"] and hi.tolist() == e["screen_upper"]

    # the same pass inside the loop: one PG step per pass, two passes (the
    # second ends the run at max_iter, after the first pass's fix and fold)
    res = ob.solve(A, y, l, u, solver="pg", K=1, eps_gap=0.0, max_iter=2, step=eta, t=t, x0=x0,
                   keep_theta=True)
    h = res.history[0]
    assert h["iters"] == 1 and h["n_active"] == A.shape[1]
    np.testing.assert_allclose(h["x"], _vec(e["x"]), rtol=1e-15, atol=1e-15)
    np.testing.assert_allclose(h["theta"], _vec(e["theta"]), rtol=1e-15, atol=1e-15)
    assert h["gap"] == pytest.approx(_num(e["gap"]), **rel)
    assert h["radius"] ** 2 == pytest.approx(_num(e["radius_squared"]), **rel)
    assert h["eps"] == pytest.approx(_num(e["eps"]), **rel)
    expect_sat = np.where(e["screen_lower"], -1, np.where(e["screen_upper"], 1, 0))
    assert res.sat.tolist() == expect_sat.tolist()
    return g, A, y, l, u


@pytest.mark.parametrize("name", ["gap_safe_bvls_pass1", "gap_safe_nnls_translation_pass1"])
def test_golden_first_pass(name):
    g, A, y, l, u = check_pass1(name)
    # the fixtures are built so that the factor 2 matters
    e = g["expected_pass1"]
    assert e["screen_lower"] != e["screen_lower_if_radius_were_sqrt_gap"]


def test_golden_bvls_decision_is_safe():
    """The coordinate the fixture's first pass screens at l_0 sits at l_0 in
    the exact optimum (exhaustive search over saturation patterns)."""
    g, A, y, l, u, t = load("gap_safe_bvls_pass1")
    xs, pat = solve_exhaustive(A, y, l, u)
    assert xs[0] == l[0] and pat[0] == -1
    assert ob.kkt_violation(A, y, l, u, xs) < 1e-12


def test_golden_kkt_violation():
    """kkt_violation (eqs. optimality1-2) reports the hand-computed violation
    at points that are not optimal: a free coordinate with a correlation, a
    lower-bound coordinate with a positive correlation, an upper-bound one
    with a negative correlation."""
    g, A, y, l, u, t = load("gap_safe_bvls_pass1")
    for case in g["kkt_violation"]:
        assert ob.kkt_violation(A, y, l, u, _vec(case["x"])) == pytest.approx(_num(case["value"]), rel=1e-15), case


def test_kkt_violation_reports_infeasibility():
    g, A, y, l, u, t = load("gap_safe_bvls_pass1")
    xs, _ = solve_exhaustive(A, y, l, u)
    bad = xs.copy()
    bad[1] = u[1] + 0.25                         # outside the box by 1/4
    assert ob.kkt_violation(A, y, l, u, bad) >= 0.25


# --- rounding floor ---------------------------------------------------------
def _floor_instance():
    m, n = 2000, 300
    rng = W.rng_for(90, 21, m, n)
    A = np.asfortranarray(W.unit_columns(rng.standard_normal((m, n))).astype(np.float32))
    l, u = -rng.random(n), rng.random(n)
    y, x, th, F = W.planted_bvls(A, l, u, int(0.02 * m), 0.05, rng)
    return A.astype(np.float64), y, l, u, x


def check_floor_safety():
    """Run the oracle well past the point where its gap reaches FP64's rounding
    floor (eps_gap = 0, 600 iterations on a planted FP32-stored instance) and
    check that every screened coordinate is saturated at the planted optimum."""
    A, y, l, u, xs = _floor_instance()
    eta = 1.0 / (1.05 * ob.lipschitz(A))
    res = ob.solve(A, y, l, u, K=10, eps_gap=0.0, max_iter=600, step=eta)
    assert np.all(xs[res.sat == -1] == l[res.sat == -1])
    assert np.all(xs[res.sat == 1] == u[res.sat == 1])
    return res, xs, l, u


def test_screening_safe_at_the_rounding_floor():
    res, xs, l, u = check_floor_safety()
    free = (xs > l) & (xs < u)
    assert res.gap < 1e-13
    assert np.count_nonzero(res.sat) == np.count_nonzero(~free)   # every saturated coordinate found


# --- planted mistakes: each must make a pin fail ---------------------------
def test_planted_mistake_radius_without_factor_two_is_caught(monkeypatch):
    """r = sqrt(Gap) instead of sqrt(2 Gap) (eq. GAP_Safe_sph).  With the
    residual dual point this smaller sphere still happens to contain theta*
    (the gap bounds ||theta - theta*||^2 there), so no safety pin can see it;
    the fixtures' decisions do."""
    monkeypatch.setattr(ob, "safe_radius", lambda gap, alpha=1.0: math.sqrt(max(gap, 0.0) / alpha))
    for name in ("gap_safe_bvls_pass1", "gap_safe_nnls_translation_pass1"):
        with pytest.raises(AssertionError):
            check_pass1(name)


def test_planted_mistake_transposed_correlation_is_caught(monkeypatch):
    """A^T r computed as A r (a transposed operand) in the residual dual point's
    correlations: the fixtures' non-symmetric matrices expose it."""
    orig = ob.safe_rule

    def rule_untransposed(A, theta, radius, u):
        return orig(np.asarray(A).T, theta, radius, u)
    monkeypatch.setattr(ob, "safe_rule", rule_untransposed)
    with pytest.raises(AssertionError):
        check_pass1("gap_safe_bvls_pass1")


def test_planted_mistake_gap_by_subtraction_is_caught(monkeypatch):
    """The loop's gap evaluated as P - D (two terms of the size of 1/2||y||^2
    subtracted) instead of the per-coordinate form: past the rounding floor
    the computed gap is noise, the radius collapses and free coordinates get
    screened."""
    monkeypatch.setattr(ob, "gap_per_coordinate",
                        lambda A, y, l, u, x, theta, delta=math.inf: ob.duality_gap(A, y, l, u, x, theta, delta))
    with pytest.raises(AssertionError):
        check_floor_safety()
