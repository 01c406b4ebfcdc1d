"""Pins for the dual update (Sec. 4): Prop. 1 (feasibility of the translated
point), Prop. 2 (admissible translation directions), Remark 4 / signed
matrices, and the BVLR residual point."""
import numpy as np
import pytest

from oracle import boxls as ob
from synth import workloads as W


def test_prop1_translation_is_feasible_and_tight():
    rng = np.random.default_rng(10)
    for s in range(30):
        A = np.abs(rng.standard_normal((12, 25)))        # Prop. 2 case 3 matrix
        z = rng.standard_normal(12)
        t = -np.ones(12)
        theta, eps = ob.translate(A, z, t, np.ones(25, bool))
        c = A.T @ theta
        assert np.all(c <= 1e-12)
        if np.any(A.T @ z > 0):
            assert np.max(c) == pytest.approx(0.0, abs=1e-12)   # the maximiser lands on 0
            assert eps > 0
        else:
            assert eps == 0.0 and np.array_equal(theta, z)      # already feasible: no move


def test_translation_identity_on_feasible_points():
    rng = np.random.default_rng(11)
    A = np.abs(rng.standard_normal((10, 20)))
    z = -np.abs(rng.standard_normal(10))                     # A^T z < 0
    theta, eps = ob.translate(A, z, -np.ones(10), np.ones(20, bool))
    assert eps == 0.0 and np.array_equal(theta, z)


def test_prop2_case1_full_column_rank():
    rng = np.random.default_rng(12)
    A = rng.standard_normal((15, 6))
    b = -0.5 - rng.random(6)
    t, *_ = np.linalg.lstsq(A.T, b, rcond=None)
    assert np.allclose(A.T @ t, b)
    assert ob.interior_direction_ok(A, np.full(6, np.inf), t)


def test_prop2_case2_orthogonal():
    rng = np.random.default_rng(13)
    Q, _ = np.linalg.qr(rng.standard_normal((9, 9)))
    beta = -0.1 - rng.random(9)
    t = Q @ beta
    np.testing.assert_allclose(Q.T @ t, beta, atol=1e-12)    # a_i^T t = beta_i ||a_i||^2
    assert ob.interior_direction_ok(Q, np.full(9, np.inf), t)


def test_prop2_case3_nonnegative_matrix():
    rng = np.random.default_rng(14)
    A = rng.random((8, 30))
    assert ob.interior_direction_ok(A, np.full(30, np.inf), -np.ones(8))
    assert ob.interior_direction_ok(A, np.full(30, np.inf), -0.1 - rng.random(8))


def test_prop2_case4_positive_gram_column():
    rng = np.random.default_rng(15)
    A = rng.random((8, 12)) + 0.05
    A[:, 3] = 1.0
    G = A.T @ A
    assert np.all(G[:, 3] > 0)
    assert ob.interior_direction_ok(A, np.full(12, np.inf), -A[:, 3])


def test_signed_gaussian_has_no_valid_minus_one():
    # C1 as specified: signed Gaussian columns, t = -1 is not interior, theta=0
    P = W.c1_nnls(0)
    assert not ob.interior_direction_ok(P.A, P.u, -np.ones(P.m))
    theta, eps, ok = ob.dual_point(P.A, P.y, P.u, np.zeros(P.n), -np.ones(P.m))
    assert not ok and not np.any(theta) and eps == 0.0


def test_bvls_dual_point_is_residual():
    P = W.tiny_bvls(0, 6, 10)
    x = np.clip(np.random.default_rng(0).standard_normal(10), P.l, P.u)
    theta, eps, ok = ob.dual_point(P.A, P.y, P.u, x, -np.ones(6))
    assert ok and eps == 0.0
    np.testing.assert_array_equal(theta, P.y - P.A @ x)


def test_translation_converges_to_theta_star():
    # Prop. 1 second part: Theta(x) -> theta* as x -> x*
    P = W.tiny_nnls(3, 10, 6)
    from oracle.brute import solve_exhaustive
    xs, _ = solve_exhaustive(P.A, P.y, P.l, P.u)
    th_star = P.y - P.A @ xs
    rng = np.random.default_rng(3)
    d = rng.standard_normal(6)
    prev = np.inf
    for h in [1e-1, 1e-2, 1e-3, 1e-4]:
        x = np.maximum(xs + h * d, 0)
        th, _, ok = ob.dual_point(P.A, P.y, P.u, x, -np.ones(10))
        dist = np.linalg.norm(th - th_star)
        assert ok and dist < prev
        prev = dist
    assert prev < 1e-2


# ---------------------------------------------------------------------------
# Translation directions computed from A (Prop. 2, Sec. 5.1 Fig. 2)
# ---------------------------------------------------------------------------
def _brute_scores(A):
    n = A.shape[1]
    s = np.zeros(n)
    for j in range(n):
        bj = A[:, j] / np.linalg.norm(A[:, j])
        for k in range(n):
            if k != j:
                s[j] += bj @ (A[:, k] / np.linalg.norm(A[:, k]))
    return s


def test_correlated_columns_match_brute_force():
    rng = np.random.default_rng(40)
    A = rng.standard_normal((9, 14))
    s = _brute_scores(A)
    t, j = ob.translation_direction(A, "neg_most_correlated")
    assert j == int(np.argmax(s))
    assert np.allclose(t, -A[:, j] / np.linalg.norm(A[:, j]))
    t, j = ob.translation_direction(A, "neg_least_correlated")
    assert j == int(np.argmin(s))
    t, j = ob.translation_direction(A, "neg_mean_column")
    assert j == -1
    assert np.allclose(t, -sum(A[:, k] / np.linalg.norm(A[:, k]) for k in range(14)) / 14)


def test_planted_mistake_argmin_for_most_correlated_is_caught(monkeypatch):
    rng = np.random.default_rng(41)
    A = rng.standard_normal((9, 14))
    real = ob.translation_direction
    monkeypatch.setattr(ob, "translation_direction",
                        lambda A, c: real(A, "neg_least_correlated" if c == "neg_most_correlated" else c))
    _, j = ob.translation_direction(A, "neg_most_correlated")
    assert j != int(np.argmax(_brute_scores(A)))


def test_prop2_case2_orthogonal_mean_column():
    rng = np.random.default_rng(42)
    Q, _ = np.linalg.qr(rng.standard_normal((12, 12)))
    t, _ = ob.translation_direction(Q, "neg_mean_column")
    # a_i^T t = -1/n for every column of an orthogonal matrix
    assert np.allclose(Q.T @ t, -np.ones(12) / 12, atol=1e-14)
    assert ob.interior_direction_ok(Q, np.full(12, np.inf), t)


def test_prop2_case4_positive_gram_column():
    # a signed matrix whose column 3 is positively correlated with every other
    rng = np.random.default_rng(43)
    c = rng.standard_normal(20)
    A = c[:, None] + 0.3 * rng.standard_normal((20, 30))
    A[:, 3] = c
    assert np.all((A.T @ A)[:, 3] > 0)
    assert not np.all(A >= 0)
    t, j = ob.translation_direction(A, "neg_most_correlated")
    assert np.all(A.T @ t < 0)                       # -a_j interior (case 4)
    assert ob.interior_direction_ok(A, np.full(30, np.inf), t)


def test_prop2_case3_every_choice_interior_for_nonnegative_A():
    rng = np.random.default_rng(44)
    A = np.abs(rng.standard_normal((15, 40)))
    for choice in ("neg_mean_column", "neg_most_correlated", "neg_least_correlated"):
        t, _ = ob.translation_direction(A, choice)
        assert np.all(A.T @ t < 0), choice


def test_prop2_case1_normal_equations_direction():
    """Prop. 2, case 1 as the oracle computes it: A^T t = -1 for a tall
    full-rank signed matrix (checked against an independent least-squares
    solve of the transposed system, whose minimum-norm solution is the same
    vector: it lies in the range of A), and t is interior."""
    rng = np.random.default_rng(45)
    A = rng.standard_normal((40, 17))
    t, j = ob.translation_direction(A, "normal_equations")
    assert j == -1
    np.testing.assert_allclose(A.T @ t, -np.ones(17), atol=1e-12)
    t_ls, *_ = np.linalg.lstsq(A.T, -np.ones(17), rcond=None)
    np.testing.assert_allclose(t, t_ls, atol=1e-12)
    assert ob.interior_direction_ok(A, np.full(17, np.inf), t)
    with pytest.raises(ValueError):
        ob.translation_direction(rng.standard_normal((5, 9)), "normal_equations")
