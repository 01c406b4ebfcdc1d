"""Pins for the oracle's objectives and gap (Sec. 3.1, 3.3, 5; App. B).

Each check ties the oracle to a fact that does not come from the oracle itself:
Fenchel-Young, weak/strong duality at planted optima, Remark 1's l1 form, and
the agreement of two independently written gap formulas.
"""
import numpy as np
import pytest

from oracle import boxls as ob
from synth import workloads as W


def _rand_box_point(rng, l, u):
    uu = np.where(np.isfinite(u), u, l + 3.0)
    return l + (uu - l) * rng.random(l.size)


def test_fconj_fenchel_young():
    # f(z) + f*(v) >= z v with equality iff v = f'(z) = z - y  (definition of f*)
    rng = np.random.default_rng(0)
    z, y, v = rng.standard_normal((3, 1000))
    f = 0.5 * (z - y) ** 2
    assert np.all(f + ob.fconj(v, y) >= z * v - 1e-12)
    np.testing.assert_allclose(f + ob.fconj(z - y, y), z * (z - y), rtol=0, atol=1e-12)


def test_fconj_is_sup_on_grid():
    # f*(v) = sup_z v z - f(z): compare with a dense grid maximisation
    y, v = 0.7, -1.3
    z = np.linspace(-10, 10, 2_000_001)
    brute = np.max(v * z - 0.5 * (z - y) ** 2)
    assert abs(brute - ob.fconj(v, y)) < 1e-9


@pytest.mark.parametrize("kind", ["bvls", "nnls"])
def test_weak_duality(kind):
    rng = np.random.default_rng(1)
    for s in range(20):
        P = W.tiny_bvls(s, 8, 12) if kind == "bvls" else W.tiny_nnls(s, 8, 12)
        A, y, l, u = P.A, P.y, P.l, P.u
        x = _rand_box_point(rng, l, u)
        th = rng.standard_normal(8)
        if kind == "nnls":
            th, _ = ob.translate(A, th, -np.ones(8), ~np.isfinite(u))
            assert ob.dual_feasible(A, u, th, tol=1e-12)
        assert ob.primal(A, y, x) >= ob.dual(A, y, l, u, th) - 1e-10


def test_strong_duality_at_planted_optimum():
    for s in range(5):
        rng = W.rng_for(99, s)
        A = W.unit_columns(rng.standard_normal((30, 60)))
        l, u = -rng.random(60), rng.random(60)
        y, x, th, F = W.planted_bvls(A, l, u, 12, 0.1, rng)
        Pv = ob.primal(A, y, x)
        Dv = ob.dual(A, y, l, u, th)
        assert abs(Pv - Dv) < 1e-12 * max(1.0, abs(Pv))
        assert ob.duality_gap(A, y, l, u, x, th) == pytest.approx(0.0, abs=1e-12)
        assert ob.kkt_violation(A, y, l, u, x) < 1e-12


def test_dual_at_zero_is_zero():
    P = W.tiny_bvls(3, 6, 9)
    assert ob.dual(P.A, P.y, P.l, P.u, np.zeros(6)) == 0.0


def test_remark1_linf_box_gives_l1_penalty():
    # u = -l = delta 1: the two box terms of D equal -delta ||A^T theta||_1
    rng = np.random.default_rng(2)
    A = rng.standard_normal((7, 11))
    y = rng.standard_normal(7)
    th = rng.standard_normal(7)
    delta = 0.37
    l, u = -delta * np.ones(11), delta * np.ones(11)
    D = ob.dual(A, y, l, u, th)
    base = -np.sum(ob.fconj(-th, y))
    assert D == pytest.approx(base - delta * np.sum(np.abs(A.T @ th)), rel=1e-13, abs=1e-13)


@pytest.mark.parametrize("kind", ["bvls", "nnls", "mixed"])
def test_gap_per_coordinate_matches_definition(kind):
    rng = np.random.default_rng(3)
    for s in range(20):
        if kind == "bvls":
            P = W.tiny_bvls(s, 9, 14)
        else:
            P = W.tiny_nnls(s, 9, 14)
            if kind == "mixed":
                P.u = P.u.copy()
                P.u[::2] = 1.0 + rng.random(7)
        A, y, l, u = P.A, P.y, P.l, P.u
        x = _rand_box_point(rng, l, u)
        t = -np.ones(9)
        theta, eps, ok = ob.dual_point(A, y, u, x, t)
        assert ok
        g_def = ob.duality_gap(A, y, l, u, x, theta)
        g_cf = ob.gap_per_coordinate(A, y, l, u, x, theta)
        assert g_cf >= 0.0
        assert abs(g_def - g_cf) <= 1e-11 * (1 + 0.5 * float(y @ y))


def test_gap_per_coordinate_zero_at_optimum():
    rng = W.rng_for(98, 0)
    A = W.unit_columns(rng.standard_normal((40, 80)))
    l, u = -rng.random(80), rng.random(80)
    y, x, th, F = W.planted_bvls(A, l, u, 15, 0.05, rng)
    assert ob.gap_per_coordinate(A, y, l, u, x, y - A @ x) < 1e-13


def test_gap_per_coordinate_any_feasible_theta():
    """The identity holds at any dual-feasible point, not only at the
    residual-based ones: random theta (BVLS, F_D = R^m) and random translated
    points (NNLS), compared with P - D in exact rational arithmetic."""
    from fractions import Fraction as Fr
    rng = np.random.default_rng(5)
    for s in range(6):
        P = W.tiny_bvls(s, 5, 7) if s % 2 == 0 else W.tiny_nnls(s, 5, 7)
        A, y, l, u = P.A, P.y, P.l, P.u
        x = _rand_box_point(rng, l, u)
        th = rng.standard_normal(5)
        if s % 2:
            th, _ = ob.translate(A, th, -np.ones(5), ~np.isfinite(u))
        c = [sum(Fr(A[i, j]) * Fr(th[i]) for i in range(5)) for j in range(7)]
        r = [Fr(y[i]) - sum(Fr(A[i, j]) * Fr(x[j]) for j in range(7)) for i in range(5)]
        Pv = sum(ri * ri for ri in r) / 2
        Dv = sum(Fr(y[i]) ** 2 - (Fr(y[i]) - Fr(th[i])) ** 2 for i in range(5)) / 2
        for j in range(7):
            Dv -= Fr(l[j]) * min(c[j], Fr(0))
            if np.isfinite(u[j]):
                Dv -= Fr(u[j]) * max(c[j], Fr(0))
        exact = float(Pv - Dv)
        assert ob.gap_per_coordinate(A, y, l, u, x, th) == pytest.approx(exact, rel=1e-12, abs=1e-14)
