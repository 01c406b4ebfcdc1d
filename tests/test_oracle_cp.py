"""Pins for the Chambolle-Pock primal-dual solver of the oracle (the paper's
second BVLS solver, Sec. 5; Chambolle & Pock 2011): the saddle point is a
fixed point of one iteration (a closed form from the optimality conditions,
Sec. 3.2), the screened solve reaches the exhaustive-search optimum on tiny
instances, and its dual iterate tends to -theta*.  Planted mistakes in the
dual step (a dropped -sigma y, a flipped sign) fail these pins."""
import numpy as np
import pytest

from oracle import boxls as ob
from oracle import brute
from synth import workloads as W


def _planted(seed, m, n, nf, scale=0.3):
    rng = W.rng_for(63, seed, m, n)
    A = W.unit_columns(rng.standard_normal((m, n)))
    l, u = -rng.random(n), rng.random(n)
    y, x_star, theta, F = W.planted_bvls(A, l, u, nf, scale, rng)
    return A, y, l, u, x_star, theta


def test_saddle_point_is_a_fixed_point():
    A, y, l, u, x_star, theta = _planted(0, 30, 80, 10)
    v_star = A @ x_star - y                       # = -theta*
    tau = sigma = 1.0 / (1.05 * np.linalg.norm(A, 2))
    xn, vn = ob.cp_step(A, y, l, u, x_star, v_star, tau, sigma)
    assert np.max(np.abs(xn - x_star)) <= 1e-13
    assert np.max(np.abs(vn - v_star)) <= 1e-13
    assert np.max(np.abs(v_star + theta)) <= 1e-12


@pytest.mark.parametrize("seed", range(4))
def test_screened_cp_reaches_the_exhaustive_optimum(seed):
    P = W.tiny_bvls(seed, 10, 8)
    xs, _ = brute.solve_exhaustive(P.A64(), P.y, P.l, P.u)
    res = ob.solve(P.A64(), P.y, P.l, P.u, solver="cp", K=10, eps_gap=1e-12, max_iter=200000)
    assert res.status == "ok"
    assert np.max(np.abs(res.x - xs)) <= 1e-5
    sl, sh = res.sat == -1, res.sat == 1
    assert np.all(xs[sl] == P.l[sl]) and np.all(xs[sh] == P.u[sh])


def test_dual_iterate_tends_to_minus_theta_star_and_screening_is_safe():
    A, y, l, u, x_star, theta = _planted(1, 50, 150, 15)
    res = ob.solve(A, y, l, u, solver="cp", K=10, eps_gap=1e-11, max_iter=100000, keep_theta=True)
    assert res.status == "ok" and np.count_nonzero(res.sat) > 0
    lo, hi = res.sat == -1, res.sat == 1
    assert np.all(x_star[lo] == l[lo]) and np.all(x_star[hi] == u[hi])
    assert np.max(np.abs(res.x - x_star)) <= 1e-4
    # the residual dual point of the last pass is within the safe radius of theta*
    h = res.history[-1]
    assert np.linalg.norm(h["theta"] - theta) <= h["radius"]


def test_unscreened_cp_same_optimum_as_pg():
    A, y, l, u, x_star, theta = _planted(2, 40, 100, 12)
    r_cp = ob.solve(A, y, l, u, solver="cp", K=10, eps_gap=1e-11, max_iter=100000, screening=False)
    r_pg = ob.solve(A, y, l, u, solver="pg", K=10, eps_gap=1e-11, max_iter=100000, screening=False)
    assert r_cp.status == r_pg.status == "ok"
    assert np.max(np.abs(r_cp.x - r_pg.x)) <= 1e-4


@pytest.mark.parametrize("mistake", ["drop_y", "flip_sign"])
def test_planted_mistake_in_the_dual_step_is_caught(monkeypatch, mistake):
    real = ob.cp_step

    def wrong(A, y, l, u, x, v, tau, sigma):
        xn = ob.project(x - tau * (A.T @ v), l, u)
        xb = 2.0 * xn - x
        if mistake == "drop_y":
            vn = (v + sigma * (A @ xb)) / (1.0 + sigma)
        else:
            vn = (v - sigma * (A @ xb - y)) / (1.0 + sigma)
        return xn, vn

    A, y, l, u, x_star, theta = _planted(0, 30, 80, 10)
    v_star = A @ x_star - y
    tau = sigma = 1.0 / (1.05 * np.linalg.norm(A, 2))
    assert np.max(np.abs(real(A, y, l, u, x_star, v_star, tau, sigma)[1] - v_star)) <= 1e-13
    monkeypatch.setattr(ob, "cp_step", wrong)
    xn, vn = ob.cp_step(A, y, l, u, x_star, v_star, tau, sigma)
    assert np.max(np.abs(vn - v_star)) > 1e-3 or np.max(np.abs(xn - x_star)) > 1e-3
