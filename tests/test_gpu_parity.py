"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs, same step, same schedule.  Sizes span several work items
and a ragged tail of columns and rows, every kernel bucket of m, FP64 and FP32
storage, PG and CD, NNLS / BVLS / mixed bounds, screened and unscreened.

Tolerance: both sides compute in FP64, so trajectory parity is checked at
1e-9 relative to max(1, ||x||_inf), far inside the 1e-6 (FP64) and 1e-4
(FP32 storage) bars; screened sets must be identical."""
import numpy as np
import pytest
import torch

from oracle import boxls as ob
from synth import workloads as W
from tests.gpu_helpers import assert_parity, check_parity, parity_vs_oracle, run_gpu, run_oracle

pytestmark = pytest.mark.gpu


def planted(seed, m, n, nf_frac=0.4, scale=0.05, dtype=np.float64, box=None):
    rng = W.rng_for(90, seed, m, n)
    A = np.asfortranarray(W.unit_columns(rng.standard_normal((m, n))).astype(dtype))
    if box is None:
        l, u = -rng.random(n), rng.random(n)
    else:
        l, u = np.full(n, box[0]), np.full(n, box[1])
    y, x, th, F = W.planted_bvls(A, l, u, int(nf_frac * m), scale, rng)
    return W.Problem(A, y, l, u, x, True, {})


def step_of(P):
    return 1.0 / (1.05 * ob.lipschitz(P.A64()))


@pytest.mark.parametrize("m,n", [(50, 173), (120, 301), (300, 1000), (700, 1800), (1500, 3333), (3001, 6007)])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_pg_bvls_trajectory_parity(m, n, dtype):
    print(f"\n[pg bvls] m={m} n={n} {np.dtype(dtype).name}", flush=True)
    P = planted(1, m, n, dtype=dtype)
    eta = step_of(P)
    kw = dict(screen_every=10, eps_gap=1e-8, max_iter=4000, step=eta)
    xg, sg, info, res = check_parity(P, "bvls", **kw)
    assert res.status == "ok" and np.count_nonzero(res.sat) > 0


def test_pg_unscreened_parity():
    P = planted(2, 300, 900)
    eta = step_of(P)
    kw = dict(screen_every=10, eps_gap=1e-9, max_iter=5000, step=eta, screening=False)
    xg, sg, info, res = check_parity(P, "bvls", **kw)
    assert not np.any(sg)


def test_pg_nnls_companion_parity():
    P = W.c1_companion(0)                       # 200 x 500, A >= 0, t = -1 interior
    eta = step_of(P)
    kw = dict(screen_every=10, eps_gap=1e-9, max_iter=3000, step=eta)
    xg, sg, info, res = check_parity(P, "nnls", **kw)
    assert info["t_valid"] == 1


def test_pg_nnls_translation_screens():
    # well-conditioned non-negative matrix: dual translation along t = -1
    # certifies most zero coordinates within a few hundred iterations
    rng = W.rng_for(93, 0)
    n = 200
    A = np.asfortranarray(np.diag(0.5 + rng.random(n)) + 0.05 * rng.random((n, n)))
    P = W.Problem(A, rng.standard_normal(n), np.zeros(n), np.full(n, np.inf))
    kw = dict(screen_every=10, eps_gap=1e-9, max_iter=5000, step=step_of(P))
    xg, sg, info, res = check_parity(P, "nnls", **kw)
    assert res.status == "ok" and np.count_nonzero(sg) > n // 2 and info["eps"] >= 0.0


def test_pg_nnls_c1_as_specified():
    # signed Gaussian columns: t = -1 is not interior, theta = 0, nothing screened
    P = W.c1_nnls(0)
    eta = step_of(P)
    kw = dict(screen_every=10, eps_gap=1e-9, max_iter=4000, step=eta)
    xg, sg, info, res = check_parity(P, "nnls", **kw)
    assert info["t_valid"] == 0 and not np.any(sg) and info["status_name"] == "ok"


def test_pg_nnls_user_direction():
    # signed A with an interior direction from an LP: screening becomes possible
    rng = W.rng_for(91, 0)
    A = np.asfortranarray(rng.standard_normal((40, 60)))
    t = W.interior_direction(A)
    assert t is not None
    y = rng.standard_normal(40)
    P = W.Problem(A, y, np.zeros(60), np.full(60, np.inf))
    eta = step_of(P)
    kw = dict(screen_every=5, eps_gap=1e-10, max_iter=20000, step=eta, t=t)
    xg, sg, info, res = check_parity(P, "nnls", **kw)


def test_pg_nnls_tall_full_rank_direction():
    """Prop. 2, first case: a tall full-rank A (n <= m), signed entries, and t
    solving A^T t = -1 is interior; the translated dual point then screens."""
    rng = W.rng_for(95, 0)
    m, n = 120, 80
    A = np.asfortranarray(W.unit_columns(rng.standard_normal((m, n))))
    t, *_ = np.linalg.lstsq(A.T, -np.ones(n), rcond=None)      # least-norm solution, A^T t = -1
    assert np.allclose(A.T @ t, -1.0) and ob.interior_direction_ok(A, np.full(n, np.inf), t)
    y = A @ np.maximum(rng.standard_normal(n), 0.0) - 0.5 * rng.random(m)
    P = W.Problem(A, y, np.zeros(n), np.full(n, np.inf))
    kw = dict(screen_every=5, eps_gap=1e-10, max_iter=20000, step=step_of(P), t=t)
    xg, sg, info, res = check_parity(P, "nnls", **kw)
    assert res.status == "ok" and info["t_valid"] == 1


def test_pg_linf_box_special_case():
    """App. A: the l-infinity-constrained problem (u = -l = c 1) is a BVLS
    instance; parity with the oracle, and coordinates screened at both ends."""
    P = planted(23, 300, 900, box=(-0.3, 0.3))
    kw = dict(screen_every=10, eps_gap=1e-9, max_iter=4000, step=step_of(P))
    xg, sg, info, res = check_parity(P, "bvls", **kw)
    assert np.count_nonzero(sg == -1) > 0 and np.count_nonzero(sg == 1) > 0


def test_pg_mixed_bounds():
    rng = W.rng_for(92, 0)
    P = W.c1_companion(1, 100, 260)
    u = P.u.copy()
    u[::3] = 0.2 + rng.random(u[::3].size)
    P = W.Problem(P.A, P.y, P.l, u)
    eta = step_of(P)
    kw = dict(screen_every=10, eps_gap=1e-9, max_iter=3000, step=eta)
    xg, sg, info, res = check_parity(P, "bvls", **kw)


@pytest.mark.parametrize("m,n", [(40, 97), (200, 450)])
def test_cd_parity(m, n):
    print(f"\n[cd bvls] m={m} n={n}", flush=True)
    P = planted(3, m, n)
    kw = dict(solver="cd", screen_every=1, eps_gap=1e-10, max_iter=2000)
    xg, sg, info, res = check_parity(P, "bvls", xtol=1e-8, **kw)


@pytest.fixture(params=[1, 0], ids=["block", "one_wg"])
def cd_block(request):
    """Single-problem CD as the block-sequential sweep (Gram blocks, one
    launch per block of 128 positions) and as the one-workgroup sweep."""
    from paper_2202_07258_amd import native as N
    N.set_cd_block(request.param)
    yield request.param
    N.set_cd_block(1)


@pytest.mark.parametrize("m,n", [(700, 1500), (2000, 1300), (4000, 900), (6000, 800), (9000, 700)])
def test_cd_parity_multiwave(m, n, cd_block):
    """Large single problems: the block-sequential sweep (several blocks, a
    ragged last block, m not a multiple of the 64-row chunks) and the
    one-workgroup sweep whose workgroup spans several waves (m > 512: 256,
    512 and 1024 threads).  Tall shapes keep |F| = 0.4 min(m, n) free
    coordinates."""
    print(f"\n[cd bvls multi-wave] m={m} n={n} block={cd_block}", flush=True)
    P = planted(23, m, n, nf_frac=0.4 * min(m, n) / m)
    kw = dict(solver="cd", screen_every=1, eps_gap=1e-10, max_iter=2000)
    xg, sg, info, res = check_parity(P, "bvls", xtol=1e-8, **kw)
    assert res.status == "ok" and np.count_nonzero(res.sat) > 0


@pytest.mark.parametrize("screening,dtype", [(True, np.float64), (False, np.float64), (True, np.float32)])
def test_cd_block_sweeps_match_oracle(screening, dtype, cd_block):
    """Fixed budget of 60 CD sweeps (Sec. 5 CD solver), screening every 5, on
    a BVLS problem of 5 blocks of 128 with a ragged last one (n = 601) and
    m = 1001 rows, A stored in FP64 or FP32: the gap and preserved-set size
    after every pass match the oracle's.  With screening the list shrinks over several passes to 400
    (4 blocks), so the Gram blocks are re-formed after those passes and
    reused after the others."""
    print(f"\n[cd bvls sweeps] screening={screening} {np.dtype(dtype).name} block={cd_block}", flush=True)
    P = planted(31, 1001, 601, dtype=dtype)
    kw = dict(solver="cd", screening=screening, screen_every=5, eps_gap=0.0, max_iter=60)
    xg, sg, info, res = check_parity(P, "bvls", xtol=1e-8, history=64, **kw)
    assert info["iters"] == res.iters == 60
    if screening:
        assert res.history[0]["n_active"] == 601 and res.history[-1]["n_active"] <= 450
    for hg, ho in zip(info["history"], res.history):
        assert hg["n_active"] == ho["n_active"]
        assert hg["gap"] == pytest.approx(ho["gap"], rel=1e-6, abs=1e-11)


@pytest.mark.parametrize("m,n", [(1, 3), (5, 64), (70, 128), (64, 129), (63, 191), (130, 300)])
def test_cd_block_edge_shapes(m, n, cd_block):
    """Block-sequential CD at its boundaries: one row; a block of exactly 64
    or 128 positions; a second block of one column; rows not filling the
    64-row chunk; the second half of a block (positions 64-127) partly used.
    A fixed budget of sweeps with screening every 5, against the oracle."""
    print(f"\n[cd edge] m={m} n={n} block={cd_block}", flush=True)
    rng = W.rng_for(95, 0, m, n)
    A = np.asfortranarray(rng.standard_normal((m, n)))
    P = W.Problem(A, rng.standard_normal(m), -np.ones(n), np.ones(n), None, False, {})
    kw = dict(solver="cd", screen_every=5, eps_gap=0.0, max_iter=30)
    xg, sg, info, res = check_parity(P, "bvls", xtol=1e-8, **kw)
    assert info["iters"] == res.iters == 30


@pytest.mark.parametrize("solver,dtype", [("pg", np.float32), ("pg", np.float64), ("cd", np.float64)])
def test_oracle_dual_point_parity(solver, dtype):
    """Screening informed with the planted dual optimum theta* (Sec. 5.1,
    Fig. 3) in place of the dual update: same passes, gaps and screened sets
    as the oracle run with the same theta*, and at least as many coordinates
    screened as with the usual dual update."""
    rng = W.rng_for(91, 0, 400, 1300)
    A = np.asfortranarray(W.unit_columns(rng.standard_normal((400, 1300))).astype(dtype))
    l, u = -rng.random(1300), rng.random(1300)
    y, x_star, theta, F = W.planted_bvls(A.astype(np.float64), l, u, 160, 0.05, rng)
    P = W.Problem(A, y, l, u, x_star, True, {})
    kw = dict(solver=solver, screen_every=10 if solver == "pg" else 1, eps_gap=1e-9, max_iter=20000)
    if solver == "pg":
        kw["step"] = step_of(P)
    xg, sg, info, res = check_parity(P, "bvls", xtol=1e-8, theta_star=theta, history=2000, **kw)
    assert res.status == "ok"
    h = info["history"]
    for hg, ho in zip(h, res.history):
        assert hg["n_active"] == ho["n_active"]
        assert hg["gap"] == pytest.approx(ho["gap"], rel=1e-6, abs=1e-11)
    lo, hi = sg == -1, sg == 1
    assert np.all(x_star[lo] == l[lo]) and np.all(x_star[hi] == u[hi])
    usual = run_oracle(P, **{k: v for k, v in kw.items()})
    assert np.count_nonzero(sg) >= np.count_nonzero(usual.sat)


@pytest.mark.parametrize("choice", ["neg_mean_column", "neg_most_correlated", "neg_least_correlated"])
def test_library_translation_direction(choice):
    """t computed by the library from A (Prop. 2 and the choices of Sec. 5.1,
    Fig. 2) on a non-negative NNLS instance: the same column as the oracle's
    choice, and the trajectory of the oracle run with the oracle's t."""
    P = W.c1_companion(4, 150, 400)
    t_ora, j = ob.translation_direction(P.A64(), choice)
    kw = dict(screen_every=10, eps_gap=1e-9, max_iter=3000, step=step_of(P))
    xg, sg, info = run_gpu(P, "nnls", t_choice=choice, **kw)
    assert info["t_column"] == j and info["t_valid"] == 1
    parity_vs_oracle(P, xg, sg, info, t=t_ora, **kw)


def test_library_translation_direction_prop2_cases_2_and_4():
    """Prop. 2 case 2 (orthogonal A: the negative mean column is interior) and
    case 4 (a signed A whose Gram matrix has a positive column: minus that
    column is interior), both chosen by the library."""
    rng = W.rng_for(92, 0)
    Q, _ = np.linalg.qr(rng.standard_normal((300, 300)))
    y = rng.standard_normal(300)
    P = W.Problem(np.asfortranarray(Q), y, np.zeros(300), np.full(300, np.inf))
    t_ora, _ = ob.translation_direction(Q, "neg_mean_column")
    # a small step keeps PG from converging in one pass, so screening fires
    kw = dict(screen_every=1, eps_gap=1e-9, max_iter=2000, step=0.2)
    xg, sg, info = run_gpu(P, "nnls", t_choice="neg_mean_column", **kw)
    assert info["t_valid"] == 1 and np.count_nonzero(sg) > 0
    parity_vs_oracle(P, xg, sg, info, t=t_ora, **kw)
    # the closed-form optimum of an orthogonal problem, x* = max(Q^T y, 0)
    assert np.max(np.abs(xg - np.maximum(Q.T @ y, 0.0))) <= 1e-4
    rng = W.rng_for(92, 1)
    c = rng.standard_normal(200)
    A = c[:, None] + 2.0 * rng.standard_normal((200, 500))
    A[:, 3] = c
    y = A @ (np.abs(rng.standard_normal(500)) * (rng.random(500) < 0.05)) + 0.5 * rng.standard_normal(200)
    P = W.Problem(np.asfortranarray(A), y, np.zeros(500), np.full(500, np.inf))
    t_ora, j = ob.translation_direction(A, "neg_most_correlated")
    assert j == 3 and np.all(A.T @ t_ora < 0) and not np.all(A >= 0)
    # a fixed budget: PG needs ~1e5 iterations to a small gap on this matrix
    kw = dict(screen_every=10, eps_gap=1e-9, max_iter=3000, step=step_of(P))
    xg, sg, info = run_gpu(P, "nnls", t_choice="neg_most_correlated", **kw)
    assert info["t_column"] == j and info["t_valid"] == 1
    parity_vs_oracle(P, xg, sg, info, t=t_ora, **kw)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_library_translation_direction_prop2_case_1(dtype):
    """Prop. 2 case 1 computed by the library: t = A v with A^T A v = -1 by
    conjugate gradients on a tall signed matrix of full column rank (where
    t = -1 is not interior); the trajectory and screened sets of the oracle
    run with its exact solve of the same system."""
    rng = W.rng_for(92, 2)
    m, n = 600, 250
    A = np.asfortranarray(W.unit_columns(rng.standard_normal((m, n))).astype(dtype))
    xs = np.abs(rng.standard_normal(n)) * (rng.random(n) < 0.3)
    y = A.astype(np.float64) @ xs + 0.1 * rng.standard_normal(m)
    P = W.Problem(A, y, np.zeros(n), np.full(n, np.inf))
    t_ora, _ = ob.translation_direction(P.A64(), "normal_equations")
    assert not ob.interior_direction_ok(P.A64(), P.u, -np.ones(m))
    kw = dict(screen_every=10, eps_gap=1e-9, max_iter=4000, step=step_of(P))
    xg, sg, info = run_gpu(P, "nnls", t_choice="normal_equations", **kw)
    assert info["t_valid"] == 1 and info["t_column"] == -1 and np.count_nonzero(sg) > 0
    parity_vs_oracle(P, xg, sg, info, t=t_ora, **kw)


def test_cd_nnls_parity():
    P = W.c1_companion(2, 150, 400)
    kw = dict(solver="cd", screen_every=1, eps_gap=1e-9, max_iter=3000)
    xg, sg, info, res = check_parity(P, "nnls", xtol=1e-8, **kw)


def _hash_start(m):
    """Start vector of the library's Lanczos estimate: 1 +- 1/4 by the top bit
    of Knuth's multiplicative hash i * 2654435761 mod 2^32 of the row index."""
    h = (np.arange(m, dtype=np.uint64) * np.uint64(2654435761)) & np.uint64(0xFFFFFFFF)
    return np.where((h >> np.uint64(31)) != 0, 1.25, 0.75)


@pytest.mark.parametrize("m,n,dtype,steps", [(500, 1500, np.float32, 0), (500, 1500, np.float64, 3),
                                             (777, 300, np.float32, 20), (6, 40, np.float64, 8),
                                             (9000, 300, np.float32, 0), (16384, 100, np.float64, 12)])
def test_step_estimate(m, n, dtype, steps):
    """The default step 1 / (1.05 L_est): L_est is the oracle's Lanczos
    estimate from the same start vector (8 steps by default), a lower bound of
    ||A||_2^2, within 10% of it from 8 steps on (exact when m <= steps)."""
    P = planted(4, m, n, dtype=dtype)
    xg, sg, info = run_gpu(P, "bvls", eps_gap=1e-6, max_iter=50, power_iters=steps)
    L = ob.lipschitz(P.A64())
    est = ob.lipschitz_lanczos(P.A64(), steps if steps > 0 else 8, _hash_start(m))
    assert info["lipschitz"] == pytest.approx(est, rel=1e-9)
    assert info["lipschitz"] <= L * (1 + 1e-12)
    if steps == 0 or steps >= 8:
        assert info["lipschitz"] >= 0.9 * L
    if m <= max(steps, 8):
        assert info["lipschitz"] == pytest.approx(L, rel=1e-9)
    assert info["step"] == pytest.approx(1.0 / (1.05 * info["lipschitz"]), rel=1e-15)


def test_warm_start_and_max_iter():
    P = planted(5, 100, 300)
    eta = step_of(P)
    x0 = np.clip(np.random.default_rng(0).standard_normal(300), P.l, P.u)
    kw = dict(screen_every=7, eps_gap=1e-14, max_iter=50, step=eta, x0=x0)
    res = run_oracle(P, **kw)
    xg, sg, info = run_gpu(P, "bvls", **kw)
    assert info["status_name"] == "maxiter" and info["iters"] == 50
    assert_parity(P, xg, sg, info, res)


def test_edge_single_column_and_row():
    rng = np.random.default_rng(7)
    for m, n in [(1, 1), (1, 7), (9, 1)]:
        A = np.asfortranarray(rng.standard_normal((m, n)))
        P = W.Problem(A, rng.standard_normal(m), -np.ones(n), np.ones(n))
        eta = step_of(P)
        kw = dict(screen_every=3, eps_gap=1e-12, max_iter=3000, step=eta)
        xg, sg, info, res = check_parity(P, "bvls", **kw)


def test_everything_screened():
    # orthonormal columns, 39 coordinates pushed far outside the box and one
    # that reaches its bound slowly (step 0.3): the preserved set empties
    Q, _ = np.linalg.qr(W.rng_for(94, 0).standard_normal((64, 40)))
    c = 3.0 * np.sign(W.rng_for(94, 1).standard_normal(40))
    c[39] = 0.55
    P = W.Problem(np.asfortranarray(Q), Q @ c, -0.5 * np.ones(40), 0.5 * np.ones(40))
    kw = dict(screen_every=1, eps_gap=1e-9, max_iter=100, step=0.3)
    xg, sg, info, res = check_parity(P, "bvls", **kw)
    assert info["n_active"] == 0 and np.all(sg != 0) and res.status == "ok"


def test_determinism():
    P = planted(6, 800, 2500, dtype=np.float32)
    kw = dict(eps_gap=1e-8, max_iter=3000)
    x1, s1, i1 = run_gpu(P, "bvls", **kw)
    x2, s2, i2 = run_gpu(P, "bvls", **kw)
    assert np.array_equal(x1, x2) and np.array_equal(s1, s2) and i1["iters"] == i2["iters"]


@pytest.mark.parametrize("solver,m,n", [("pg", 300, 900), ("cd", 300, 900), ("pg", 9000, 400)])
def test_graph_replay_matches_direct_launches(solver, m, n):
    """Regular passes replayed from one captured HIP graph give bit-identical
    results to direct launches, with the program's own eager work (other
    solves, host synchronisation) between calls; pass records agree too.
    The 9000-row case replays the two-pass sweeps of the largest row class."""
    P = planted(16, m, n, dtype=np.float32)
    eta = step_of(P)
    kw = dict(solver=solver, eps_gap=1e-9, max_iter=4000, step=eta, screen_every=5, history=1000)
    xd, sd, idd = run_gpu(P, "bvls", graph=False, **kw)
    for _ in range(2):
        xg, sg, ig = run_gpu(P, "bvls", graph=True, **kw)
        assert np.array_equal(xd, xg) and np.array_equal(sd, sg)
        assert idd["iters"] == ig["iters"] and idd["passes"] == ig["passes"] and idd["gap"] == ig["gap"]
        assert [h["gap"] for h in idd["history"]] == [h["gap"] for h in ig["history"]]
        assert [h["iters"] for h in idd["history"]] == [h["iters"] for h in ig["history"]]
        run_gpu(planted(17, 100, 300), "bvls", eps_gap=1e-8, max_iter=500)       # unrelated eager work
    parity_vs_oracle(P, xg, sg, ig, solver=solver, eps_gap=1e-9, max_iter=4000, step=eta, screen_every=5)


def test_cd_block_profile_mode_matches_direct():
    """Block CD with per-sweep events (profile mode: the host waits on events,
    the launches are still sized by the published preserved-list length)
    gives the direct launches' result bit for bit."""
    P = planted(16, 300, 900, dtype=np.float32)
    kw = dict(solver="cd", eps_gap=1e-9, max_iter=4000, step=step_of(P), screen_every=5)
    xd, sd, idd = run_gpu(P, "bvls", **kw)
    xp, sp, ip = run_gpu(P, "bvls", profile=True, **kw)
    assert np.array_equal(xd, xp) and np.array_equal(sd, sp)
    assert idd["iters"] == ip["iters"] and idd["passes"] == ip["passes"] and idd["gap"] == ip["gap"]
    assert ip["sweep_launches"] > 0 and np.count_nonzero(sd) > 0


def test_history_records():
    P = planted(7, 200, 600)
    eta = step_of(P)
    res = run_oracle(P, screen_every=10, eps_gap=1e-9, step=eta)
    xg, sg, info = run_gpu(P, "bvls", screen_every=10, eps_gap=1e-9, step=eta, history=1000)
    h = info["history"]
    assert len(h) == res.passes
    for hg, ho in zip(h, res.history):
        assert hg["iters"] == ho["iters"] and hg["n_active"] == ho["n_active"]
        assert hg["gap"] == pytest.approx(ho["gap"], rel=1e-6, abs=1e-11)


def test_info_dual_margin_and_free_count():
    """info.dual is the dual objective of the last pass (primal - gap, a lower
    bound of the optimum), info.n_free the count of coordinates strictly
    inside the box, info.max_margin the correlation margin per unit norm."""
    P = planted(9, 250, 700)
    kw = dict(screen_every=10, eps_gap=1e-9, step=step_of(P))
    xg, sg, info = run_gpu(P, "bvls", **kw)
    assert info["dual"] == pytest.approx(info["primal"] - info["gap"], rel=1e-15, abs=1e-15)
    p_star = ob.primal(P.A64(), P.y, P.x_true)
    assert info["dual"] <= p_star * (1 + 1e-12) + 1e-15
    assert info["n_free"] == int(np.count_nonzero((xg > P.l) & (xg < P.u)))
    assert 0.0 < info["max_margin"] < 1e-10


def test_device_side_validation():
    import paper_2202_07258_amd as bx
    P = planted(8, 30, 50)
    A, y, l, u = (torch.tensor(v, device="cuda") for v in (P.A, P.y, P.l, P.u))
    A = bx.colmajor(P.A)
    ybad = y.clone(); ybad[3] = float("nan")
    with pytest.raises(bx.BoxscreenError, match="err_nonfinite"):
        bx.solve_bvls(A, ybad, l, u)
    lbad = l.clone(); lbad[5] = u[5] + 1.0
    with pytest.raises(bx.BoxscreenError, match="err_bounds"):
        bx.solve_bvls(A, y, lbad, u)
    lbad = l.clone(); lbad[5] = -float("inf")
    with pytest.raises(bx.BoxscreenError, match="err_bounds"):
        bx.solve_bvls(A, y, lbad, u)
    Abad = P.A.copy(); Abad[7, 11] = np.inf
    with pytest.raises(bx.BoxscreenError, match="err_nonfinite"):
        bx.solve_bvls(bx.colmajor(Abad), y, l, u)
    # one failing instance of a batch fails the call; the others still run and
    # the next call is unaffected
    good = {"A": A, "y": y, "l": l, "u": u}
    with pytest.raises(bx.BoxscreenError, match="err_nonfinite"):
        bx.solve_bvls_varbatch([good, {"A": A, "y": ybad, "l": l, "u": u}, good], eps_gap=1e-9)
    x, _, info = bx.solve_bvls(A, y, l, u, eps_gap=1e-9, step=step_of(P))
    assert info["status_name"] == "ok"
    res = ob.solve(P.A64(), P.y, P.l, P.u, K=10, eps_gap=1e-9, step=step_of(P))
    assert np.max(np.abs(x.cpu().numpy() - res.x)) <= 1e-9 * max(1.0, float(np.max(np.abs(res.x))))


def test_varbatch_parity():
    shapes = [(37, 120), (64, 200), (130, 300), (257, 700), (513, 1100), (1100, 2500), (2100, 4400)]
    probs = [planted(10 + i, m, n, dtype=np.float32, box=(0.0, 1.0)) for i, (m, n) in enumerate(shapes)]
    eta = 1.0 / (1.05 * max(ob.lipschitz(P.A64()) for P in probs))
    import paper_2202_07258_amd as bx
    from tests.gpu_helpers import to_dev
    dev = []
    for P in probs:
        A, y, l, u = to_dev(P)
        dev.append({"A": A, "y": y, "l": l, "u": u})
    kw = dict(screen_every=10, eps_gap=1e-8, max_iter=5000, step=eta)
    xs, sats, infos, status = bx.solve_bvls_varbatch(dev, **kw)
    torch.cuda.synchronize()
    for P, x, s, info in zip(probs, xs, sats, infos):
        parity_vs_oracle(P, x.cpu().numpy(), s.cpu().numpy(), info, **kw)
    assert status == "ok"
    # the same batch with every regular pass replayed from one captured graph:
    # bit-identical results, twice, with unrelated eager work in between
    for _ in range(2):
        xg, sg, ig, stg = bx.solve_bvls_varbatch(dev, graph=True, **kw)
        torch.cuda.synchronize()
        assert stg == status
        for a, b, c, d, i1, i2 in zip(xs, xg, sats, sg, infos, ig):
            assert torch.equal(a, b) and torch.equal(c, d)
            assert (i1["iters"], i1["passes"], i1["gap"]) == (i2["iters"], i2["passes"], i2["gap"])
        run_gpu(planted(17, 100, 300), "bvls", eps_gap=1e-8, max_iter=500)


def _padded_colmajor(A, device="cuda"):
    """Column-major device copy with the leading dimension rounded up to 4
    elements (16-byte aligned columns), as the uneven-batch benchmark lays
    its matrices out."""
    m, n = A.shape
    lda = (m + 3) // 4 * 4
    T = torch.zeros((n, lda), dtype=torch.float32, device=device)
    T[:, :m] = torch.from_numpy(np.ascontiguousarray(np.asarray(A, dtype=np.float32).T)).to(device)
    return T[:, :m].t()


def test_c4_stratified_sample():
    """Instances of the C4 uneven batch (2048 BVLS problems, m log-uniform in
    [64, 2048], n/m log-uniform in [2, 8], Gaussian unit columns in FP32,
    bounds [0, 1], 30% of x* saturated, y = A x*), 24 of them spread evenly
    over the sizes m*n of the whole batch (smallest and largest included),
    solved together in one call to gap 1e-6 with each instance's own step
    from the library's Lanczos estimate, in the benchmark's layout (16-byte
    aligned columns).  Each must follow the oracle run with that step."""
    import paper_2202_07258_amd as bx
    ms, ns = W.c4_sizes(0, 2048)
    order = np.argsort(ms * ns, kind="stable")
    pick = order[np.linspace(0, len(order) - 1, 24).round().astype(int)]
    probs = [W.c4_instance(0, int(i), int(ms[i]), int(ns[i])) for i in pick]
    dev = [{"A": _padded_colmajor(P.A), "y": torch.tensor(P.y, device="cuda"),
            "l": torch.tensor(P.l, device="cuda"), "u": torch.tensor(P.u, device="cuda")} for P in probs]
    kw = dict(screen_every=10, eps_gap=1e-6, max_iter=20000)
    print(f"\n[c4 sample] {len(probs)} instances, m {ms[pick].min()}..{ms[pick].max()}", flush=True)
    xs, sats, infos, status = bx.solve_bvls_varbatch(dev, **kw)
    torch.cuda.synchronize()
    assert status == "ok"
    for P, x, s, info in zip(probs, xs, sats, infos):
        assert info["step"] > 0
        parity_vs_oracle(P, x.cpu().numpy(), s.cpu().numpy(), info, step=info["step"], **kw)


@pytest.mark.parametrize("m,n", [(9000, 1200), (16384, 800)])
def test_large_row_classes(m, n):
    """The two largest row classes (up to 8192 and 16384 rows, the maximum an
    instance may have), FP32 storage.  The tolerance stays well above the
    oracle's rounding floor: its gap has no rounding margins, so once the
    iteration reaches that floor its sphere becomes smaller than the rounding
    error of a_j^T theta and its rule is no longer safe (the certified GPU gap
    carries margins of about 1e-11 at these sizes)."""
    print(f"\n[large m] m={m} n={n}", flush=True)
    P = planted(20, m, n, nf_frac=0.02, dtype=np.float32)
    eta = step_of(P)
    kw = dict(screen_every=10, eps_gap=1e-9, max_iter=400, step=eta)
    xg, sg, info, res = check_parity(P, "bvls", **kw)
    free = (P.x_true > P.l) & (P.x_true < P.u)
    assert np.count_nonzero(sg) > 0 and not np.any(sg[free])


def test_largest_class_nnls_two_pass():
    """NNLS with the dual translation on the largest row class, whose sweeps
    run as a dot pass and a product pass (step, screening sweep with the step
    taken ahead, fold): screening fires and the trajectory matches the oracle."""
    rng = W.rng_for(94, 0)
    m, n = 9000, 600
    # non-negative entries (t = -1 is interior), a strong diagonal block
    A = 0.002 * rng.random((m, n))
    A[:n, :] += np.diag(0.5 + rng.random(n))
    P = W.Problem(np.asfortranarray(A.astype(np.float32)), rng.standard_normal(m), np.zeros(n), np.full(n, np.inf))
    print(f"\n[two-pass nnls] m={m} n={n}", flush=True)
    kw = dict(screen_every=10, eps_gap=1e-8, max_iter=5000, step=step_of(P))
    xg, sg, info, res = check_parity(P, "nnls", **kw)
    assert res.status == "ok" and info["n_lower"] > n // 2


@pytest.mark.parametrize("scale", [0.015625, 4.0])
def test_work_item_spread_extremes(scale):
    """The tuning knob that sets how many work items (and partial products) an
    instance is split into does not change the result: parity at the
    smallest and largest spread (one long item, and the 4-column minimum)."""
    from paper_2202_07258_amd import native as N
    P = planted(21, 700, 2600, dtype=np.float32)
    cls = N.row_class(P.m)
    before = N.group_scale(cls)
    try:
        N.set_group_scale(cls, scale)
        eta = step_of(P)
        check_parity(P, "bvls", screen_every=10, eps_gap=1e-8, max_iter=3000, step=eta)
    finally:
        N.set_group_scale(cls, before)
