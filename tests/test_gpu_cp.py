"""GPU parity of the Chambolle-Pock primal-dual solver (Sec. 5, the paper's
second BVLS solver) against the oracle's twin: the same tau = sigma, the same
screening schedule, the same passes, iterates and screened sets, for FP64 and
FP32 storage, BVLS and NNLS, screened and unscreened, the two-pass row class
and replay from a captured graph."""
import numpy as np
import pytest

from oracle import boxls as ob
from synth import workloads as W
from tests.gpu_helpers import check_parity, run_gpu, parity_vs_oracle
from tests.test_gpu_parity import planted

pytestmark = pytest.mark.gpu


def cp_step_of(P):
    return 1.0 / (1.05 * np.sqrt(ob.lipschitz(P.A64())))


@pytest.mark.parametrize("m,n", [(60, 173), (300, 1000), (1500, 3333)])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_cp_bvls_trajectory_parity(m, n, dtype):
    print(f"\n[cp bvls] m={m} n={n} {np.dtype(dtype).name}", flush=True)
    P = planted(41, m, n, dtype=dtype)
    kw = dict(solver="cp", screen_every=10, eps_gap=1e-8, max_iter=6000, step=cp_step_of(P))
    xg, sg, info, res = check_parity(P, "bvls", **kw)
    assert res.status == "ok" and np.count_nonzero(res.sat) > 0


def test_cp_unscreened_and_nnls():
    P = planted(42, 200, 600)
    kw = dict(solver="cp", screen_every=10, eps_gap=1e-9, max_iter=8000, step=cp_step_of(P), screening=False)
    xg, sg, info, res = check_parity(P, "bvls", **kw)
    assert not np.any(sg)
    Q = W.c1_companion(5, 150, 400)
    kw = dict(solver="cp", screen_every=10, eps_gap=1e-7, max_iter=5000, step=cp_step_of(Q))
    xg, sg, info, res = check_parity(Q, "nnls", **kw)
    assert info["t_valid"] == 1


def test_cp_two_pass_row_class():
    print("\n[cp two-pass] m=9000 n=1200", flush=True)
    P = planted(43, 9000, 1200, nf_frac=0.02, dtype=np.float32)
    kw = dict(solver="cp", screen_every=10, eps_gap=1e-7, max_iter=3000, step=cp_step_of(P))
    check_parity(P, "bvls", xtol=1e-8, **kw)


def test_cp_default_step_and_graph_replay():
    P = planted(44, 300, 900, dtype=np.float32)
    kw = dict(solver="cp", screen_every=5, eps_gap=1e-9, max_iter=6000, history=2000)
    xd, sd, idd = run_gpu(P, "bvls", **kw)
    # the library's step: tau = sigma = 1 / (1.05 sqrt(L_est)), L_est <= ||A||^2
    L = ob.lipschitz(P.A64())
    assert idd["step"] >= 1.0 / (1.05 * np.sqrt(L)) * (1 - 1e-12)
    assert idd["step"] ** 2 * L < 1.0
    xg, sg, ig = run_gpu(P, "bvls", graph=True, **kw)
    assert np.array_equal(xd, xg) and np.array_equal(sd, sg) and idd["iters"] == ig["iters"]
    parity_vs_oracle(P, xd, sd, idd, solver="cp", screen_every=5, eps_gap=1e-9, max_iter=6000, step=idd["step"])
