"""bfloat16 storage of A (BXS_BF16): every element is promoted exactly to FP64,
so the solver must follow the oracle run on the bf16-rounded matrix (as
FP64) exactly as it does for FP32 storage: same passes, iterates, gaps and
screened sets.  Instances are planted on the rounded matrix, so their
optimum is exact for the stored problem."""
import numpy as np
import pytest
import torch

from oracle import boxls as ob
from synth import workloads as W
from tests.gpu_helpers import assert_parity

pytestmark = pytest.mark.gpu


def _bf16_instance(seed, m, n, nf):
    import paper_2202_07258_amd as bx
    rng = W.rng_for(93, seed, m, n)
    A32 = W.unit_columns(rng.standard_normal((m, n))).astype(np.float32)
    At = torch.tensor(A32).to(torch.bfloat16)
    A64 = At.double().numpy()                      # the stored problem, exactly
    l, u = -rng.random(n), rng.random(n)
    y, x_star, theta, F = W.planted_bvls(A64, l, u, nf, 0.05, rng)
    dA = bx.colmajor(At, device="cuda")
    return dA, np.asfortranarray(A64), y, l, u, x_star


@pytest.mark.parametrize("m,n,solver", [(300, 1000, "pg"), (1500, 3333, "pg"), (9000, 1200, "pg"),
                                        (200, 450, "cd"), (700, 1800, "cp")])
def test_bf16_storage_trajectory_parity(m, n, solver):
    import paper_2202_07258_amd as bx
    print(f"\n[bf16 {solver}] m={m} n={n}", flush=True)
    nf = int(0.4 * min(m, n)) if m < n else int(0.02 * m)
    dA, A64, y, l, u, x_star = _bf16_instance(0, m, n, nf)
    assert dA.dtype == torch.bfloat16
    kw = dict(solver=solver, screen_every=1 if solver == "cd" else 10, eps_gap=1e-8, max_iter=6000)
    if solver == "pg":
        kw["step"] = 1.0 / (1.05 * ob.lipschitz(A64))
    elif solver == "cp":
        kw["step"] = 1.0 / (1.05 * np.sqrt(ob.lipschitz(A64)))
    dv = [torch.tensor(v, dtype=torch.float64, device="cuda") for v in (y, l, u)]
    x, sat, info = bx.solve_bvls(dA, *dv, **kw)
    torch.cuda.synchronize()
    res = ob.solve(A64, y, l, u, solver=solver, K=kw["screen_every"], eps_gap=1e-8, max_iter=6000,
                   step=kw.get("step"))
    P = W.Problem(A64, y, l, u)
    assert_parity(P, x.cpu().numpy(), sat.cpu().numpy(), info, res, xtol=1e-8)
    lo, hi = res.sat == -1, res.sat == 1
    assert np.all(x_star[lo] == l[lo]) and np.all(x_star[hi] == u[hi])
