"""GPU parity for the Huber fidelity (Sec. 3.3: eq. GAP_Safe_sph with
alpha = 1 for a fidelity whose gradient is 1-Lipschitz; Sec. 4.1's dual
update -grad F = clip(y' - Ax, -delta, delta)).

The library's PG path (single problems, FP64 and FP32 storage of A, the
two-pass row class, the uneven batch) against the oracle's Huber solve on the
same inputs and schedule: same iterations, passes and screened sets, x within
1e-9, matching certified gap and primal value.  The instances are tall, with
10% of the rows shifted by 2-5 so that the optimum has residuals beyond delta,
and with x0 spread over [-3, 3] so that many coordinates end on a bound.
"""
import math

import numpy as np
import pytest
import torch

from oracle import boxls as ob
from synth import workloads as W
from tests.gpu_helpers import check_parity, parity_vs_oracle

pytestmark = pytest.mark.gpu

DELTA = 0.5


def huber_instance(seed, m, n, dtype=np.float64, frac_out=0.1):
    rng = W.rng_for(71, seed, m, n)
    A = np.asfortranarray(W.unit_columns(rng.standard_normal((m, n))).astype(dtype))
    x0 = rng.uniform(-3.0, 3.0, n)
    y = A.astype(np.float64) @ x0 + 0.05 * rng.standard_normal(m)
    k = int(frac_out * m)
    idx = rng.choice(m, k, replace=False)
    y[idx] += rng.choice([-1.0, 1.0], k) * rng.uniform(2.0, 5.0, k)
    return W.Problem(A, y, -np.ones(n), np.ones(n), None, True, {})


def _kw(P, **extra):
    eta = 1.0 / (1.05 * ob.lipschitz(P.A64()))
    kw = dict(fidelity="huber", huber_delta=DELTA, screen_every=10, eps_gap=1e-8, max_iter=20000, step=eta)
    kw.update(extra)
    return kw


@pytest.mark.parametrize("m,n,dtype", [(200, 97, np.float64), (500, 260, np.float32), (1200, 500, np.float64),
                                       (3001, 1307, np.float32), (3001, 1307, np.float64),
                                       (16384, 200, np.float64)])
def test_huber_pg_parity(m, n, dtype):
    print(f"\n[huber pg] m={m} n={n} {np.dtype(dtype).name}", flush=True)
    P = huber_instance(0, m, n, dtype)
    xg, sg, info, res = check_parity(P, "bvls", **_kw(P))
    assert res.status == "ok" and np.count_nonzero(res.sat) > 0
    r = P.y - P.A64() @ res.x
    assert np.any(np.abs(r) > 2 * DELTA)                         # the Huber regime is active
    assert info["primal"] == pytest.approx(res.primal, rel=1e-9)


@pytest.mark.parametrize("m,n,dtype", [(500, 260, np.float64), (1200, 500, np.float32)])
def test_huber_chambolle_pock_parity(m, n, dtype):
    """The primal-dual solver with the clipped dual step (the Huber F*'s
    prox): same trajectory as the oracle's."""
    print(f"\n[huber cp] m={m} n={n} {np.dtype(dtype).name}", flush=True)
    P = huber_instance(4, m, n, dtype)
    eta = 1.0 / (1.05 * math.sqrt(ob.lipschitz(P.A64())))
    kw = dict(solver="cp", fidelity="huber", huber_delta=DELTA, screen_every=10, eps_gap=1e-8, max_iter=20000,
              step=eta)
    xg, sg, info, res = check_parity(P, "bvls", **kw)
    assert res.status == "ok" and np.count_nonzero(res.sat) > 0


def test_huber_unbounded_columns_use_theta_zero():
    """Columns with u_j = +inf: no translation for this fidelity, theta = 0
    (t_valid = 0), nothing screened; the iterates still match."""
    print("\n[huber pg, u = +inf columns]", flush=True)
    P = huber_instance(1, 400, 150)
    u = P.u.copy()
    u[:7] = math.inf
    P = W.Problem(P.A, P.y, P.l, u, None, True, {})
    kw = _kw(P, max_iter=300)
    kw["eps_gap"] = 0.0
    xg, sg, info, res = check_parity(P, "bvls", **kw)
    assert not info["t_valid"] and not res.t_valid
    assert not np.any(sg) and not np.any(res.sat)


def test_huber_varbatch_parity():
    print("\n[huber varbatch]", flush=True)
    import paper_2202_07258_amd as bx
    from tests.gpu_helpers import to_dev
    shapes = [(200, 97), (700, 333), (1500, 600)]
    probs = [huber_instance(10 + i, m, n, np.float32) for i, (m, n) in enumerate(shapes)]
    eta = 1.0 / (1.05 * max(ob.lipschitz(P.A64()) for P in probs))
    dev = []
    for P in probs:
        A, y, l, u = to_dev(P)
        dev.append({"A": A, "y": y, "l": l, "u": u})
    kw = dict(fidelity="huber", huber_delta=DELTA, screen_every=10, eps_gap=1e-8, max_iter=20000, step=eta)
    xs, sats, infos, status = bx.solve_bvls_varbatch(dev, **kw)
    torch.cuda.synchronize()
    assert status == "ok"
    for P, x, s, info in zip(probs, xs, sats, infos):
        res = parity_vs_oracle(P, x.cpu().numpy(), s.cpu().numpy(), info, **kw)
        assert np.count_nonzero(res.sat) > 0


def test_least_squares_unchanged_by_huber_option_fields():
    """huber_delta is ignored by the LS fidelity: identical results."""
    import paper_2202_07258_amd as bx
    from tests.gpu_helpers import run_gpu
    P = huber_instance(2, 300, 120)
    kw = dict(screen_every=10, eps_gap=1e-9, max_iter=3000, step=1.0 / (1.05 * ob.lipschitz(P.A64())))
    xa, sa, ia = run_gpu(P, "bvls", **kw)
    xb, sb, ib = run_gpu(P, "bvls", huber_delta=0.25, **kw)
    np.testing.assert_array_equal(xa, xb)
    assert ia["gap"] == ib["gap"] and ia["iters"] == ib["iters"]
