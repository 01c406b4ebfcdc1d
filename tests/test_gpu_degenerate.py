"""GPU parity on the degenerate inputs the method admits, for the three
solvers: zero columns (a_j = 0: no gradient, never screened, skipped by CD),
fixed coordinates (l_j = u_j), duplicated columns (a non-unique optimum; the
iterates are still determined), a start outside the box (clipped first) and
y = 0 (the projection of 0 is optimal, the first gap is 0).  Each run is
compared with the oracle on the same schedule: same passes, iterates and
screened sets."""
import numpy as np
import pytest

from oracle import boxls as ob
from synth import workloads as W
from tests.gpu_helpers import check_parity

pytestmark = pytest.mark.gpu


def _base(seed, m=120, n=300):
    rng = W.rng_for(99, seed, m, n)
    A = W.unit_columns(rng.standard_normal((m, n)))
    l, u = -rng.random(n), rng.random(n)
    y = A @ np.clip(rng.standard_normal(n), l, u) + 0.05 * rng.standard_normal(m)
    return rng, A, y, l, u


def _kw(P, solver):
    L = ob.lipschitz(P.A64())
    step = 1.0 / (1.05 * L) if solver == "pg" else (1.0 / (1.05 * np.sqrt(L)) if solver == "cp" else 0.0)
    kw = dict(solver=solver, screen_every=1 if solver == "cd" else 10, eps_gap=1e-9, max_iter=20000)
    if solver != "cd":
        kw["step"] = step
    return kw


@pytest.mark.parametrize("solver", ["pg", "cd", "cp"])
def test_zero_fixed_and_duplicate_columns(solver):
    # a planted instance (so that screening fires), then the degenerate edits
    rng = W.rng_for(99, 0, 120, 300)
    A = W.unit_columns(rng.standard_normal((120, 300)))
    l, u = -rng.random(300), rng.random(300)
    y, _, _, _ = W.planted_bvls(A, l, u, 48, 0.05, rng)
    A[:, 5] = 0.0                       # zero columns
    A[:, 77] = 0.0
    A[:, 40] = A[:, 41]                 # a duplicated column
    l[[10, 11, 12]] = u[[10, 11, 12]]   # fixed coordinates
    l[13] = u[13] = 0.0
    P = W.Problem(np.asfortranarray(A), y, l, u)
    xg, sg, info, res = check_parity(P, "bvls", **_kw(P, solver))
    assert res.status == "ok" and np.count_nonzero(sg) > 100
    assert sg[5] == 0 and sg[77] == 0   # a zero column is never screened
    for j in (10, 11, 12, 13):
        assert xg[j] == l[j]


@pytest.mark.parametrize("solver", ["pg", "cd", "cp"])
def test_start_outside_the_box_and_zero_data(solver):
    rng, A, y, l, u = _base(1)
    P = W.Problem(np.asfortranarray(A), y, l, u)
    x0 = 3.0 * rng.standard_normal(A.shape[1])          # mostly outside [l, u]
    check_parity(P, "bvls", x0=x0, **_kw(P, solver))
    Z = W.Problem(np.asfortranarray(A), np.zeros(A.shape[0]), l, u)
    xg, sg, info, res = check_parity(Z, "bvls", **_kw(Z, solver))
    assert res.status == "ok" and info["passes"] == 1 and np.all(xg == 0.0)
