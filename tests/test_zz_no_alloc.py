"""The allocation-free entry point solve_bvls_noalloc (for callers that cannot
allocate) against solve_bvls: the same kernels on the library's fixed device
scratch array must give the same solution, screened set and iteration count,
on two calls in a row (the second smaller, so it runs on the array the first
left dirty), and a problem larger than the array must be refused before any
launch."""
import ctypes as C

import numpy as np
import pytest
import torch

from synth import workloads as W

pytestmark = pytest.mark.gpu


def _instance(seed, m, n, dtype):
    rng = W.rng_for(4242, seed)
    A = W.unit_columns(rng.standard_normal((m, n)))
    if dtype == np.float32:
        A = A.astype(np.float32)
    l, u = -rng.random(n), rng.random(n)
    y, _, _, _ = W.planted_bvls(A.astype(np.float64), l, u, max(1, m // 3), 0.05, rng)
    return A, y, l, u


def _solve_both(A, y, l, u, **kw):
    import paper_2202_07258_amd as bx
    dA = bx.colmajor(A, device="cuda")
    dv = [torch.tensor(v, dtype=torch.float64, device="cuda") for v in (y, l, u)]
    x1, s1, i1 = bx.solve_bvls(dA, *dv, **kw)
    x2, s2, i2 = bx.solve_bvls_noalloc(dA, *dv, **kw)
    torch.cuda.synchronize()
    return (x1.cpu().numpy(), s1.cpu().numpy(), i1), (x2.cpu().numpy(), s2.cpu().numpy(), i2)


def _check(ref, got, tol):
    (x1, s1, i1), (x2, s2, i2) = ref, got
    assert i2["status_name"] == i1["status_name"] == "ok", (i1["status_name"], i2["status_name"])
    assert i2["iters"] == i1["iters"] and i2["passes"] == i1["passes"]
    assert np.array_equal(s1, s2)
    assert np.max(np.abs(x1 - x2)) <= tol * max(1.0, float(np.max(np.abs(x1))))
    assert abs(i2["gap"] - i1["gap"]) <= 1e-12 * max(1.0, i1["gap"])


def test_noalloc_matches_solve_bvls_two_calls():
    # first call: FP32 storage, several work items and a ragged row tail
    A, y, l, u = _instance(0, 700, 2500, np.float32)
    print("noalloc call 1: 700x2500 fp32", flush=True)
    ref, got = _solve_both(A, y, l, u, screen_every=10, eps_gap=1e-8, max_iter=50000, history=64)
    _check(ref, got, 1e-4)
    assert np.count_nonzero(got[1]) > 0
    assert got[2]["history"] == ref[2]["history"]
    # second call, smaller, FP64 storage, on the scratch the first call left behind
    A, y, l, u = _instance(1, 130, 390, np.float64)
    print("noalloc call 2: 130x390 fp64", flush=True)
    ref, got = _solve_both(A, y, l, u, screen_every=10, eps_gap=1e-9, max_iter=50000)
    _check(ref, got, 1e-6)


def test_noalloc_huber_matches_solve_bvls():
    # the Huber fidelity through the fixed scratch: same kernels, same result
    P = W.huber_bvls(3, 600, 250)
    print("noalloc huber: 600x250 fp64", flush=True)
    ref, got = _solve_both(P.A, P.y, P.l, P.u, fidelity="huber", huber_delta=0.5, screen_every=10, eps_gap=1e-8,
                           max_iter=50000)
    _check(ref, got, 1e-9)
    assert np.count_nonzero(got[1]) > 0


def test_noalloc_refuses_a_problem_larger_than_its_scratch():
    import paper_2202_07258_amd as bx
    from paper_2202_07258_amd import native as N
    m, n = 16000, 4000
    opts, _ = N.make_opts()
    need = N.workspace_bytes(m, n, opts)
    assert need > N.NOALLOC_SCRATCH_BYTES
    torch.manual_seed(9)
    A = torch.randn(n, m, dtype=torch.float32, device="cuda").t()   # column-major m x n
    y = torch.zeros(m, dtype=torch.float64, device="cuda")
    l = -torch.ones(n, dtype=torch.float64, device="cuda")
    u = torch.ones(n, dtype=torch.float64, device="cuda")
    print(f"noalloc oversize: {m}x{n} needs {need} bytes", flush=True)
    with pytest.raises(N.BoxscreenError) as ei:
        bx.solve_bvls_noalloc(A, y, l, u, max_iter=10)
    assert ei.value.status == N.BXS_ERR_NOMEM
    assert "fixed scratch" in str(ei.value)


def test_noalloc_rejects_workspace_graph_and_profile():
    import paper_2202_07258_amd as bx
    from paper_2202_07258_amd import native as N
    lib = N.load()
    A, y, l, u = _instance(2, 64, 128, np.float64)
    dA = bx.colmajor(A, device="cuda")
    dy, dl, du = (torch.tensor(v, dtype=torch.float64, device="cuda") for v in (y, l, u))
    x = torch.zeros(128, dtype=torch.float64, device="cuda")
    sat = torch.empty(128, dtype=torch.int8, device="cuda")
    for field in ("workspace", "graph", "profile"):
        o, _ = N.make_opts()
        setattr(o, field, 1 << 20 if field == "workspace" else 1)
        if field == "workspace":
            o.workspace_bytes = 1 << 20
        info = N.Info()
        st = lib.solve_bvls_noalloc(64, 128, N.BXS_F64, dA.data_ptr(), 64, dy.data_ptr(), dl.data_ptr(),
                                    du.data_ptr(), x.data_ptr(), sat.data_ptr(), C.byref(o), C.byref(info))
        assert st == N.BXS_ERR_ARG, field
        assert field in lib.bxs_last_error().decode()
