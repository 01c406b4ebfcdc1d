"""Benchmark workloads beyond the headline one (bench.py --workload ...).

c1      NNLS 200x500, N(0,1) unit columns, FP64, PG K=10, gap 1e-9: one
        instance (latency-bound), and 1024 seeded instances in one batch call
c3      batched NNLS, shared A 1024x4096 (U[0,1] unit columns, FP32), 8192
        right-hand sides: BF16x3 MFMA engine vs FP64 GEMM engine, same iteration
        budget (their trajectories agree), time per iteration and GEMM rate
c4      2048 independent BVLS instances of uneven shape (m log-uniform in
        [64, 2048], n/m log-uniform in [2, 8]), FP32, one batch call
c5      differentiable NNLS layer: A 512x1024 N(0,1) FP32, Y 512x512 U[0,1],
        forward solve + implicit adjoint of sum_b ||x_b - t_b||^2
table2  the paper's Table 2 BVLS setup (m=1000, n=3000, |N(0,1)| entries,
        bounds [0,1], noise N(0,1)): screened vs unscreened PG

Every input is seeded and synthetic (synth.workloads).  Only the
`cpu_baseline` parts call the FP64 oracle.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np
import torch

import paper_2202_07258_amd as bx
from paper_2202_07258_amd import native as N
from synth import workloads as W

HBM_PEAK = 8000.0
BF16_PEAK_TFLOPS = 2500.0
FP64_PEAK_TFLOPS = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _cores():
    try:
        from threadpoolctl import threadpool_info
        return max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        return os.cpu_count() or 1


def _upload(P, device):
    A = bx.colmajor(P.A, device=device)
    y, l, u = (torch.tensor(v, dtype=torch.float64, device=device) for v in (P.y, P.l, P.u))
    return A, y, l, u


def _sync():
    torch.cuda.synchronize()


# --------------------------------------------------------------------------
def bench_c1(args, device):
    P = W.c1_nnls(0)
    A, y, l, u = _upload(P, device)
    kw = dict(screen_every=10, eps_gap=1e-9, max_iter=100000)
    bx.solve_nnls(A, y, **kw)
    _sync()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        x, sat, info = bx.solve_nnls(A, y, **kw)
    _sync()
    dt = (time.perf_counter() - t0) / args.steps
    # the same solve with each regular pass replayed from a captured HIP graph
    t0 = time.perf_counter()
    for _ in range(args.steps):
        bx.solve_nnls(A, y, graph=True, **kw)
    _sync()
    dt_graph = (time.perf_counter() - t0) / args.steps
    # coordinate descent (one sweep per iteration, screening every 10 sweeps)
    bx.solve_nnls(A, y, solver="cd", **kw)
    _sync()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, _, info_cd = bx.solve_nnls(A, y, solver="cd", **kw)
    _sync()
    dt_cd = (time.perf_counter() - t0) / args.steps
    # the non-negative companion (t = -1 interior: screening fires)
    Pc = W.c1_companion(0)
    Ac, yc, _, _ = _upload(Pc, device)
    comp = {}
    for solver in ["pg", "cd"]:
        for screening in [True, False]:
            bx.solve_nnls(Ac, yc, solver=solver, screening=screening, **kw)
            _sync()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                _, _, ic = bx.solve_nnls(Ac, yc, solver=solver, screening=screening, **kw)
            _sync()
            comp[f"{solver}_{'screened' if screening else 'unscreened'}"] = {
                "ms_per_solve": round(1e3 * (time.perf_counter() - t0) / args.steps, 3), "iters": ic["iters"],
                "n_screened": ic["n_lower"], "status": ic["status_name"], "gap": ic["gap"]}
    # many instances of the same law in one batch call (C1 x N: 4096 seeds,
    # 3.3 GB of A, HBM-bound where the single instance is latency-bound)
    count = 4096
    probs = []
    for i in range(count):
        Q = W.c1_nnls(1000 + i)
        Ad, yd, _, _ = _upload(Q, device)
        probs.append({"A": Ad, "y": yd, "l": None, "u": None})
    bx.solve_bvls_varbatch(probs, **kw)
    _sync()
    t0 = time.perf_counter()
    xs, sats, infos, status = bx.solve_bvls_varbatch(probs, **kw)
    _sync()
    dtb = time.perf_counter() - t0
    out = {"workload": "C1: NNLS 200x500 N(0,1) unit columns FP64, PG K=10, gap 1e-9",
           "single": {"solves_per_s": round(1 / dt, 2), "ms_per_solve": round(1e3 * dt, 3), "iters": info["iters"],
                      "t_valid": info["t_valid"], "n_screened": info["n_lower"], "status": info["status_name"],
                      "ms_per_solve_graph_replay": round(1e3 * dt_graph, 3)},
           "single_cd": {"solves_per_s": round(1 / dt_cd, 2), "ms_per_solve": round(1e3 * dt_cd, 3),
                         "sweeps": info_cd["iters"], "status": info_cd["status_name"]},
           "companion_nonneg_A": comp,
           "batch": {"instances": count, "solves_per_s": round(count / dtb, 1), "seconds": round(dtb, 3),
                     "status": status, "max_iters": max(i["iters"] for i in infos),
                     # algorithmic bytes of the primal sweeps: every preserved column of
                     # every iteration once in FP64 (plus x/l/u/index) and the residual
                     "roofline": _batch_roofline(infos, P.m, 8, dtb)}}
    if not args.no_cpu_baseline:
        from oracle import boxls as ob
        A64 = P.A64()
        t0 = time.perf_counter()
        res = ob.solve(A64, P.y, P.l, P.u, K=10, eps_gap=1e-9, step=1.0 / (1.05 * ob.lipschitz(A64)))
        dtc = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(1 / dtc, 3), "unit": "solves/s", "cores": _cores(), "kind": "oracle",
                               "sample": f"one full oracle solve ({res.iters} iterations)"}
    return out


def _batch_roofline(infos, m, elem_bytes, seconds):
    """Whole-call HBM rate of a batch: the primal sweeps' algorithmic bytes
    (sum over instances of col_iters x (m s_A + 36) + iters x 8 m) over the
    call's wall time, against 8 TB/s."""
    byts = sum(i["col_iters"] * (m * elem_bytes + 36) + i["iters"] * 8 * m for i in infos)
    ach = byts / seconds / 1e9
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK, 4), "traffic": None, "algorithmic_bytes": int(byts),
            "note": "whole call (setup, screening passes and launch gaps included)"}


# --------------------------------------------------------------------------
def bench_c3(args, device):
    B = args.c3_rhs
    log(f"[c3] generating A 1024x4096, {B} right-hand sides")
    A, Y, Xt = W.c3_shared(0, B=B)
    dA = bx.colmajor(A, device=device)
    dY = torch.tensor(Y.T.copy(), dtype=torch.float64, device=device).t()
    iters = args.c3_iters
    out = {"workload": f"C3: batched NNLS, shared A 1024x4096 U[0,1] unit columns FP32, {B} RHS, "
                       f"t = -1, PG K=10, fixed budget of {iters} iterations",
           "note": "PG on this matrix (L ~ 3.1e3, nearly parallel columns) cannot reach gap 1e-6 in any "
                   "practical budget; both engines run the same budget and follow the same trajectory"}
    res = {}
    keep = {}
    for prec in ["bf16x3", "f64"]:
        kw = dict(iter_precision=prec, screen_every=10, eps_gap=1e-6, max_iter=iters)
        bx.solve_nnls_batched_shared(dA, dY, **dict(kw, max_iter=10))
        _sync()
        # the timed solve runs as a user runs it (passes enqueued ahead, no
        # events); a profiled repeat times the GEMM pairs
        t0 = time.perf_counter()
        X, S, infos = bx.solve_nnls_batched_shared(dA, dY, **kw)
        _sync()
        dt = time.perf_counter() - t0
        _, _, pinfos = bx.solve_nnls_batched_shared(dA, dY, profile=True, **kw)
        _sync()
        gaps = np.array([i["gap"] for i in infos])
        pairs = pinfos[0]["sweep_launches"]
        gemm_s = pinfos[0]["sweep_ms"] * 1e-3
        useful = 4.0 * 1024 * 4096 * B                     # two m x n x B products per iteration
        r = {"seconds": round(dt, 3), "ms_per_iter": round(1e3 * dt / iters, 3),
             "rhs_iters_per_s": round(B * iters / dt, 1),
             "gap_median": float(np.median(gaps)), "gap_max": float(gaps.max()),
             "screened_total": int(sum(i["n_lower"] for i in infos)),
             "gemm_pair_us": round(1e6 * gemm_s / max(pairs, 1), 1),
             "useful_tflops": round(useful / (gemm_s / max(pairs, 1)) / 1e12, 1)}
        if prec == "bf16x3":
            r["mfma_tflops_executed"] = round(3 * r["useful_tflops"], 1)
            r["roofline"] = {"bound": "mfma", "achieved": r["mfma_tflops_executed"], "peak": BF16_PEAK_TFLOPS,
                             "unit": "TFLOP/s", "frac": round(r["mfma_tflops_executed"] / BF16_PEAK_TFLOPS, 4),
                             "traffic": None,
                             "kernel": "k_gemm_bf16x3<0>/<1> (A D and G -= A^T U, three bf16 MFMAs per product)"}
        else:
            r["roofline"] = {"bound": "mfma", "achieved": r["useful_tflops"], "peak": FP64_PEAK_TFLOPS,
                             "unit": "TFLOP/s", "frac": round(r["useful_tflops"] / FP64_PEAK_TFLOPS, 4),
                             "traffic": None, "kernel": "k_dgemm<0,0>/<1,0> (R = Y - A X and G = A^T R, FP64 MFMA 16x16x4)"}
        res[prec] = r
        keep[prec] = X
        keep[prec + "_gaps"] = gaps
        del S
        torch.cuda.empty_cache()
    res["bf16x3_speedup_vs_f64"] = round(res["f64"]["seconds"] / res["bf16x3"]["seconds"], 3)
    res["bf16x3_max_abs_diff_vs_f64_engine"] = float((keep["bf16x3"] - keep["f64"]).abs().max())
    out.update(res)
    if not args.no_cpu_baseline:
        from oracle import boxls as ob
        A64 = A.astype(np.float64)
        nb = 4
        t0 = time.perf_counter()
        eta = 1.0 / (1.05 * ob.lipschitz_power(A64, 20))
        for b in range(nb):
            ob.solve(A64, Y[:, b], np.zeros(4096), np.full(4096, np.inf), K=10, eps_gap=1e-6, max_iter=iters, step=eta)
        dtc = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(nb * iters / dtc, 1), "unit": "rhs_iters/s", "cores": _cores(),
                               "kind": "oracle", "sample": f"{nb} right-hand sides x {iters} iterations"}
        # the oracle's own FP64 gap (eq. Dual_Gap, t = -1) at sampled BF16x3 solutions
        Xb = keep["bf16x3"].cpu().numpy()
        sample = np.random.default_rng(5).choice(B, size=4, replace=False)
        gaps = []
        for b in sample:
            x = Xb[:, b]
            theta, _, _ = ob.dual_point(A64, Y[:, b], np.full(4096, np.inf), x, -np.ones(1024))
            gaps.append(ob.duality_gap(A64, Y[:, b], np.zeros(4096), np.full(4096, np.inf), x, theta))
        # the GPU's certified gap is an upper bound on the exact one at its own x
        out["bf16x3_gap_check_sampled"] = {"rhs": [int(b) for b in sample], "oracle_fp64_gap": gaps,
                                           "gpu_certified_gap": [float(keep["bf16x3_gaps"][b]) for b in sample]}
    return out


# --------------------------------------------------------------------------
def _c4_worker_init():
    # one BLAS thread per generator process (the pool already fills the cores)
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(limits=1)
    except ImportError:
        pass


def _c4_problem(args_):
    i, m, n, planted = args_
    P = (W.c4_planted_instance if planted else W.c4_instance)(0, i, int(m), int(n))
    return i, P.A, P.y


def bench_c4(args, device):
    count = args.c4_count
    planted = bool(getattr(args, "c4_planted", False))
    ms, ns = W.c4_sizes(0, count)
    log(f"[c4] generating {count} {'planted ' if planted else ''}instances, "
        f"{float(np.sum(ms * ns)) * 4 / 1e9:.1f} GB of FP32 A")
    from multiprocessing import Pool
    probs = [None] * count
    t0 = time.perf_counter()
    done = 0
    with Pool(min(16, os.cpu_count() or 1), initializer=_c4_worker_init) as pool:
        for i, A, y in pool.imap_unordered(_c4_problem, [(i, ms[i], ns[i], planted) for i in range(count)],
                                           chunksize=4):
            done += 1
            if done % 256 == 0:
                log(f"[c4] {done} of {count} instances generated ({time.perf_counter() - t0:.1f}s)")
            m, n = A.shape
            lda = (m + 3) // 4 * 4                     # 16-byte aligned columns
            T = torch.zeros((n, lda), dtype=torch.float32, device=device)
            T[:, :m] = torch.from_numpy(np.ascontiguousarray(A.T)).to(device)
            probs[i] = {"A": T[:, :m].t(), "y": torch.tensor(y, dtype=torch.float64, device=device),
                        "l": torch.zeros(n, dtype=torch.float64, device=device),
                        "u": torch.ones(n, dtype=torch.float64, device=device)}
    log(f"[c4] generated in {time.perf_counter() - t0:.1f}s")
    classes = sorted({N.row_class(int(m)) for m in ms})
    log(f"[c4] autotuning the sweep shapes of row classes {classes}")
    tuned = bx.autotune.tuned(device=device, classes=classes, batch=True, iters=30, reps=1)
    log(f"[c4] tuning table {tuned['key']}: reused {tuned['cached']}, tuned {tuned['tuned']} "
        f"({tuned['seconds']} s)")
    kw = dict(screen_every=10, eps_gap=1e-6, max_iter=20000)
    _sync()
    # the timed solve as a user runs it (no events); a profiled repeat gives
    # the sweep launch times for the roofline
    log("[c4] timed solve")
    t0 = time.perf_counter()
    xs, sats, infos, status = bx.solve_bvls_varbatch(probs, **kw)
    _sync()
    dt = time.perf_counter() - t0
    log(f"[c4] solved in {dt:.2f}s; profiled repeat")
    _, _, pinfos, _ = bx.solve_bvls_varbatch(probs, profile=True, **kw)
    _sync()
    col_bytes = sum(infos[i]["col_iters"] * (int(ms[i]) * 4 + 36) for i in range(count))
    launches = pinfos[0]["sweep_launches"]
    sweep_s = pinfos[0]["sweep_ms"] * 1e-3
    iters = [i["iters"] for i in infos]
    # the timed launch groups are all but the first iteration of each pass:
    # their share of the column bytes is taken as their share of the groups
    col_bytes *= launches / max(max(iters), 1)
    achieved = col_bytes / sweep_s / 1e9 if sweep_s > 0 else None
    out = {}
    if not args.no_cpu_baseline:
        # a stratified oracle sample: 64 instances spread evenly over the sizes
        # m*n of the batch, each solved by the oracle with the instance's own
        # step (the library's Lanczos estimate) and checked against the GPU
        from oracle import boxls as ob
        order = np.argsort(ms * ns, kind="stable")
        pick = order[np.linspace(0, count - 1, 64).round().astype(int)]
        t0 = time.perf_counter()
        same_iters, max_err, same_sat, done = 0, 0.0, 0, 0
        # smallest first, within a CPU-time budget (the largest planted
        # instances take minutes on the host)
        for i in pick:
            if time.perf_counter() - t0 > args.c4_oracle_budget:
                break
            P = (W.c4_planted_instance if planted else W.c4_instance)(0, int(i), int(ms[i]), int(ns[i]))
            res = ob.solve(P.A64(), P.y, P.l, P.u, K=10, eps_gap=1e-6, max_iter=20000, step=infos[i]["step"])
            xg = xs[i].cpu().numpy()
            same_iters += int(res.iters == infos[i]["iters"])
            same_sat += int(np.array_equal(res.sat, sats[i].cpu().numpy()))
            max_err = max(max_err, float(np.max(np.abs(xg - res.x))) / max(1.0, float(np.max(np.abs(res.x)))))
            done += 1
            log(f"[c4] oracle instance {done}: {ms[i]}x{ns[i]}, {res.iters} iterations "
                f"(GPU {infos[i]['iters']}), {time.perf_counter() - t0:.1f}s")
        dtc = time.perf_counter() - t0
        out["oracle_sample"] = {"instances": done, "same_iteration_count": same_iters,
                                "same_screened_set": same_sat, "max_rel_err_x": max_err,
                                "largest": f"{ms[pick[done - 1]]}x{ns[pick[done - 1]]}" if done else None}
        out["cpu_baseline"] = {"value": round(done / dtc, 3), "unit": "solves/s", "cores": _cores(),
                               "kind": "oracle",
                               "sample": f"{done} of 64 instances spread evenly over the sizes of the batch "
                                         f"(smallest first, {args.c4_oracle_budget:.0f} s budget), one at a time",
                               "seconds": round(dtc, 2)}
    law = ("planted optimum, |F| = 0.4 m free, ||theta*|| ~ 0.01 sqrt(m) (C4-pl)" if planted else
           "30% saturated, y = A x*")
    return {**out,
            "workload": f"C4{'-pl' if planted else ''}: {count} BVLS instances, m log-uniform [64,2048], "
                        f"n/m log-uniform [2,8], Gaussian unit columns FP32, bounds [0,1], {law}",
            "solves_per_s": round(count / dt, 2), "seconds": round(dt, 3), "status": status,
            "iters_median": int(np.median(iters)), "iters_max": int(max(iters)),
            "n_screened_total": int(sum(i["n_lower"] + i["n_upper"] for i in infos)),
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1) if achieved else None, "peak": HBM_PEAK,
                         "unit": "GB/s", "frac": round(achieved / HBM_PEAK, 4) if achieved else None,
                         "traffic": None, "kernel": "k_sweep PG launches over all unfinished instances",
                         "launch_groups": launches},
            "autotune": {"seconds": tuned["seconds"], "key": tuned["key"], "reused_classes": tuned["cached"],
                         "best": {int(c): r["best"] for c, r in tuned["classes"].items()},
                         "previous": {int(c): r.get("previous") for c, r in tuned["classes"].items()},
                         "spread": {int(c): r["scale"] for c, r in tuned["classes"].items()}}}


# --------------------------------------------------------------------------
def bench_c5(args, device):
    rejected = []
    for rep in range(40):
        A, Y, T = W.c5_layer(rep)
        t = W.interior_direction(A)
        if t is not None:
            break
        rejected.append(rep)
    log(f"[c5] seed {rep} admits a translation direction (rejected {rejected})")
    At = torch.tensor(A, dtype=torch.float32, device=device, requires_grad=True)
    Yt = torch.tensor(Y, dtype=torch.float32, device=device, requires_grad=True)
    Tt = torch.tensor(T, dtype=torch.float32, device=device)
    tt = torch.tensor(t, dtype=torch.float64, device=device)
    iters = args.c5_iters
    res = {}
    for prec in ["f64", "bf16x3"]:
        kw = dict(eps_gap=1e-6, max_iter=iters, screen_every=10, iter_precision=prec, cg_max_iter=2000, cg_tol=1e-10)
        X = bx.nnls_layer(At, Yt, tt, on_inexact="ignore", **dict(kw, max_iter=20))   # warm-up (library load)
        ((X - Tt) ** 2).sum().backward()
        _sync()
        At.grad = None
        Yt.grad = None
        stats = {}
        t0 = time.perf_counter()
        X = bx.nnls_layer(At, Yt, tt, stats=stats, on_inexact="ignore", **kw)   # counts reported below
        _sync()
        t1 = time.perf_counter()
        loss = ((X - Tt) ** 2).sum()
        loss.backward()
        _sync()
        t2 = time.perf_counter()
        fw = stats["forward"]
        gaps = np.array([i["gap"] for i in fw])
        nfree = (X.detach() > 0).sum(0).cpu().numpy()
        res[prec] = {"forward_s": round(t1 - t0, 4), "backward_s": round(t2 - t1, 4),
                     "fwd_bwd_per_s": round(1 / (t2 - t0), 3), "loss": float(loss.detach()),
                     "converged": int(sum(i["status_name"] == "ok" for i in fw)), "batch": len(fw),
                     "gap_median": float(np.median(gaps)), "gap_max": float(gaps.max()),
                     "free_median": int(np.median(nfree)), "free_max": int(nfree.max()),
                     "free_gt_m": int((nfree > A.shape[0]).sum()),
                     "cg_iters": stats.get("cg_iters"), "cg_status": stats.get("cg_status"),
                     "grad_A_norm": float(At.grad.norm()), "grad_Y_norm": float(Yt.grad.norm()),
                     "grads_finite": bool(torch.isfinite(At.grad).all() and torch.isfinite(Yt.grad).all())}
        At.grad = None
        Yt.grad = None
        log(f"[c5] {prec}: {res[prec]}")
    return {"workload": f"C5: NNLS layer, A 512x1024 N(0,1) FP32 (seed {rep}; seeds {rejected} rejected: no "
                        f"translation direction), Y 512x512 U[0,1], loss sum ||x_b - t_b||^2; forward PG K=10 "
                        f"to gap 1e-6 or {iters} iterations (gap reached is reported), CG tol 1e-10",
            "note": "the free sets have ~500 of 512 rows and cond(A_F) ~ 150-250, so PG needs ~1e5+ iterations "
                    "for a certified 1e-6 gap; the gradient check against FP64 central differences runs in the "
                    "GPU tests on the 32x64 subproblem",
            **res}


# --------------------------------------------------------------------------
def _fig1_point(A, y, P, b, device, reps):
    n = P.n
    l = torch.full((n,), -b, dtype=torch.float64, device=device)
    u = torch.full((n,), b, dtype=torch.float64, device=device)
    out = {"b": b}
    for screening in (True, False):
        kw = dict(screening=screening, screen_every=10, eps_gap=1e-6, max_iter=200000)
        bx.solve_bvls(A, y, l, u, **dict(kw, max_iter=20))
        _sync()
        best = None
        for _ in range(reps):
            t0 = time.perf_counter()
            x, sat, info = bx.solve_bvls(A, y, l, u, **kw)
            _sync()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        xs = x.cpu().numpy()
        rec = {"seconds": round(best, 5), "iters": info["iters"], "status": info["status_name"],
               "gap": info["gap"], "n_screened": info["n_lower"] + info["n_upper"],
               "ms_setup": round(info["ms_setup"], 3),
               "mean_preserved_fraction": round(info["col_iters"] / max(info["iters"], 1) / n, 4),
               # wall time per primal iteration, setup (column norms, Lanczos) excluded
               "us_per_iter": round((1e6 * best - 1e3 * info["ms_setup"]) / max(info["iters"], 1), 2)}
        if screening:
            rec["saturation_ratio"] = round(float(np.mean(np.abs(np.abs(xs) - b) <= 1e-12 * b)), 4)
        out["screened" if screening else "unscreened"] = rec
    out["speedup"] = round(out["unscreened"]["seconds"] / out["screened"]["seconds"], 3)
    out["speedup_per_iter"] = round(out["unscreened"]["us_per_iter"] / out["screened"]["us_per_iter"], 3)
    return out


def bench_fig1(args, device):
    """Sec. 5.1, Fig. 1: speedup of screening against the saturation ratio,
    PG on BVLS with a_ij ~ N(0,1), y ~ N(0,1) and the box b [-1, 1]; at the
    paper's size (4000 x 2000, FP64) and at sizes where a sweep is
    HBM-bound: C2's shape (4000 x 16000 FP32, 256 MB) and 8000 x 16000 FP32
    (512 MB, twice the 256 MiB Infinity Cache)."""
    sizes = [(4000, 2000, np.float64, [0.0005, 0.001, 0.002, 0.005, 0.01, 0.05]),
             (4000, 16000, np.float32, [0.0005, 0.001, 0.002, 0.005, 0.01]),
             (8000, 16000, np.float32, [0.0005, 0.001, 0.002, 0.005, 0.01])]
    out = {"workload": "Fig. 1 law (Sec. 5.1): BVLS, a_ij ~ N(0,1), y ~ N(0,1), box b[-1,1]; PG K=10 to gap 1e-6; "
                       "wall time per solve (best of 3), per-iteration times exclude setup",
           "sizes": []}
    for (m, n, dt, bs) in sizes:
        P = W.fig1_bvls(0, m, n, 1.0, dtype=dt)
        A = bx.colmajor(P.A, device=device)
        y = torch.tensor(P.y, dtype=torch.float64, device=device)
        pts = []
        for b in bs:
            pt = _fig1_point(A, y, P, b, device, reps=3)
            log(f"[fig1] {m}x{n} {np.dtype(dt).name} b={b}: sat {pt['screened']['saturation_ratio']} "
                f"speedup {pt['speedup']} (per iter {pt['speedup_per_iter']}), "
                f"{pt['screened']['us_per_iter']} vs {pt['unscreened']['us_per_iter']} us/iter at preserved "
                f"{pt['screened']['mean_preserved_fraction']}")
            pts.append(pt)
        entry = {"m": m, "n": n, "a_storage": np.dtype(dt).name, "points": pts}
        # per-iteration time against the preserved fraction: t = a + c f (least squares over the points,
        # screened and unscreened runs alike)
        f = np.array([p["screened"]["mean_preserved_fraction"] for p in pts] + [1.0] * len(pts))
        t = np.array([p["screened"]["us_per_iter"] for p in pts] + [p["unscreened"]["us_per_iter"] for p in pts])
        c, a = np.polyfit(f, t, 1)
        entry["per_iter_fit_us"] = {"fixed": round(float(a), 2), "per_unit_preserved_fraction": round(float(c), 2)}
        if (m, n) == (8000, 16000):
            # sweep roofline above the Infinity Cache size, unscreened
            l = torch.full((n,), -0.01, dtype=torch.float64, device=device)
            _, _, info = bx.solve_bvls(A, y, l, -l, screening=False, screen_every=10, eps_gap=0.0,
                                       max_iter=200, profile=True)
            _sync()
            per_launch = n * (m * 4 + 36) + 8 * m
            avg_s = info["sweep_ms"] * 1e-3 / max(info["sweep_launches"], 1)
            ach = per_launch / avg_s / 1e9
            entry["sweep_roofline_unscreened"] = {
                "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK, 4), "algorithmic_bytes_per_launch": per_launch,
                "avg_launch_us": round(avg_s * 1e6, 2), "launches": info["sweep_launches"],
                "note": "A is 512 MB, twice the Infinity Cache: every sweep streams it from HBM"}
        out["sizes"].append(entry)
        del A
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        from oracle import boxls as ob
        P = W.fig1_bvls(0, 4000, 2000, 0.002)
        A64 = P.A64()
        eta = 1.0 / (1.05 * ob.lipschitz(A64))
        res = {}
        for screening in (True, False):
            t0 = time.perf_counter()
            r = ob.solve(A64, P.y, P.l, P.u, K=10, eps_gap=1e-6, step=eta, screening=screening)
            res[screening] = (time.perf_counter() - t0, r)
        out["cpu_baseline"] = {"value": round(1.0 / res[True][0], 3), "unit": "solves/s", "cores": _cores(),
                               "kind": "oracle",
                               "sample": f"one screened oracle solve at 4000x2000 FP64, b=0.002 "
                                         f"({res[True][1].iters} iterations)",
                               "oracle_screened_s": round(res[True][0], 3),
                               "oracle_unscreened_s": round(res[False][0], 3),
                               "oracle_speedup": round(res[False][0] / res[True][0], 3)}
    return out


def bench_sweep(args, device):
    """The fused PG sweep alone on a Fig. 1-law instance of any size (FP32
    storage), unscreened, a fixed number of iterations: the command the
    rocprofv3 traffic counters are read on for sizes above and below the
    256 MiB Infinity Cache."""
    m, n = args.sweep_m, args.sweep_n
    P = W.fig1_bvls(0, m, n, 0.01, dtype=np.float32)
    A = bx.colmajor(P.A, device=device)
    y, l, u = (torch.tensor(v, dtype=torch.float64, device=device) for v in (P.y, P.l, P.u))
    kw = dict(screening=False, screen_every=10, eps_gap=0.0, max_iter=args.sweep_iters, step=1e-6)
    bx.solve_bvls(A, y, l, u, **dict(kw, max_iter=10))
    _sync()
    _, _, info = bx.solve_bvls(A, y, l, u, profile=True, **kw)
    _sync()
    per_launch = n * (m * 4 + 36) + 8 * m
    avg_s = info["sweep_ms"] * 1e-3 / max(info["sweep_launches"], 1)
    ach = per_launch / avg_s / 1e9
    # reference: a plain device copy of A's size (read + write), event-timed
    src = A.t().contiguous().view(-1)
    dst = torch.empty_like(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    dst.copy_(src)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    _sync()
    copy_gbs = 5 * 2 * src.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    return {"workload": f"fused PG sweep, Fig. 1-law {m}x{n} FP32 ({4 * m * n / 2**20:.0f} MiB of A), "
                        f"{args.sweep_iters} unscreened iterations",
            "kernel": f"k_sweep variant {N.variant_for_rows(m)} for {m} rows",
            "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK, "unit": "GB/s",
                         "frac": round(ach / HBM_PEAK, 4), "algorithmic_bytes_per_launch": per_launch,
                         "avg_launch_us": round(avg_s * 1e6, 2), "launches": info["sweep_launches"],
                         "empty_kernel_events_us": round(1e3 * info["event_overhead_ms"], 2)},
            "device_copy_gbs_same_size": round(copy_gbs, 1)}


# --------------------------------------------------------------------------
def bench_table2(args, device):
    out = {"workload": "Paper Table 2 setup: BVLS m=1000 n=3000, |N(0,1)| entries, x-bar 5% U(0,1), "
                       "noise N(0,1), bounds [0,1]; PG K=10, gap 1e-6",
           "paper": {"baseline_s": 347.05, "screened_s": 48.46, "speedup": 7.16,
                     "hardware": "unstated (CPU/MATLAB setting)"}}
    P = W.table2_bvls(0, 1000, 3000)
    A, y, l, u = _upload(P, device)
    cls = N.row_class(P.m)
    tuned = bx.autotune.tune(device=device, classes=[cls], iters=100, reps=3)
    out["autotune"] = {"seconds": tuned["seconds"], "class": cls, "variant": tuned["classes"][cls]["best"],
                       "spread": tuned["classes"][cls]["scale"]}
    for screening in [True, False]:
        kw = dict(screening=screening, screen_every=10, eps_gap=1e-6, max_iter=2000000)
        t0 = time.perf_counter()
        x, sat, info = bx.solve_bvls(A, y, l, u, **kw)
        _sync()
        dt = time.perf_counter() - t0
        out["screened" if screening else "unscreened"] = {
            "seconds": round(dt, 3), "iters": info["iters"], "status": info["status_name"], "gap": info["gap"],
            "n_screened": info["n_lower"] + info["n_upper"],
            "us_per_iter": round(1e6 * dt / max(info["iters"], 1), 2),
            # average preserved fraction of the columns over the iterations
            "mean_preserved_fraction": round(info["col_iters"] / max(info["iters"], 1) / P.n, 4)}
    out["speedup"] = round(out["unscreened"]["seconds"] / out["screened"]["seconds"], 3)
    out["note"] = ("A is 1000 x 3000 (24 MB): an iteration is a few microseconds of HBM traffic plus a fixed "
                   "launch cost, so screening trims only the traffic part")
    # the primal-dual rows of Tab. 2: Chambolle-Pock, n = 500 ... 3000
    paper_pd = {500: (0.26, 0.08), 1000: (0.84, 0.19), 2000: (2.92, 0.59), 3000: (5.20, 0.95)}
    rows = []
    for n in (500, 1000, 2000, 3000):
        Q = W.table2_bvls(0, 1000, n)
        A, y, l, u = _upload(Q, device)
        row = {"n": n, "paper_baseline_s": paper_pd[n][0], "paper_screened_s": paper_pd[n][1]}
        for screening in (True, False):
            kw = dict(solver="cp", screening=screening, screen_every=10, eps_gap=1e-6, max_iter=2000000)
            bx.solve_bvls(A, y, l, u, **dict(kw, max_iter=20))
            _sync()
            t0 = time.perf_counter()
            x, sat, info = bx.solve_bvls(A, y, l, u, **kw)
            _sync()
            dt = time.perf_counter() - t0
            row["screened" if screening else "unscreened"] = {
                "seconds": round(dt, 4), "iters": info["iters"], "status": info["status_name"],
                "n_screened": info["n_lower"] + info["n_upper"],
                "mean_preserved_fraction": round(info["col_iters"] / max(info["iters"], 1) / n, 4)}
        row["speedup"] = round(row["unscreened"]["seconds"] / row["screened"]["seconds"], 3)
        log(f"[table2] CP n={n}: {row}")
        rows.append(row)
    out["chambolle_pock"] = rows
    return out


def bench_table1(args, device):
    """Paper Tab. 1 setup (context): NNLS with a_ij = |N(0,1)|, m = 2000,
    n = 1000 ... 6000, x-bar 5% nonzero, noise N(0,1); coordinate descent
    (one sweep per iteration, screening after every 10 sweeps), gap 1e-6,
    screened and unscreened, t = -1 (interior: Prop. 2 case 3)."""
    paper = {1000: (2.19, 0.71), 2000: (10.2, 2.09), 4000: (64.28, 9.52), 6000: (146.12, 18.63)}
    out = {"workload": "Paper Table 1 setup: NNLS m=2000, |N(0,1)| entries, x-bar 5% |N(0,1)|, noise N(0,1); "
                       "CD, screening every 10 sweeps, gap 1e-6",
           "rows": []}
    for n in args.table1_n:
        P = W.table1_nnls(0, 2000, n)
        A, y, _, _ = _upload(P, device)
        row = {"n": n, "paper_baseline_s": paper.get(n, (None, None))[0], "paper_screened_s": paper.get(n, (None, None))[1]}
        # n >= 4000: a budget of 20000 sweeps (the gap reached is reported)
        budget = args.table1_budget or (100000 if n <= 2000 else 20000)
        for screening in (True, False):
            kw = dict(solver="cd", screening=screening, screen_every=10, eps_gap=1e-6, max_iter=budget)
            bx.solve_nnls(A, y, **dict(kw, max_iter=20))
            _sync()
            t0 = time.perf_counter()
            x, sat, info = bx.solve_nnls(A, y, **kw)
            _sync()
            dt = time.perf_counter() - t0
            row["screened" if screening else "unscreened"] = {
                "seconds": round(dt, 4), "sweeps": info["iters"], "status": info["status_name"], "gap": info["gap"],
                "n_screened": info["n_lower"], "us_per_sweep": round(1e6 * dt / max(info["iters"], 1), 2),
                "mean_preserved_fraction": round(info["col_iters"] / max(info["iters"], 1) / n, 4)}
            log(f"[table1] n={n} {'screened' if screening else 'unscreened'}: {dt:.2f} s, {info['iters']} sweeps, "
                f"gap {info['gap']:.3e}")
        row["speedup"] = round(row["unscreened"]["seconds"] / row["screened"]["seconds"], 3)
        log(f"[table1] CD n={n}: {row}")
        out["rows"].append(row)
        del A, y
        torch.cuda.empty_cache()
    return out


def bench_huber(args, device):
    """Huber fidelity (eq. GAP_Safe_sph with alpha = 1, Sec. 3.3) on a tall
    BVLS problem with gross outliers, 16000 x 4000 FP32 (the Fig. 1 aspect at
    C2's 256 MB): screened and unscreened PG solves, the LS solve of the same
    data for reference, and the oracle's Huber solve of the full instance with
    the same step (iterate, passes and screened set compared)."""
    m, n, delta = 16000, 4000, 0.5
    log(f"[huber] generating {m}x{n} fp32")
    P = W.huber_bvls(0, m, n, np.float32)
    A, y, l, u = _upload(P, device)
    out = {"workload": f"Huber BVLS {m}x{n} unit N(0,1) columns stored FP32, x-bar ~ U(-3,3), box [-1,1], "
                       f"10% of rows shifted by +-U(2,5), delta {delta}; PG K=10, gap 1e-6",
           "delta": delta}
    reps = max(1, args.steps)
    for name, kw in (("screened", dict(fidelity="huber", huber_delta=delta, screening=True)),
                     ("unscreened", dict(fidelity="huber", huber_delta=delta, screening=False)),
                     ("ls_screened", dict(screening=True))):
        kw.update(screen_every=10, eps_gap=1e-6, max_iter=100000)
        bx.solve_bvls(A, y, l, u, **kw)
        _sync()
        t0 = time.perf_counter()
        for _ in range(reps):
            x, sat, info = bx.solve_bvls(A, y, l, u, **kw)
        _sync()
        dt = (time.perf_counter() - t0) / reps
        out[name] = {"solves_per_s": round(1.0 / dt, 3), "ms_per_solve": round(1e3 * dt, 3), "iters": info["iters"],
                     "status": info["status_name"], "gap": info["gap"], "primal": info["primal"],
                     "n_screened": info["n_lower"] + info["n_upper"],
                     "mean_preserved_fraction": round(info["col_iters"] / max(info["iters"], 1) / n, 4)}
        log(f"[huber] {name}: {out[name]}")
    out["speedup_screened"] = round(out["unscreened"]["ms_per_solve"] / out["screened"]["ms_per_solve"], 3)
    if not args.no_cpu_baseline:
        log("[huber] oracle solve of the full instance (same step)")
        from oracle import boxls as ob
        A64 = P.A64()
        eta = 1.0 / (1.05 * ob.lipschitz(A64))
        kw = dict(fidelity="huber", huber_delta=delta, screen_every=10, eps_gap=1e-6, max_iter=100000, step=eta)
        xg, sg, ig = bx.solve_bvls(A, y, l, u, **kw)
        _sync()
        t0 = time.perf_counter()
        res = ob.solve(A64, P.y, P.l, P.u, solver="pg", K=10, eps_gap=1e-6, max_iter=100000, step=eta,
                       huber_delta=delta)
        dt = time.perf_counter() - t0
        xg = xg.cpu().numpy()
        out["oracle_check"] = {
            "same_iters_passes": bool(ig["iters"] == res.iters and ig["passes"] == res.passes),
            "same_screened_set": bool(np.array_equal(sg.cpu().numpy(), res.sat)),
            "max_abs_x_diff": float(np.max(np.abs(xg - res.x))),
            "gap_gpu": ig["gap"], "gap_oracle": res.gap, "iters": res.iters}
        out["cpu_baseline"] = {"value": round(1.0 / dt, 4), "unit": "solves/s", "cores": _cores(), "kind": "oracle",
                               "sample": f"one full oracle Huber solve ({res.iters} iterations)"}
        log(f"[huber] oracle: {out['oracle_check']}")
    return out


def run(name, args, device):
    return {"c1": bench_c1, "c3": bench_c3, "c4": bench_c4, "c5": bench_c5, "table2": bench_table2,
            "table1": bench_table1, "huber": bench_huber,
            "fig1": bench_fig1, "sweep": bench_sweep}[name](args, device)
