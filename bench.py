#!/usr/bin/env python3
"""Throughput benchmark of the screened box-constrained LS solver on one MI355X.

Workload (default): BVLS, A 4000 x 16000 with i.i.d. N(0,1) entries and unit
l2 columns stored in FP32, l_j ~ U[-1,0], u_j ~ U[0,1], 40% of x* on a bound,
y = A x* + N(0, 0.01^2); projected gradient, screening pass every 10
iterations, stop at certified duality gap < 1e-6.  The matrix defines the
problem; all arithmetic is FP64.

One step = one complete solve from x0 = 0 (setup: column statistics, power
iteration for the step; then the screening loop) with every input already
resident in HBM.  `value` is screened solves per second, timed as a user runs
them (no timing events).  The same line also carries the unscreened baseline,
a planted non-degenerate companion of the same shape (where screening fires),
the roofline of the dominant kernel (the fused projected-gradient sweep) from
HIP events recorded on the solve's stream around each of its launches during
a second, profiled set of the same timed solves, and the FP64 oracle timed on
the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "solves/sec to gap 1e-6 (screened vs unscreened), HBM GB/s % of peak"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pg_sweep_c2_traffic.md")
SWEEP_SOURCE = os.path.join(ROOT, "paper_2202_07258_amd", "csrc", "sweep.h")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def upload(P, device):
    import torch
    import paper_2202_07258_amd as bx
    A = bx.colmajor(P.A, device=device)
    y, l, u = (torch.tensor(v, dtype=torch.float64, device=device) for v in (P.y, P.l, P.u))
    return A, y, l, u


def time_solves(dev_inputs, steps, warmup, **kw):
    import torch
    import paper_2202_07258_amd as bx
    A, y, l, u = dev_inputs
    out = None
    for _ in range(warmup):
        out = bx.solve_bvls(A, y, l, u, **kw)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(steps):
        out = bx.solve_bvls(A, y, l, u, **kw)
        infos.append(out[2])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dt, infos, out


def sweep_roofline(infos, m, n, elem_bytes):
    """Algorithmic bytes of one fused PG sweep launch: every preserved column
    once (m * elem_bytes), its x read and write, l, u and index (36 B), plus
    the residual m-vector (8 m), with the preserved-set size averaged over
    the solve's iterations (the timed launches are all but the first of each
    screening pass).  Duration: HIP events recorded on the solve's stream
    around each launch (dispatch included)."""
    col_iters = sum(i["col_iters"] for i in infos)
    iters = sum(i["iters"] for i in infos)
    launches = sum(i["sweep_launches"] for i in infos)
    ms = sum(i["sweep_ms"] for i in infos)
    if launches == 0 or ms <= 0 or iters == 0:
        return None
    per_launch = col_iters / iters * (m * elem_bytes + 36) + 8 * m
    avg_s = ms * 1e-3 / launches
    # the event pair around a launch also spans its dispatch, so this duration
    # is an upper bound of the kernel's own (reported: the same pair's elapsed
    # time around an empty kernel)
    overhead = max(i.get("event_overhead_ms", 0.0) for i in infos) * 1e-3
    achieved = per_launch / avg_s / 1e9
    # the counter summary was taken on an unscreened sweep over all n columns:
    # it describes only launches that still read every column
    traffic = measured_traffic(sweep_kernel_name(m), m) if col_iters == iters * n else None
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": sweep_kernel_name(m),
            "algorithmic_bytes_per_launch": int(per_launch), "avg_launch_us": round(avg_s * 1e6, 2),
            "empty_kernel_events_us": round(overhead * 1e6, 2),
            "launches": launches}


def _source_digest(path):
    """Digest of the column-sweep kernel's source text (the whole of sweep.h:
    the kernel template and its launchers)."""
    import hashlib
    try:
        with open(path, "rb") as f:
            return hashlib.sha256(f.read()).hexdigest()[:16]
    except OSError:
        return None


def measured_traffic(kernel, m):
    """HBM bytes per launch of the sweep from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration),
    or None when the summary is missing or was taken on another version of
    the kernel source, another kernel shape, another row count or another
    work-item spread (which sets how many partial products are written)."""
    try:
        with open(TRAFFIC_FILE) as f:
            kv = dict(line.split(":", 1) for line in f.read().splitlines()
                      if ":" in line and not line.startswith(("#", " ", "|", "`")))
        kv = {k.strip(): v.strip() for k, v in kv.items()}
        if kv.get("kernel_source_sha256") != _source_digest(SWEEP_SOURCE):
            return None
        if kv.get("kernel") != kernel or int(kv.get("rows", -1)) != m:
            return None
        from paper_2202_07258_amd import native as N
        if float(kv.get("spread", -1)) != N.group_scale(N.row_class(m)):
            return None
        return int(float(kv["bytes_per_launch"]))
    except (OSError, ValueError, KeyError):
        return None


def copy_calibration(device):
    """A plain device-to-device copy of known size, for scaling the HBM byte
    counters (FETCH_SIZE / WRITE_SIZE) read on the sweep."""
    import torch
    n = 1 << 28
    src = torch.ones(n, dtype=torch.float32, device=device)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    return {"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 3}


def sweep_kernel_name(m):
    """Shape of the fused PG sweep the library runs for m rows."""
    from paper_2202_07258_amd import native as N
    v = N.sweep_variants()[N.variant_for_rows(m)]
    return (f"k_sweep<float,{v['tpc']},{v['ng']},{v['rows']},4,{v['cbi']},{v['pd']},kModePG> "
            "(fused A^T r / projected step / A x)")


def cpu_baseline(P, budget_iters=None):
    """The FP64 oracle (NumPy) solving the same instance on the host cores."""
    import numpy as np
    from oracle import boxls as ob
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    A64 = P.A64()
    t0 = time.perf_counter()
    eta = 1.0 / (1.05 * ob.lipschitz_power(A64, 20))
    kw = dict(K=10, eps_gap=1e-6, step=eta)
    if budget_iters:
        kw["max_iter"] = budget_iters
    res = ob.solve(A64, P.y, P.l, P.u, **kw)
    dt = time.perf_counter() - t0
    return dt, res, cores


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-companion", action="store_true")
    ap.add_argument("--no-unscreened", action="store_true")
    ap.add_argument("--no-bf16", action="store_true", help="skip the bfloat16-storage leg of the C2 run")
    ap.add_argument("--cpu-iters", type=int, default=0,
                    help="bound the oracle baseline to this many iterations (0: full solve)")
    ap.add_argument("--workload", default="c2", choices=["c2", "c1", "c3", "c4", "c5", "table1", "table2", "fig1", "sweep", "huber"],
                    help="c2 (default): the headline workload; the others are measured separately")
    ap.add_argument("--sweep-m", type=int, default=8000)
    ap.add_argument("--sweep-n", type=int, default=16000)
    ap.add_argument("--sweep-iters", type=int, default=50)
    ap.add_argument("--c3-rhs", type=int, default=8192)
    ap.add_argument("--c3-iters", type=int, default=200)
    ap.add_argument("--c4-count", type=int, default=2048)
    ap.add_argument("--c4-planted", action="store_true", help="C4-pl: the planted, non-degenerate companion")
    ap.add_argument("--c4-oracle-budget", type=float, default=60.0,
                    help="host seconds for the C4 oracle sample (smallest instances first)")
    ap.add_argument("--c5-iters", type=int, default=20000)
    ap.add_argument("--table1-n", type=int, nargs="+", default=[1000, 2000, 4000, 6000],
                    help="Tab. 1 column counts to run (m = 2000)")
    ap.add_argument("--table1-budget", type=int, default=0,
                    help="sweep budget per Tab. 1 solve (0: 100000 for n <= 2000, else 20000)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (for scaling rocprofv3 byte counters) and exit")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; --gpus > 1 is not supported "
                                   "(the solve of one instance is a single-GPU workload)"}))
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2202_07258_amd as bx
    from synth import workloads as W

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    bx.load()
    device = "cuda:0"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        print(json.dumps(copy_calibration(device)), flush=True)
        return
    if args.workload != "c2":
        import bench_workloads
        out = bench_workloads.run(args.workload, args, device)
        print(json.dumps(out), flush=True)
        return

    log("[bench] generating C2 (4000x16000 fp32 BVLS)")
    P = W.c2_bvls(0)
    dev = upload(P, device)
    m, n = P.m, P.n

    log("[bench] screened solves")
    # `value`: the solves as a user runs them (default options: direct
    # launches, no timing events).  The roofline: the same solves
    # again with HIP events around every PG sweep launch (profile mode), which
    # adds a few microseconds between kernels but not to the kernels.
    dt, _, (x, sat, info) = time_solves(dev, args.steps, args.warmup, screening=True, eps_gap=1e-6,
                                        screen_every=10)
    value = args.steps / dt
    dtp, infos, _ = time_solves(dev, args.steps, 0, screening=True, eps_gap=1e-6, screen_every=10, profile=True)
    roof = sweep_roofline(infos, m, n, 4)
    if roof:
        roof["profiled_ms_per_step"] = round(1e3 * dtp / args.steps, 3)
    xg = x.cpu().numpy()
    result = {
        "metric": METRIC, "value": round(value, 3), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * dt / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "C2: BVLS 4000x16000, N(0,1) unit columns stored FP32, FP64 gap/screening, "
                               "PG with screening every 10 iterations, certified gap < 1e-6",
                   "m": m, "n": n, "a_storage": "fp32", "solver": "pg", "screen_every": 10, "eps_gap": 1e-6},
        "solve": {"iters": info["iters"], "passes": info["passes"], "gap": info["gap"],
                  "n_screened": info["n_lower"] + info["n_upper"], "status": info["status_name"],
                  "ms_setup": round(info["ms_setup"], 3), "ms_solve": round(info["ms_solve"], 3)},
        "roofline": roof,
    }


    if not args.no_unscreened:
        log("[bench] unscreened solves")
        dt0, infos0, (x0, _, info0) = time_solves(dev, args.steps, args.warmup, screening=False,
                                                  eps_gap=1e-6, screen_every=10)
        result["unscreened"] = {"value": round(args.steps / dt0, 3), "unit": "solves/s",
                                "ms_per_step": round(1e3 * dt0 / args.steps, 3), "iters": info0["iters"],
                                "speedup_screened": round((args.steps / dt) / (args.steps / dt0), 3)}
    if not args.no_companion:
        log("[bench] planted companion C2-pl (same shape, non-degenerate)")
        Q = W.c2_planted(0)
        devq = upload(Q, device)
        dts, _, (xq, sq, iq) = time_solves(devq, args.steps, args.warmup, screening=True, eps_gap=1e-6,
                                           screen_every=10)
        _, infs, _ = time_solves(devq, 1, 0, screening=True, eps_gap=1e-6, screen_every=10, profile=True)
        comp = {"workload": "C2-pl: planted optimum, |F| = 0.4 m free, 90% saturated, same law as C2",
                "screened": {"value": round(args.steps / dts, 3), "ms_per_step": round(1e3 * dts / args.steps, 3),
                             "iters": iq["iters"], "n_screened": iq["n_lower"] + iq["n_upper"],
                             "gap": iq["gap"],
                             "max_abs_err_vs_planted_optimum": float(np.max(np.abs(xq.cpu().numpy() - Q.x_true)))},
                "roofline_screened": sweep_roofline(infs, Q.m, Q.n, 4)}
        if not args.no_unscreened:
            dtu, _, (_, _, iu) = time_solves(devq, args.steps, args.warmup, screening=False, eps_gap=1e-6,
                                             screen_every=10)
            comp["unscreened"] = {"value": round(args.steps / dtu, 3),
                                  "ms_per_step": round(1e3 * dtu / args.steps, 3), "iters": iu["iters"]}
            comp["speedup_screened"] = round(dtu / dts, 3)
        # the ceiling of the dual update (Sec. 5.1, Fig. 3): the same solve
        # screened with the planted dual optimum in place of the dual update
        ts = torch.tensor(Q.meta["theta"], dtype=torch.float64, device=device)
        dto, _, (_, _, io) = time_solves(devq, 1, 1, screening=True, eps_gap=1e-6, screen_every=10, theta_star=ts)
        comp["screened_oracle_dual_point"] = {"value": round(1 / dto, 3), "ms_per_step": round(1e3 * dto, 3),
                                              "iters": io["iters"], "n_screened": io["n_lower"] + io["n_upper"],
                                              "mean_preserved_fraction":
                                                  round(io["col_iters"] / max(io["iters"], 1) / Q.n, 4)}
        if "unscreened" in comp:
            comp["speedup_oracle_dual_point"] = round(dtu / args.steps / dto, 3)
        result["companion"] = comp
        del devq
        torch.cuda.empty_cache()

    if not args.no_companion:
        # where screening pays at C2's shape: the saturation-ratio law of
        # Sec. 5.1, Fig. 1 (a_ij, y_i ~ N(0,1), box b [-1, 1]) with b = 0.0005,
        # 97% of the coordinates saturated at the optimum
        log("[bench] Fig. 1 law at C2's shape, b = 0.0005 (screening pays)")
        Q = W.fig1_bvls(0, m, n, 0.0005, dtype=np.float32)
        devq = upload(Q, device)
        dts, _, (xq, sq, iq) = time_solves(devq, args.steps, args.warmup, screening=True, eps_gap=1e-6,
                                           screen_every=10)
        leg = {"workload": f"Fig. 1 law: BVLS {m}x{n} N(0,1) entries (columns not normalised) stored FP32, "
                           "y ~ N(0,1), box 0.0005 [-1, 1], PG K=10, gap 1e-6",
               "screened": {"value": round(args.steps / dts, 3), "ms_per_step": round(1e3 * dts / args.steps, 3),
                            "iters": iq["iters"], "n_screened": iq["n_lower"] + iq["n_upper"], "gap": iq["gap"],
                            "mean_preserved_fraction": round(iq["col_iters"] / max(iq["iters"], 1) / n, 4)}}
        if not args.no_unscreened:
            dtu, _, (_, _, iu) = time_solves(devq, args.steps, args.warmup, screening=False, eps_gap=1e-6,
                                             screen_every=10)
            leg["unscreened"] = {"value": round(args.steps / dtu, 3), "ms_per_step": round(1e3 * dtu / args.steps, 3),
                                 "iters": iu["iters"]}
            leg["speedup_screened"] = round(dtu / dts, 3)
        result["screening_pays"] = leg
        del devq
        torch.cuda.empty_cache()

    if not args.no_bf16:
        # precision tiering of the storage: the same instance with A rounded to
        # bfloat16 (half the bytes per sweep; every element still promoted
        # exactly to FP64, so the solve is exact for the stored problem)
        log("[bench] C2 with bfloat16 storage of A")
        Ab = dev[0].to(torch.bfloat16)
        devb = (Ab, dev[1], dev[2], dev[3])
        dtb, _, (xb, sb, ib) = time_solves(devb, args.steps, args.warmup, screening=True, eps_gap=1e-6,
                                           screen_every=10)
        _, infb, _ = time_solves(devb, 1, 0, screening=True, eps_gap=1e-6, screen_every=10, profile=True)
        rb = sweep_roofline(infb, m, n, 2)
        if rb:
            rb["traffic"] = None
            rb["kernel"] = rb["kernel"].replace("k_sweep<float,", "k_sweep<__bf16,").replace(",4,", ",8,", 1)
        result["c2_bf16_storage"] = {
            "value": round(args.steps / dtb, 3), "unit": "solves/s", "ms_per_step": round(1e3 * dtb / args.steps, 3),
            "iters": ib["iters"], "gap": ib["gap"], "status": ib["status_name"],
            "speedup_vs_fp32_storage": round((args.steps / dtb) / value, 3),
            "max_abs_diff_x_vs_fp32_storage": float((xb - x).abs().max()),
            "roofline": rb}
        del Ab, devb
    del dev
    torch.cuda.empty_cache()

    if not args.no_cpu_baseline:
        log("[bench] FP64 oracle on the host (cpu baseline)")
        dtc, res, cores = cpu_baseline(P, args.cpu_iters or None)
        full = res.status == "ok"
        if full:
            val = 1.0 / dtc
            sample = f"one full oracle solve of the C2 instance ({res.iters} PG iterations, {res.passes} passes)"
        else:
            val = (res.iters / dtc) / max(info["iters"], 1)
            sample = (f"first {res.iters} oracle PG iterations of the C2 instance, scaled to the "
                      f"{info['iters']}-iteration solve")
        result["cpu_baseline"] = {"value": round(val, 5), "unit": "solves/s", "cores": cores, "kind": "oracle",
                                  "sample": sample, "seconds": round(dtc, 2)}
        # the same oracle on one thread, on a bounded sample (30 PG iterations,
        # scaled to the solve's iteration count)
        try:
            from threadpoolctl import threadpool_limits
            with threadpool_limits(limits=1):
                dt1, res1, _ = cpu_baseline(P, 30)
            result["cpu_baseline"]["value_1_thread"] = round((res1.iters / dt1) / max(info["iters"], 1), 5)
            result["cpu_baseline"]["sample_1_thread"] = (f"first {res1.iters} oracle PG iterations on one thread, "
                                                         f"scaled to the {info['iters']}-iteration solve")
        except ImportError:
            pass
        # the oracle's own FP64 gap (eq. Dual_Gap) at the GPU's returned x
        from oracle import boxls as ob
        A64 = P.A64()
        theta = ob.residual_dual_point(A64, P.y, xg)
        result["solve"]["gap_oracle_at_x"] = ob.duality_gap(A64, P.y, P.l, P.u, xg, theta)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
