"""Autotuner for the column-sweep shapes of libboxscreen.

The sweep kernels are compiled for a fixed set of shapes (threads per column,
column groups per workgroup, rows per thread, columns per round, prefetch
depth); the row classes are the shapes 0..8 in order of row capacity, and an
instance with m rows belongs to the smallest class that holds m.  For every
requested class this module builds a synthetic BVLS instance with the class's
largest row count (Gaussian unit columns, FP32 storage, bounds [-1, 1]), runs
a fixed number of unscreened PG iterations with each compiled shape that can
hold those rows, times every sweep launch with the library's own HIP events
(`opts.profile`), and installs the fastest shape for the class with
`bxs_set_sweep_variant`.  The table can be saved as JSON and re-applied later
in the same or another process.
"""
from __future__ import annotations

import json
import time

import torch

from . import native


def _instance(m: int, n: int, device, seed: int):
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    At = torch.randn((n, m), generator=g, device=device, dtype=torch.float32)
    At /= At.norm(dim=1, keepdim=True)
    A = At.t()                                            # (m, n) column-major view
    y = torch.randn(m, generator=g, device=device, dtype=torch.float64)
    l = -torch.ones(n, dtype=torch.float64, device=device)
    u = torch.ones(n, dtype=torch.float64, device=device)
    return A, y, l, u


def _time_variant(inst, iters: int, reps: int) -> float:
    """Average sweep launch duration in microseconds."""
    A, y, l, u = inst
    kw = dict(screening=False, screen_every=10, max_iter=iters, eps_gap=0.0, step=0.5, profile=True)
    native.solve_bvls(A, y, l, u, **dict(kw, max_iter=10))          # warm-up
    ms = 0.0
    launches = 0
    for _ in range(reps):
        _, _, info = native.solve_bvls(A, y, l, u, **kw)
        ms += info["sweep_ms"]
        launches += info["sweep_launches"]
    return 1e3 * ms / max(launches, 1)


def tune(device: str = "cuda:0", classes=None, iters: int = 40, reps: int = 2, cols_per_row: int = 4,
         max_bytes: int = 256 << 20, apply: bool = True, seed: int = 0, log=None) -> dict:
    """Time every candidate shape per row class; returns
    {"classes": {cls: {"m", "n", "best", "us": {variant: us}}}, "seconds"}.
    With apply=True the best shape of every tuned class is installed."""
    variants = native.sweep_variants()
    n_classes = 9
    classes = list(range(n_classes)) if classes is None else sorted(set(int(c) for c in classes))
    t0 = time.perf_counter()
    table = {}
    for c in classes:
        m = variants[c]["capacity"]
        n = max(64, min(cols_per_row * m, max_bytes // (4 * m)))
        inst = _instance(m, n, device, seed + c)
        cands = [v["id"] for v in variants if v["capacity"] >= m]
        before = native.variant_for_rows(m)
        us = {}
        for v in cands:
            native.set_sweep_variant(c, v)
            us[v] = _time_variant(inst, iters, reps)
            if log:
                log(f"[autotune] class {c} (m={m}, n={n}) variant {v}: {us[v]:.2f} us/launch")
        best = min(us, key=us.get)
        native.set_sweep_variant(c, best if apply else before)
        table[c] = {"m": m, "n": n, "best": best, "previous": before,
                    "us": {int(k): round(v, 3) for k, v in us.items()}}
        del inst
    torch.cuda.synchronize()
    return {"classes": table, "seconds": round(time.perf_counter() - t0, 3), "device": torch.cuda.get_device_name()}


def apply_table(table: dict) -> None:
    """Install the shapes of a table returned by tune() (or loaded by load())."""
    for c, row in table["classes"].items():
        native.set_sweep_variant(int(c), int(row["best"]))


def save(table: dict, path: str) -> None:
    with open(path, "w") as f:
        json.dump(table, f, indent=1)


def load(path: str) -> dict:
    with open(path) as f:
        return json.load(f)
