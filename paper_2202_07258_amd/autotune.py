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
`bxs_set_sweep_variant`.  With that shape it then times whole solves for
several work-item spreads (`bxs_set_group_scale`: fewer, longer work items
write fewer partial products) and installs the fastest.  The table can be saved as JSON and re-applied later
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


def _solve(inst, copies: int, **kw) -> dict:
    """One unscreened solve of the instance, or, when `inst` is a list of
    instances of one shape, of all of them in one batch call; returns the
    info of the first problem."""
    if not isinstance(inst, list):
        A, y, l, u = inst
        return native.solve_bvls(A, y, l, u, **kw)[2]
    probs = [{"A": A, "y": y, "l": l, "u": u} for (A, y, l, u) in inst]
    return native.solve_bvls_varbatch(probs, **kw)[2][0]


def _time_variant(inst, iters: int, reps: int, copies: int = 1) -> float:
    """Average duration of one sweep launch (one per row class and iteration,
    over all copies) in microseconds."""
    kw = dict(screening=False, screen_every=10, max_iter=iters, eps_gap=0.0, step=0.5, profile=True)
    _solve(inst, copies, **dict(kw, max_iter=10))          # warm-up
    ms = 0.0
    launches = 0
    for _ in range(reps):
        info = _solve(inst, copies, **kw)
        ms += info["sweep_ms"]
        launches += info["sweep_launches"]
    return 1e3 * ms / max(launches, 1)


def _time_iteration(inst, iters: int, reps: int, copies: int = 1) -> float:
    """Device time per primal iteration of a whole unscreened solve (sweeps,
    partial reductions, screening passes), in microseconds, without timing
    events around the kernels."""
    kw = dict(screening=False, screen_every=10, max_iter=iters, eps_gap=0.0, step=0.5)
    _solve(inst, copies, **dict(kw, max_iter=10))
    best = float("inf")
    for _ in range(reps):
        info = _solve(inst, copies, **kw)
        best = min(best, 1e3 * info["ms_solve"] / max(info["iters"], 1))
    return best


SCALES = (1.0, 0.5, 0.25, 0.125, 0.0625)


def tune(device: str = "cuda:0", classes=None, iters: int = 40, reps: int = 2, cols_per_row: int = 4,
         max_bytes: int = 256 << 20, apply: bool = True, seed: int = 0, scales=SCALES, batch: bool = False,
         log=None) -> dict:
    """Time every candidate shape per row class (per sweep launch), then, with
    the fastest shape, every work-item spread in `scales` (per iteration of a
    whole solve, since fewer items also shorten the partial reduction).
    Returns {"classes": {cls: {"m", "n", "best", "us": {variant: us},
    "scale", "scale_us": {scale: us}}}, "seconds"}.  With apply=True the best
    shape and spread of every tuned class are installed.  batch=True times a
    batch call over distinct instances of the class's shape (as many as fit
    in max_bytes, at most 256), the setting of many independent instances:
    the best shape there is the one with the best throughput, not the lowest
    latency."""
    variants = native.sweep_variants()
    n_classes = 9
    classes = list(range(n_classes)) if classes is None else sorted(set(int(c) for c in classes))
    t0 = time.perf_counter()
    table = {}
    for c in classes:
        m = variants[c]["capacity"]
        n = max(64, min(cols_per_row * m, max_bytes // (4 * m)))
        copies = max(1, min(256, max_bytes // (4 * m * n))) if batch else 1
        inst = (_instance(m, n, device, seed + c) if copies == 1 else
                [_instance(m, n, device, seed + 1000 * (c + 1) + k) for k in range(copies)])
        cands = [v["id"] for v in variants if v["capacity"] >= m]
        before = native.variant_for_rows(m)
        us = {}
        for v in cands:
            native.set_sweep_variant(c, v)
            us[v] = _time_variant(inst, iters, reps, copies)
            if log:
                log(f"[autotune] class {c} (m={m}, n={n}) variant {v}: {us[v]:.2f} us/launch")
        best = min(us, key=us.get)
        native.set_sweep_variant(c, best)
        scale_before = native.group_scale(c)
        sus = {}
        for sc in scales:
            native.set_group_scale(c, sc)
            sus[sc] = _time_iteration(inst, iters, reps, copies)
            if log:
                log(f"[autotune] class {c} variant {best} spread {sc}: {sus[sc]:.2f} us/iteration")
        best_scale = min(sus, key=sus.get)
        native.set_sweep_variant(c, best if apply else before)
        native.set_group_scale(c, best_scale if apply else scale_before)
        table[c] = {"m": m, "n": n, "copies": copies, "best": best, "previous": before,
                    "us": {int(k): round(v, 3) for k, v in us.items()},
                    "scale": best_scale, "previous_scale": scale_before,
                    "scale_us": {float(k): round(v, 3) for k, v in sus.items()}}
        del inst
    torch.cuda.synchronize()
    return {"classes": table, "seconds": round(time.perf_counter() - t0, 3), "device": torch.cuda.get_device_name()}


def apply_table(table: dict) -> None:
    """Install the shapes and spreads of a table returned by tune() (or loaded
    by load())."""
    for c, row in table["classes"].items():
        native.set_sweep_variant(int(c), int(row["best"]))
        if "scale" in row:
            native.set_group_scale(int(c), float(row["scale"]))


def save(table: dict, path: str) -> None:
    with open(path, "w") as f:
        json.dump(table, f, indent=1)


def load(path: str) -> dict:
    with open(path) as f:
        return json.load(f)


# --------------------------------------------------------------------------
# Persistent table, keyed by what the timings depend on
# --------------------------------------------------------------------------
def cache_key(device: str = "cuda:0", batch: bool = False) -> str:
    """GPU architecture, HIP runtime, library version and tuning setting:
    a table tuned under one key is reused only under the same key."""
    props = torch.cuda.get_device_properties(torch.device(device))
    arch = getattr(props, "gcnArchName", props.name)
    return "|".join([arch, f"hip {torch.version.hip}", native.version(), "batch" if batch else "single"])


def default_cache_path() -> str:
    import os
    return os.environ.get("BOXSCREEN_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "boxscreen", "autotune.json"))


def tuned(device: str = "cuda:0", classes=None, batch: bool = False, path: str | None = None, log=None,
          **tune_kw) -> dict:
    """Install tuned shapes and spreads for `classes`, reusing the rows of
    the persistent table stored under this device's key and tuning (then
    storing) only the classes it lacks.  Returns {"classes", "seconds",
    "key", "cached": [classes reused], "tuned": [classes tuned now]}."""
    import os
    path = path or default_cache_path()
    key = cache_key(device, batch)
    store = {}
    try:
        store = load(path)
    except (OSError, ValueError):
        store = {}
    rows = {int(c): r for c, r in store.get(key, {}).items()}
    want = list(range(9)) if classes is None else sorted(set(int(c) for c in classes))
    missing = [c for c in want if c not in rows]
    t0 = time.perf_counter()
    if missing:
        fresh = tune(device=device, classes=missing, batch=batch, log=log, **tune_kw)
        rows.update({int(c): r for c, r in fresh["classes"].items()})
        store[key] = {str(c): r for c, r in sorted(rows.items())}
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            tmp = path + ".tmp"
            save(store, tmp)
            os.replace(tmp, path)
        except OSError:
            pass                                  # read-only home: the table lives for this process
    table = {"classes": {c: rows[c] for c in want}}
    apply_table(table)
    table.update({"seconds": round(time.perf_counter() - t0, 3), "key": key,
                  "cached": [c for c in want if c not in missing], "tuned": missing})
    return table
