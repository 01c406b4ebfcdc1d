"""ctypes binding of libboxscreen.so: argument marshalling only.

Every function takes PyTorch tensors that already live on the GPU, passes
their device pointers and the current HIP stream to the C ABI declared in
include/boxscreen.h, and returns the output tensors plus the info record.  All
arithmetic of the solve happens in the library's HIP kernels; there is no
fallback of any kind: if the shared library is missing or fails to load, every
call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Any

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIBRARY_PATH = os.path.join(_PKG, "libboxscreen.so")

BXS_OK, BXS_ERR_ARG, BXS_ERR_SHAPE, BXS_ERR_NONFINITE, BXS_ERR_BOUNDS, BXS_ERR_DEVICE, BXS_ERR_NOMEM, BXS_MAXITER, \
    BXS_SINGULAR = range(9)
STATUS_NAMES = {0: "ok", 1: "err_arg", 2: "err_shape", 3: "err_nonfinite", 4: "err_bounds",
                5: "err_device", 6: "err_nomem", 7: "maxiter", 8: "singular"}
BXS_PG, BXS_CD, BXS_CP = 0, 1, 2
BXS_F64, BXS_F32, BXS_BF16 = 0, 1, 2
MAX_ROWS = 16384
T_CHOICES = {"given": 0, "neg_mean_column": 1, "neg_most_correlated": 2, "neg_least_correlated": 3,
             "normal_equations": 4}


class PassRecord(C.Structure):
    _fields_ = [("iters", C.c_long), ("n_active", C.c_long), ("gap", C.c_double), ("radius", C.c_double),
                ("eps", C.c_double), ("primal", C.c_double), ("n_screened", C.c_long)]


class Opts(C.Structure):
    _fields_ = [("solver", C.c_int), ("screening", C.c_int), ("screen_every", C.c_int),
                ("max_iter", C.c_long), ("eps_gap", C.c_double), ("step", C.c_double),
                ("power_iters", C.c_int), ("t", C.c_void_p), ("stream", C.c_void_p),
                ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t),
                ("history", C.POINTER(PassRecord)), ("history_cap", C.c_long), ("profile", C.c_int),
                ("iter_precision", C.c_int), ("graph", C.c_int), ("theta_star", C.c_void_p),
                ("t_choice", C.c_int), ("fidelity", C.c_int), ("deterministic", C.c_int),
                ("huber_delta", C.c_double)]


class Info(C.Structure):
    _fields_ = [("status", C.c_int), ("t_valid", C.c_int), ("iters", C.c_long), ("passes", C.c_long),
                ("n_active", C.c_long), ("n_lower", C.c_long), ("n_upper", C.c_long),
                ("gap", C.c_double), ("primal", C.c_double), ("radius", C.c_double), ("eps", C.c_double),
                ("step", C.c_double), ("lipschitz", C.c_double), ("ms_setup", C.c_double),
                ("ms_solve", C.c_double), ("col_iters", C.c_long), ("sweep_ms", C.c_double),
                ("sweep_launches", C.c_long), ("event_overhead_ms", C.c_double), ("t_column", C.c_long),
                ("dual", C.c_double), ("max_margin", C.c_double), ("n_free", C.c_long)]


class Problem(C.Structure):
    _fields_ = [("m", C.c_long), ("n", C.c_long), ("lda", C.c_long), ("A", C.c_void_p),
                ("y", C.c_void_p), ("l", C.c_void_p), ("u", C.c_void_p), ("x", C.c_void_p),
                ("sat", C.c_void_p)]


NOALLOC_SCRATCH_BYTES = 32 << 20   # BXS_NOALLOC_SCRATCH_BYTES of include/boxscreen.h

EXPORTED = ["bxs_default_opts", "bxs_workspace_size", "bxs_workspace_size_batch", "solve_bvls", "solve_bvls_noalloc",
            "solve_nnls", "solve_bvls_varbatch", "bxs_last_error", "bxs_version",
            "bxs_num_sweep_variants", "bxs_sweep_variant_info", "bxs_row_class", "bxs_set_sweep_variant",
            "bxs_sweep_variant_for_rows", "bxs_set_group_scale", "bxs_group_scale", "bxs_set_cd_block",
            "solve_nnls_batched_shared", "bxs_workspace_size_batched", "nnls_adjoint", "bvls_adjoint",
            "bxs_workspace_size_adjoint"]

_lib = None


def load(path: str = LIBRARY_PATH) -> C.CDLL:
    """Load libboxscreen.so (raises if it is absent: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with python -m paper_2202_07258_amd.build "
                           "(hipcc --offload-arch=gfx950); the solvers have no CPU fallback")
    lib = C.CDLL(path)
    lib.bxs_default_opts.argtypes = [C.POINTER(Opts)]
    lib.bxs_default_opts.restype = None
    lib.bxs_workspace_size.argtypes = [C.c_long, C.c_long, C.POINTER(Opts), C.POINTER(C.c_size_t)]
    lib.bxs_workspace_size.restype = C.c_int
    lib.bxs_workspace_size_batch.argtypes = [C.c_long, C.POINTER(C.c_long), C.POINTER(C.c_long),
                                             C.POINTER(Opts), C.POINTER(C.c_size_t)]
    lib.bxs_workspace_size_batch.restype = C.c_int
    lib.solve_bvls.argtypes = [C.c_long, C.c_long, C.c_int, C.c_void_p, C.c_long, C.c_void_p, C.c_void_p,
                               C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(Opts), C.POINTER(Info)]
    lib.solve_bvls.restype = C.c_int
    lib.solve_bvls_noalloc.argtypes = lib.solve_bvls.argtypes
    lib.solve_bvls_noalloc.restype = C.c_int
    lib.solve_nnls.argtypes = [C.c_long, C.c_long, C.c_int, C.c_void_p, C.c_long, C.c_void_p, C.c_void_p,
                               C.c_void_p, C.POINTER(Opts), C.POINTER(Info)]
    lib.solve_nnls.restype = C.c_int
    lib.solve_bvls_varbatch.argtypes = [C.c_long, C.c_int, C.POINTER(Problem), C.POINTER(Opts), C.POINTER(Info)]
    lib.solve_bvls_varbatch.restype = C.c_int
    lib.bxs_last_error.argtypes = []
    lib.bxs_last_error.restype = C.c_char_p
    lib.bxs_version.argtypes = []
    lib.bxs_version.restype = C.c_char_p
    lib.bxs_num_sweep_variants.argtypes = []
    lib.bxs_num_sweep_variants.restype = C.c_int
    lib.bxs_sweep_variant_info.argtypes = [C.c_int] + [C.POINTER(C.c_int)] * 5 + [C.POINTER(C.c_long)]
    lib.bxs_sweep_variant_for_rows.argtypes = [C.c_long]
    lib.bxs_sweep_variant_for_rows.restype = C.c_int
    lib.bxs_sweep_variant_info.restype = C.c_int
    lib.bxs_row_class.argtypes = [C.c_long]
    lib.bxs_row_class.restype = C.c_int
    lib.bxs_set_sweep_variant.argtypes = [C.c_int, C.c_int]
    lib.bxs_set_sweep_variant.restype = C.c_int
    lib.bxs_set_group_scale.argtypes = [C.c_int, C.c_double]
    lib.bxs_set_group_scale.restype = C.c_int
    lib.bxs_group_scale.argtypes = [C.c_int]
    lib.bxs_group_scale.restype = C.c_double
    lib.bxs_set_cd_block.argtypes = [C.c_int]
    lib.bxs_set_cd_block.restype = C.c_int
    lib.solve_nnls_batched_shared.argtypes = [C.c_long, C.c_long, C.c_long, C.c_int, C.c_void_p, C.c_long,
                                              C.c_void_p, C.c_long, C.c_void_p, C.c_long, C.c_void_p, C.c_long,
                                              C.POINTER(Opts), C.POINTER(Info)]
    lib.solve_nnls_batched_shared.restype = C.c_int
    lib.bxs_workspace_size_batched.argtypes = [C.c_long, C.c_long, C.c_long, C.POINTER(Opts), C.POINTER(C.c_size_t)]
    lib.bxs_workspace_size_batched.restype = C.c_int
    lib.nnls_adjoint.argtypes = [C.c_long, C.c_long, C.c_long, C.c_int, C.c_void_p, C.c_long, C.c_void_p, C.c_long,
                                 C.c_void_p, C.c_long, C.c_void_p, C.c_long, C.c_void_p, C.c_long, C.c_void_p,
                                 C.c_long, C.c_void_p, C.c_long, C.POINTER(Opts), C.POINTER(C.c_long)]
    lib.nnls_adjoint.restype = C.c_int
    lib.bvls_adjoint.argtypes = [C.c_long, C.c_long, C.c_long, C.c_int, C.c_void_p, C.c_long, C.c_void_p, C.c_long,
                                 C.c_void_p, C.c_long, C.c_void_p, C.c_void_p, C.c_void_p, C.c_long, C.c_void_p,
                                 C.c_long, C.c_void_p, C.c_long, C.c_void_p, C.c_long, C.c_void_p, C.c_long,
                                 C.POINTER(Opts), C.POINTER(C.c_long)]
    lib.bvls_adjoint.restype = C.c_int
    lib.bxs_workspace_size_adjoint.argtypes = [C.c_long, C.c_long, C.c_long, C.POINTER(C.c_size_t)]
    lib.bxs_workspace_size_adjoint.restype = C.c_int
    _lib = lib
    return lib


class BoxscreenError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else t.data_ptr()


def _check_matrix(A: torch.Tensor):
    if not (A.is_cuda and A.dim() == 2):
        raise ValueError("A must be a 2-D tensor on the GPU")
    if A.dtype not in (torch.float32, torch.float64, torch.bfloat16):
        raise ValueError("A must be float32, float64 or bfloat16")
    m, n = A.shape
    if A.stride(0) != 1 and m > 1:
        raise ValueError("A must be column-major (stride(0) == 1); use colmajor()")
    lda = A.stride(1) if n > 1 else max(m, 1)
    dt = {torch.float32: BXS_F32, torch.float64: BXS_F64, torch.bfloat16: BXS_BF16}[A.dtype]
    return m, n, max(lda, m), dt


def _vec(v: torch.Tensor | None, length: int, name: str):
    if v is None:
        return None
    if not (v.is_cuda and v.dtype == torch.float64 and v.dim() == 1 and v.numel() == length and v.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float64 GPU vector of length {length}")
    return v


def colmajor(A: Any, device="cuda", dtype=None) -> torch.Tensor:
    """(m, n) column-major GPU tensor from a numpy array or tensor (copy)."""
    T = torch.as_tensor(A)
    if dtype is not None:
        T = T.to(dtype)
    return T.t().contiguous().to(device).t()


def make_opts(*, solver="pg", screening=True, screen_every=10, max_iter=100000, eps_gap=1e-6, step=0.0,
              power_iters=0, t: torch.Tensor | None = None, history=0, stream=None,
              profile=False, iter_precision="f64", graph=False,
              theta_star: torch.Tensor | None = None, t_choice="given", fidelity="ls",
              deterministic=True, huber_delta=0.0) -> tuple[Opts, Any]:
    lib = load()
    o = Opts()
    lib.bxs_default_opts(C.byref(o))
    o.solver = {"pg": BXS_PG, "cd": BXS_CD, "cp": BXS_CP}[solver] if isinstance(solver, str) else int(solver)
    o.screening = 1 if screening else 0
    o.screen_every = int(screen_every)
    o.max_iter = int(max_iter)
    o.eps_gap = float(eps_gap)
    o.step = float(step)
    o.power_iters = int(power_iters)
    o.t = _ptr(t)
    o.stream = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    o.profile = 1 if profile else 0
    o.iter_precision = {"f64": 0, "bf16x3": 1}[iter_precision] if isinstance(iter_precision, str) else int(iter_precision)
    o.graph = 1 if graph else 0
    o.theta_star = _ptr(theta_star)
    o.t_choice = T_CHOICES[t_choice] if isinstance(t_choice, str) else int(t_choice)
    o.fidelity = {"ls": 0, "huber": 1}[fidelity] if isinstance(fidelity, str) else int(fidelity)
    o.huber_delta = float(huber_delta)
    o.deterministic = 1 if deterministic else 0
    hist = None
    if history:
        hist = (PassRecord * int(history))()
        o.history = C.cast(hist, C.POINTER(PassRecord))
        o.history_cap = int(history)
    return o, hist


def _info_dict(info: Info, hist=None, n_hist=0) -> dict:
    d = {f: getattr(info, f) for f, _ in Info._fields_}
    d["status_name"] = STATUS_NAMES.get(info.status, str(info.status))
    if hist is not None:
        d["history"] = [{f: getattr(hist[k], f) for f, _ in PassRecord._fields_} for k in range(n_hist)]
    return d


def _raise(lib, status):
    msg = lib.bxs_last_error().decode()
    raise BoxscreenError(status, msg)


def workspace_bytes(m: int, n: int, opts: Opts) -> int:
    lib = load()
    b = C.c_size_t(0)
    st = lib.bxs_workspace_size(int(m), int(n), C.byref(opts), C.byref(b))
    if st != BXS_OK:
        _raise(lib, st)
    return int(b.value)


def _run_single(kind, A, y, l, u, x0, kw):
    lib = load()
    m, n, lda, dt = _check_matrix(A)
    dev = A.device
    y = _vec(y, m, "y")
    if kind in ("bvls", "bvls_noalloc"):
        l = _vec(l, n, "l")
        u = _vec(u, n, "u")
    t = _vec(kw.pop("t", None), m, "t")
    if kw.get("theta_star") is not None:
        _vec(kw["theta_star"], m, "theta_star")
    x = torch.zeros(n, dtype=torch.float64, device=dev) if x0 is None else _vec(x0, n, "x0").clone()
    sat = torch.empty(n, dtype=torch.int8, device=dev)
    opts, hist = make_opts(t=t, **kw)
    if kind != "bvls_noalloc":
        wbytes = workspace_bytes(m, n, opts)
        wst = torch.empty(wbytes, dtype=torch.uint8, device=dev)
        opts.workspace = wst.data_ptr()
        opts.workspace_bytes = wbytes
    info = Info()
    if kind in ("bvls", "bvls_noalloc"):
        fn = lib.solve_bvls if kind == "bvls" else lib.solve_bvls_noalloc
        st = fn(m, n, dt, A.data_ptr(), lda, y.data_ptr(), l.data_ptr(), u.data_ptr(),
                x.data_ptr(), sat.data_ptr(), C.byref(opts), C.byref(info))
    else:
        st = lib.solve_nnls(m, n, dt, A.data_ptr(), lda, y.data_ptr(), x.data_ptr(), sat.data_ptr(),
                            C.byref(opts), C.byref(info))
    if st not in (BXS_OK, BXS_MAXITER):
        _raise(lib, st)
    n_hist = min(int(info.passes), int(opts.history_cap)) if hist is not None else 0
    return x, sat, _info_dict(info, hist, n_hist)


def solve_bvls(A, y, l, u, x0=None, **kw):
    """Box-constrained LS via libboxscreen (Alg. 1).  Returns (x, sat, info)."""
    return _run_single("bvls", A, y, l, u, x0, dict(kw))


def solve_bvls_noalloc(A, y, l, u, x0=None, **kw):
    """solve_bvls through the allocation-free entry point: the library's fixed
    device scratch replaces the workspace (only x and sat are allocated here,
    as outputs).  Returns (x, sat, info)."""
    return _run_single("bvls_noalloc", A, y, l, u, x0, dict(kw))


def solve_nnls(A, y, x0=None, **kw):
    """Non-negative LS via libboxscreen (Alg. 2).  Returns (x, sat, info)."""
    return _run_single("nnls", A, y, None, None, x0, dict(kw))


def solve_bvls_varbatch(problems: list[dict], **kw):
    """Uneven batch.  Each problem is a dict with A (column-major GPU tensor),
    y, l, u (GPU float64; l/u may be None), optional x0.  All matrices must
    share one dtype.  Returns (xs, sats, infos, status)."""
    lib = load()
    count = len(problems)
    arr = (Problem * count)()
    xs, sats, keep = [], [], []
    dt0 = None
    ms = (C.c_long * count)()
    ns = (C.c_long * count)()
    for i, p in enumerate(problems):
        m, n, lda, dt = _check_matrix(p["A"])
        if dt0 is None:
            dt0 = dt
        elif dt != dt0:
            raise ValueError("all matrices of a batch must share one dtype")
        y = _vec(p["y"], m, "y")
        l = _vec(p.get("l"), n, "l")
        u = _vec(p.get("u"), n, "u")
        x0 = p.get("x0")
        x = torch.zeros(n, dtype=torch.float64, device=p["A"].device) if x0 is None else _vec(x0, n, "x0").clone()
        sat = torch.empty(n, dtype=torch.int8, device=p["A"].device)
        arr[i] = Problem(m, n, lda, p["A"].data_ptr(), y.data_ptr(), _ptr(l), _ptr(u), x.data_ptr(), sat.data_ptr())
        xs.append(x)
        sats.append(sat)
        keep.append((y, l, u))
        ms[i] = m
        ns[i] = n
    kw = dict(kw)
    kw.pop("history", None)
    opts, _ = make_opts(**kw)
    b = C.c_size_t(0)
    st = lib.bxs_workspace_size_batch(count, ms, ns, C.byref(opts), C.byref(b))
    if st != BXS_OK:
        _raise(lib, st)
    wst = torch.empty(int(b.value), dtype=torch.uint8, device=problems[0]["A"].device)
    opts.workspace = wst.data_ptr()
    opts.workspace_bytes = int(b.value)
    infos = (Info * count)()
    st = lib.solve_bvls_varbatch(count, dt0, arr, C.byref(opts), infos)
    if st not in (BXS_OK, BXS_MAXITER):
        _raise(lib, st)
    return xs, sats, [_info_dict(infos[i]) for i in range(count)], STATUS_NAMES[st]


def version() -> str:
    return load().bxs_version().decode()


def sweep_variants() -> list[dict]:
    """The compiled column-sweep shapes (id, threads per column, groups per
    workgroup, rows per thread, columns per round, row capacity)."""
    lib = load()
    out = []
    for v in range(lib.bxs_num_sweep_variants()):
        a, b, c, d, e = (C.c_int() for _ in range(5))
        cap = C.c_long()
        lib.bxs_sweep_variant_info(v, C.byref(a), C.byref(b), C.byref(c), C.byref(d), C.byref(e), C.byref(cap))
        out.append({"id": v, "tpc": a.value, "ng": b.value, "rows": c.value, "cbi": d.value, "pd": e.value,
                    "capacity": cap.value})
    return out


def row_class(m: int) -> int:
    return load().bxs_row_class(int(m))


def variant_for_rows(m: int) -> int:
    return load().bxs_sweep_variant_for_rows(int(m))


def set_sweep_variant(row_class_: int, variant: int) -> None:
    lib = load()
    st = lib.bxs_set_sweep_variant(int(row_class_), int(variant))
    if st != BXS_OK:
        _raise(lib, st)


def set_group_scale(row_class_: int, scale: float) -> None:
    """Spread the work items of instances of this row class over `scale` x the
    chip's resident workgroups (fewer, longer items for scale < 1)."""
    lib = load()
    st = lib.bxs_set_group_scale(int(row_class_), float(scale))
    if st != BXS_OK:
        _raise(lib, st)


def group_scale(row_class_: int) -> float:
    return float(load().bxs_group_scale(int(row_class_)))


def set_cd_block(enable: bool) -> None:
    """Block-sequential coordinate descent for single problems (default on);
    off runs each sweep in one workgroup."""
    lib = load()
    st = lib.bxs_set_cd_block(1 if enable else 0)
    if st != BXS_OK:
        _raise(lib, st)


def solve_nnls_batched_shared(A, Y, X0=None, **kw):
    """Batched NNLS with one shared matrix.  A (m, n) column-major GPU tensor
    (float32/float64); Y (m, B) column-major float64 GPU tensor (column b is
    right-hand side b).  Returns (X (n, B) column-major float64, sat (n, B)
    int8, infos list)."""
    lib = load()
    m, n, lda, dt = _check_matrix(A)
    if not (Y.is_cuda and Y.dtype == torch.float64 and Y.dim() == 2 and Y.shape[0] == m and Y.stride(0) == 1):
        raise ValueError("Y must be an (m, B) column-major float64 GPU tensor")
    B = Y.shape[1]
    ldy = Y.stride(1) if B > 1 else m
    dev = A.device
    X = torch.zeros((B, n), dtype=torch.float64, device=dev) if X0 is None else X0.t().contiguous().clone()
    sat = torch.empty((B, n), dtype=torch.int8, device=dev)
    t = _vec(kw.pop("t", None), m, "t")
    kw.pop("history", None)
    opts, _ = make_opts(t=t, **kw)
    b = C.c_size_t(0)
    st = lib.bxs_workspace_size_batched(m, n, B, C.byref(opts), C.byref(b))
    if st != BXS_OK:
        _raise(lib, st)
    wst = torch.empty(int(b.value), dtype=torch.uint8, device=dev)
    opts.workspace = wst.data_ptr()
    opts.workspace_bytes = int(b.value)
    infos = (Info * B)()
    st = lib.solve_nnls_batched_shared(m, n, B, dt, A.data_ptr(), lda, Y.data_ptr(), ldy, X.data_ptr(), n,
                                       sat.data_ptr(), n, C.byref(opts), infos)
    if st not in (BXS_OK, BXS_MAXITER):
        _raise(lib, st)
    return X.t(), sat.t(), [_info_dict(infos[i]) for i in range(B)]


def _colmajor64(T: torch.Tensor, rows: int, name: str) -> torch.Tensor:
    if not (T.is_cuda and T.dim() == 2 and T.shape[0] == rows):
        raise ValueError(f"{name} must be a 2-D GPU tensor with {rows} rows")
    return T.to(torch.float64).t().contiguous().t()


def nnls_adjoint(A, Y, X, dX, *, max_iter=10000, tol=1e-12, need_dA=True, need_dl=False, stream=None):
    """Implicit-differentiation adjoint of the batched NNLS map (C ABI
    nnls_adjoint).  A (m, n) column-major GPU tensor; Y (m, B), X (n, B),
    dX (n, B) GPU tensors.  Returns (dY (m, B) float64, dA (m, n) float64 or
    None, cg_iterations, status), and with need_dl=True also dl (n, B)
    float64, the gradient with respect to the lower bounds l = 0."""
    lib = load()
    m, n, lda, dt = _check_matrix(A)
    Y64 = _colmajor64(Y, m, "Y")
    B = Y64.shape[1]
    X64 = _colmajor64(X, n, "X")
    G64 = _colmajor64(dX, n, "dX")
    dY = torch.empty((B, m), dtype=torch.float64, device=A.device).t()
    dA = torch.empty((n, m), dtype=torch.float64, device=A.device).t() if need_dA else None
    dl = torch.empty((B, n), dtype=torch.float64, device=A.device).t() if need_dl else None
    o, _ = make_opts(max_iter=max_iter, eps_gap=tol, stream=stream)
    b = C.c_size_t(0)
    st = lib.bxs_workspace_size_adjoint(m, n, B, C.byref(b))
    if st != BXS_OK:
        _raise(lib, st)
    wst = torch.empty(int(b.value), dtype=torch.uint8, device=A.device)
    o.workspace = wst.data_ptr()
    o.workspace_bytes = int(b.value)
    it = C.c_long(0)
    st = lib.nnls_adjoint(m, n, B, dt, A.data_ptr(), lda, Y64.data_ptr(), m, X64.data_ptr(), n, G64.data_ptr(), n,
                          dY.data_ptr(), m, dA.data_ptr() if dA is not None else None, m,
                          dl.data_ptr() if dl is not None else None, n, C.byref(o), C.byref(it))
    if st not in (BXS_OK, BXS_MAXITER, BXS_SINGULAR):
        _raise(lib, st)
    if need_dl:
        return dY, dA, int(it.value), STATUS_NAMES[st], dl
    return dY, dA, int(it.value), STATUS_NAMES[st]


def bvls_adjoint(A, Y, X, dX, l=None, u=None, *, max_iter=10000, tol=1e-12, need_dA=True, stream=None):
    """Implicit-differentiation adjoint of the batched box-constrained map
    with bounds shared by the right-hand sides (C ABI bvls_adjoint).  l, u:
    (n,) float64 GPU tensors or None (0 and +inf).  Returns (dY, dA or None,
    dl, du, cg_iterations, status), every gradient float64."""
    lib = load()
    m, n, lda, dt = _check_matrix(A)
    Y64 = _colmajor64(Y, m, "Y")
    B = Y64.shape[1]
    X64 = _colmajor64(X, n, "X")
    G64 = _colmajor64(dX, n, "dX")
    lv = _vec(l, n, "l") if l is not None else None
    uv = _vec(u, n, "u") if u is not None else None
    dY = torch.empty((B, m), dtype=torch.float64, device=A.device).t()
    dA = torch.empty((n, m), dtype=torch.float64, device=A.device).t() if need_dA else None
    dl = torch.empty((B, n), dtype=torch.float64, device=A.device).t()
    du = torch.empty((B, n), dtype=torch.float64, device=A.device).t()
    o, _ = make_opts(max_iter=max_iter, eps_gap=tol, stream=stream)
    b = C.c_size_t(0)
    st = lib.bxs_workspace_size_adjoint(m, n, B, C.byref(b))
    if st != BXS_OK:
        _raise(lib, st)
    wst = torch.empty(int(b.value), dtype=torch.uint8, device=A.device)
    o.workspace = wst.data_ptr()
    o.workspace_bytes = int(b.value)
    it = C.c_long(0)
    st = lib.bvls_adjoint(m, n, B, dt, A.data_ptr(), lda, Y64.data_ptr(), m, X64.data_ptr(), n,
                          _ptr(lv), _ptr(uv), G64.data_ptr(), n, dY.data_ptr(), m,
                          dA.data_ptr() if dA is not None else None, m, dl.data_ptr(), n, du.data_ptr(), n,
                          C.byref(o), C.byref(it))
    if st not in (BXS_OK, BXS_MAXITER, BXS_SINGULAR):
        _raise(lib, st)
    return dY, dA, dl, du, int(it.value), STATUS_NAMES[st]
