"""Differentiable batched NNLS layer: X = argmin_{X >= 0} 1/2 ||A X - Y||_F^2.

Forward: solve_nnls_batched_shared (projected gradient with Gap-safe
screening, certified gap per column).  Backward: nnls_adjoint (implicit
differentiation on each column's free set).  Both run in libboxscreen.so; this
module only converts tensor layouts and dtypes around the two calls.
"""
from __future__ import annotations

import warnings

import torch

from . import native


class InexactGradientWarning(UserWarning):
    """The forward solve did not reach its gap tolerance on some column, or
    the adjoint solve broke down or did not converge: the gradients of those
    columns are not the derivative of the exact solution map (a broken-down
    column contributes zero)."""


def _report(policy: str, msg: str):
    if policy == "raise":
        raise native.BoxscreenError(native.BXS_MAXITER, msg)
    if policy == "warn":
        warnings.warn(msg, InexactGradientWarning, stacklevel=3)


class _NNLSLayer(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, Y, t, opts, adj_opts, stats, policy):
        Ac = A.detach().t().contiguous().t()            # column-major copy
        Y64 = Y.detach().to(torch.float64).t().contiguous().t()
        X, sat, infos = native.solve_nnls_batched_shared(Ac, Y64, t=t, **opts)
        ctx.save_for_backward(Ac, Y64, X)
        ctx.adj_opts = adj_opts
        ctx.stats = stats
        ctx.policy = policy
        # a gradient is only the derivative of the solution map at an optimum
        ctx.unconverged = sum(1 for i in infos if i["status_name"] != "ok")
        if stats is not None:
            stats["forward"] = infos
        return X.to(Y.dtype)

    @staticmethod
    def backward(ctx, gX):
        Ac, Y64, X = ctx.saved_tensors
        need_dA = ctx.needs_input_grad[0]
        dY, dA, iters, status = native.nnls_adjoint(Ac, Y64, X, gX.to(torch.float64), need_dA=need_dA,
                                                    **ctx.adj_opts)
        if ctx.stats is not None:
            ctx.stats["cg_iters"] = iters
            ctx.stats["cg_status"] = status
        problems = []
        if ctx.unconverged:
            problems.append(f"{ctx.unconverged} of {X.shape[1]} forward columns did not reach the gap tolerance")
        if status != "ok":
            problems.append(f"the adjoint returned '{status}' (a singular column gets zero gradient)")
        if problems:
            _report(ctx.policy, "nnls_layer gradients are not exact: " + "; ".join(problems))
        gA = dA.to(Ac.dtype) if (need_dA and dA is not None) else None
        gY = dY.to(gX.dtype) if ctx.needs_input_grad[1] else None
        return gA, gY, None, None, None, None, None


def nnls_layer(A: torch.Tensor, Y: torch.Tensor, t: torch.Tensor | None = None, *,
               eps_gap: float = 1e-8, max_iter: int = 100000, screen_every: int = 10,
               iter_precision: str = "f64", step: float = 0.0, cg_max_iter: int = 10000,
               cg_tol: float = 1e-12, stats: dict | None = None, on_inexact: str = "warn") -> torch.Tensor:
    """Non-negative least-squares layer on the GPU.

    A (m, n) float32/float64, Y (m, B): column b of the result solves
    min_{x >= 0} 1/2 ||A x - Y[:, b]||^2.  t (m,) float64 is the dual
    translation direction (default -1, valid for non-negative A; for a signed
    A supply a direction with A^T t < 0).  If ``stats`` is a dict it receives
    the per-column forward infos ("forward": status, certified gap, iterations)
    and, after backward, the CG iteration count and status ("cg_iters",
    "cg_status": "ok", "maxiter" or "singular").

    ``on_inexact`` says what backward does when some forward column stopped
    at max_iter before its gap tolerance, or the adjoint reports a singular
    free set or an unconverged CG: "warn" (InexactGradientWarning, the
    default), "raise" (BoxscreenError) or "ignore"."""
    if on_inexact not in ("warn", "raise", "ignore"):
        raise ValueError("on_inexact must be 'warn', 'raise' or 'ignore'")
    opts = dict(eps_gap=eps_gap, max_iter=max_iter, screen_every=screen_every, iter_precision=iter_precision,
                step=step)
    adj = dict(max_iter=cg_max_iter, tol=cg_tol)
    return _NNLSLayer.apply(A, Y, t, opts, adj, stats, on_inexact)
