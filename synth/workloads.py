"""Seeded problem generators.

Every generator draws from ``numpy.random.Generator(PCG64(SeedSequence(
[2202, 7258, cfg, rep, *extra])))`` so that an instance can be regenerated on
any host from its integers alone.  Draw order is fixed: the matrix first (drawn
row-major), then the saturation pattern / support, then the values, then noise.

Matrices are returned column-major (``numpy`` Fortran order, shape (m, n)):
column j is contiguous, which is the layout the GPU kernels read.  "Unit-l2
columns" means the columns are normalised in FP64 *before* rounding to the
storage dtype; the problem that every solver then solves is the one defined by
the rounded matrix promoted back to FP64 (promotion is exact).

The ``planted_*`` generators build an instance whose exact optimum is known by
construction from the first-order optimality conditions of the box-constrained
problem (Sec. 3.2, eqs. optimality1-2): pick the free set F, pick a residual
orthogonal to the columns of A_F, and place every other coordinate on the bound
that the sign of its correlation with that residual dictates.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Problem", "rng_for", "unit_columns",
    "c1_nnls", "c1_companion", "c2_bvls", "c2_planted",
    "c3_shared", "c4_sizes", "c4_instance", "c4_planted_instance", "c5_layer",
    "tiny_bvls", "tiny_nnls", "planted_bvls", "orthonormal_bvls",
    "table1_nnls", "table2_bvls", "fig1_bvls", "interior_direction",
]


@dataclass
class Problem:
    """One box-constrained least-squares instance.

    A      (m, n) column-major, storage dtype (float64 / float32)
    y      (m,)   float64
    l, u   (n,)   float64, u may hold +inf (non-negative / mixed problems)
    x_true (n,)   float64 or None: the vector y was generated from, or the
                  exact optimum for planted instances (``exact=True``)
    """
    A: np.ndarray
    y: np.ndarray
    l: np.ndarray
    u: np.ndarray
    x_true: np.ndarray | None = None
    exact: bool = False
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return self.A.shape[0]

    @property
    def n(self) -> int:
        return self.A.shape[1]

    def A64(self) -> np.ndarray:
        """The problem's matrix promoted to FP64 (exact for FP32 storage)."""
        return np.asfortranarray(self.A, dtype=np.float64)


def rng_for(cfg: int, rep: int = 0, *extra: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(
        np.random.SeedSequence([2202, 7258, int(cfg), int(rep), *map(int, extra)])))


def unit_columns(A: np.ndarray) -> np.ndarray:
    """Scale every column to unit Euclidean norm (FP64)."""
    A = np.asarray(A, dtype=np.float64)
    nrm = np.sqrt(np.einsum("ij,ij->j", A, A))
    nrm[nrm == 0.0] = 1.0
    return A / nrm


def _colmajor(A: np.ndarray, dtype) -> np.ndarray:
    return np.asfortranarray(np.asarray(A, dtype=dtype))


def _gaussian(rng, m, n):
    return rng.standard_normal((m, n))


# --------------------------------------------------------------------------
# C1: NNLS, 200x500, Gaussian unit columns, FP64, 10% support, noise 0.01
# --------------------------------------------------------------------------
def c1_nnls(rep: int = 0, m: int = 200, n: int = 500, nonneg_matrix: bool = False) -> Problem:
    """NNLS instance: A with i.i.d. N(0,1) entries (or |N(0,1)| when
    ``nonneg_matrix``) and unit-l2 columns, x* with 10% nonzeros drawn as
    |N(0,1)|, y = A x* + N(0, 0.01^2)."""
    cfg = 11 if nonneg_matrix else 1
    rng = rng_for(cfg, rep)
    G = _gaussian(rng, m, n)
    if nonneg_matrix:
        G = np.abs(G)
    A = _colmajor(unit_columns(G), np.float64)
    k = int(round(0.10 * n))
    supp = rng.choice(n, size=k, replace=False)
    x = np.zeros(n)
    x[supp] = np.abs(rng.standard_normal(k))
    y = A @ x + 0.01 * rng.standard_normal(m)
    return Problem(A, y, np.zeros(n), np.full(n, np.inf), x, False,
                   {"name": "c1-nn" if nonneg_matrix else "c1", "kind": "nnls"})


def c1_companion(rep: int = 0, m: int = 200, n: int = 500) -> Problem:
    """C1's shape with a non-negative matrix (the paper's NNLS regime,
    Sec. 5: A >= 0 so that t = -1 lies in Int(F_D), Prop. 2 case 3)."""
    return c1_nnls(rep, m, n, nonneg_matrix=True)


# --------------------------------------------------------------------------
# C2: BVLS, 4000x16000, Gaussian unit columns, FP32 storage
# --------------------------------------------------------------------------
def c2_bvls(rep: int = 0, m: int = 4000, n: int = 16000, dtype=np.float32,
            sat_frac: float = 0.4, noise: float = 0.01) -> Problem:
    """BVLS instance: unit-column Gaussian A, l_j ~ U[-1,0], u_j ~ U[0,1],
    40% of x* on a bound (half lower, half upper), the rest U(l_j, u_j),
    y = A x* + N(0, noise^2)."""
    rng = rng_for(2, rep)
    A = _colmajor(unit_columns(_gaussian(rng, m, n)), dtype)
    l = -rng.random(n)
    u = rng.random(n)
    ns = int(round(sat_frac * n))
    perm = rng.permutation(n)
    lo, hi, fr = perm[: ns // 2], perm[ns // 2: ns], perm[ns:]
    x = np.empty(n)
    x[lo] = l[lo]
    x[hi] = u[hi]
    x[fr] = l[fr] + (u[fr] - l[fr]) * rng.random(fr.size)
    y = A.astype(np.float64) @ x + noise * rng.standard_normal(m)
    return Problem(A, y, l, u, x, False, {"name": "c2", "kind": "bvls"})


def planted_bvls(A: np.ndarray, l: np.ndarray, u: np.ndarray, n_free: int,
                 theta_scale: float, rng: np.random.Generator):
    """Planted optimum for min 1/2||Ax-y||^2 s.t. l<=x<=u.

    F (|F| = n_free < m) is drawn uniformly; theta* is a Gaussian vector made
    orthogonal to range(A_F) (so a_j^T theta* = 0 on F); coordinates outside F
    sit at l_j where a_j^T theta* < 0 and at u_j where it is > 0; x*_F is
    drawn inside the box; y = A x* + theta*.  These are exactly the optimality
    conditions of the problem with theta* = y - A x*, so x* is an optimum and
    theta* the unique dual optimum.  Returns (y, x*, theta*, F)."""
    A64 = np.asarray(A, dtype=np.float64)
    m, n = A64.shape
    if not (0 <= n_free < m):
        raise ValueError("planted instance needs |F| < m")
    perm = rng.permutation(n)
    F = np.sort(perm[:n_free])
    th0 = theta_scale * rng.standard_normal(m)
    if n_free > 0:
        Q, _ = np.linalg.qr(A64[:, F])
        th = th0 - Q @ (Q.T @ th0)
        th = th - Q @ (Q.T @ th)          # second projection: re-orthogonalise
    else:
        th = th0
    g = A64.T @ th
    x = np.where(g < 0, l, u)
    if np.any(~np.isfinite(x)):
        raise ValueError("planted BVLS needs finite bounds off the free set")
    x[F] = l[F] + (u[F] - l[F]) * (0.05 + 0.9 * rng.random(F.size))
    y = A64 @ x + th
    return y, x, th, F


def c2_planted(rep: int = 0, m: int = 4000, n: int = 16000, dtype=np.float32,
               free_frac_of_m: float = 0.4) -> Problem:
    """Non-degenerate companion of C2 (same shape, dtype, bounds law): a
    planted optimum with |F| = 0.4 m free coordinates, every other coordinate
    on a bound, and ||theta*|| ~ 0.01 sqrt(m) (noise-sized residual)."""
    rng = rng_for(12, rep)
    A = _colmajor(unit_columns(_gaussian(rng, m, n)), dtype)
    l = -rng.random(n)
    u = rng.random(n)
    y, x, th, F = planted_bvls(A, l, u, int(round(free_frac_of_m * m)), 0.01, rng)
    return Problem(A, y, l, u, x, True, {"name": "c2-pl", "kind": "bvls", "theta": th, "F": F})


# --------------------------------------------------------------------------
# C3: batched NNLS sharing A (1024x4096, U[0,1] unit columns), 8192 RHS
# --------------------------------------------------------------------------
def c3_shared(rep: int = 0, m: int = 1024, n: int = 4096, B: int = 8192,
              support_frac: float = 0.05, noise: float = 0.005):
    """Returns (A float32 (m,n) column-major, Y float64 (m,B) column-major,
    Xtrue float32 (n,B))."""
    rng = rng_for(3, rep)
    A = _colmajor(unit_columns(rng.random((m, n))), np.float32)
    k = int(round(support_frac * n))
    X = np.zeros((n, B), dtype=np.float64)
    for b in range(B):
        s = rng.choice(n, size=k, replace=False)
        X[s, b] = np.abs(rng.standard_normal(k))
    Y = A.astype(np.float64) @ X + noise * rng.standard_normal((m, B))
    return A, np.asfortranarray(Y), X


# --------------------------------------------------------------------------
# C4: uneven batch of independent BVLS instances
# --------------------------------------------------------------------------
def c4_sizes(rep: int = 0, count: int = 2048, m_lo: int = 64, m_hi: int = 2048,
             r_lo: float = 2.0, r_hi: float = 8.0):
    """m_i = round(exp(U[ln m_lo, ln m_hi])), n_i = round(m_i exp(U[ln r_lo, ln r_hi]))."""
    rng = rng_for(4, rep)
    m = np.rint(np.exp(rng.uniform(math.log(m_lo), math.log(m_hi), count))).astype(np.int64)
    n = np.rint(m * np.exp(rng.uniform(math.log(r_lo), math.log(r_hi), count))).astype(np.int64)
    return m, n


def c4_instance(rep: int, i: int, m: int, n: int, dtype=np.float32,
                sat_frac: float = 0.3) -> Problem:
    """Instance i of the uneven batch: Gaussian unit columns, bounds [0,1],
    30% of x* saturated (half at 0, half at 1), the rest U(0,1), y = A x*
    (no noise).  Seeded per instance so any instance regenerates alone."""
    rng = rng_for(4, rep, i)
    A = _colmajor(unit_columns(_gaussian(rng, m, n)), dtype)
    l = np.zeros(n)
    u = np.ones(n)
    ns = int(round(sat_frac * n))
    perm = rng.permutation(n)
    x = rng.random(n)
    x[perm[: ns // 2]] = 0.0
    x[perm[ns // 2: ns]] = 1.0
    y = A.astype(np.float64) @ x
    return Problem(A, y, l, u, x, False, {"name": f"c4[{i}]", "kind": "bvls"})


def c4_planted_instance(rep: int, i: int, m: int, n: int, dtype=np.float32,
                        free_frac_of_m: float = 0.4) -> Problem:
    """Non-degenerate companion of C4 instance i: planted, |F| = 0.4 m,
    ||theta*|| ~ 0.01 sqrt(m), bounds [0,1]."""
    rng = rng_for(14, rep, i)
    A = _colmajor(unit_columns(_gaussian(rng, m, n)), dtype)
    l = np.zeros(n)
    u = np.ones(n)
    y, x, th, F = planted_bvls(A, l, u, int(round(free_frac_of_m * m)), 0.01, rng)
    return Problem(A, y, l, u, x, True, {"name": f"c4-pl[{i}]", "kind": "bvls"})


# --------------------------------------------------------------------------
# C5: differentiable NNLS layer
# --------------------------------------------------------------------------
def c5_layer(rep: int = 0, m: int = 512, n: int = 1024, B: int = 512, target_frac: float = 0.1):
    """Returns (A float64 (m,n) N(0,1) *unnormalised*, Y (m,B) U[0,1],
    T (n,B) targets 10%-sparse |N(0,1)|)."""
    rng = rng_for(5, rep)
    A = np.asfortranarray(rng.standard_normal((m, n)))
    Y = np.asfortranarray(rng.random((m, B)))
    k = int(round(target_frac * n))
    T = np.zeros((n, B))
    for b in range(B):
        s = rng.choice(n, size=k, replace=False)
        T[s, b] = np.abs(rng.standard_normal(k))
    return A, Y, T


# --------------------------------------------------------------------------
# Paper's own synthetic setups (Sec. 5.1)
# --------------------------------------------------------------------------
def table1_nnls(rep: int, m: int, n: int) -> Problem:
    """Table 1 setup: a_ij = |N(0,1)|, x-bar 5% nonzero with |N(0,1)| values,
    y = A x-bar + N(0,1) noise, l = 0, u = +inf."""
    rng = rng_for(21, rep, m, n)
    A = _colmajor(np.abs(_gaussian(rng, m, n)), np.float64)
    k = max(1, int(round(0.05 * n)))
    x = np.zeros(n)
    s = rng.choice(n, size=k, replace=False)
    x[s] = np.abs(rng.standard_normal(k))
    y = A @ x + rng.standard_normal(m)
    return Problem(A, y, np.zeros(n), np.full(n, np.inf), x, False, {"name": "table1", "kind": "nnls"})


def table2_bvls(rep: int, m: int, n: int) -> Problem:
    """Table 2 setup: as Table 1 but x-bar_j ~ U(0,1) on the support and
    bounds l = 0, u = 1."""
    rng = rng_for(22, rep, m, n)
    A = _colmajor(np.abs(_gaussian(rng, m, n)), np.float64)
    k = max(1, int(round(0.05 * n)))
    x = np.zeros(n)
    s = rng.choice(n, size=k, replace=False)
    x[s] = rng.random(k)
    y = A @ x + rng.standard_normal(m)
    return Problem(A, y, np.zeros(n), np.ones(n), x, False, {"name": "table2", "kind": "bvls"})


def huber_bvls(rep: int, m: int, n: int, dtype=np.float64, frac_out: float = 0.1) -> Problem:
    """Input for the Huber fidelity (a fidelity with a 1-Lipschitz gradient,
    eq. GAP_Safe_sph with alpha = 1): a tall matrix with N(0,1) entries
    scaled to unit columns, x-bar ~ U(-3, 3) against the box [-1, 1] (so many
    coordinates of the optimum sit on a bound), y = A x-bar + N(0, 0.05^2)
    noise, and a fraction frac_out of the rows shifted by +-U(2, 5) (gross
    outliers, the residuals the Huber function caps)."""
    rng = rng_for(71, rep, m, n)
    A = _colmajor(unit_columns(_gaussian(rng, m, n)), dtype)
    x = rng.uniform(-3.0, 3.0, n)
    y = np.asarray(A, dtype=np.float64) @ x + 0.05 * rng.standard_normal(m)
    k = int(frac_out * m)
    idx = rng.choice(m, k, replace=False)
    y[idx] += rng.choice([-1.0, 1.0], k) * rng.uniform(2.0, 5.0, k)
    return Problem(A, y, -np.ones(n), np.ones(n), None, False, {"name": "huber", "kind": "bvls"})


def fig1_bvls(rep: int, m: int, n: int, b: float, dtype=np.float64) -> Problem:
    """The saturation-ratio experiment of Sec. 5.1 (Fig. 1): a_ij ~ N(0,1)
    (columns not normalised), y_i ~ N(0,1) drawn independently of A, box
    b [-1, 1]; a smaller b saturates more coordinates of the optimum.  The
    matrix and y depend on (rep, m, n) only, so every b shares them."""
    rng = rng_for(31, rep, m, n)
    A = _colmajor(_gaussian(rng, m, n), dtype)
    y = rng.standard_normal(m)
    return Problem(A, y, np.full(n, -float(b)), np.full(n, float(b)), None, False,
                   {"name": f"fig1[b={b}]", "kind": "bvls"})


# --------------------------------------------------------------------------
# Tiny instances for exhaustive checks
# --------------------------------------------------------------------------
def tiny_bvls(seed: int, m: int, n: int, scale: float = 2.0) -> Problem:
    """Small dense BVLS with l ~ U[-1,0], u ~ U[0,1] and y scaled so that a
    good share of coordinates saturate."""
    rng = rng_for(31, seed, m, n)
    A = _colmajor(rng.standard_normal((m, n)), np.float64)
    l = -rng.random(n)
    u = rng.random(n)
    y = scale * rng.standard_normal(m)
    return Problem(A, y, l, u, None, False, {"name": "tiny-bvls", "kind": "bvls"})


def tiny_nnls(seed: int, m: int, n: int, nonneg_matrix: bool = True) -> Problem:
    rng = rng_for(32, seed, m, n)
    G = rng.standard_normal((m, n))
    if nonneg_matrix:
        G = np.abs(G)
    A = _colmajor(G, np.float64)
    y = rng.standard_normal(m) + (A @ np.abs(rng.standard_normal(n))) * 0.3
    return Problem(A, y, np.zeros(n), np.full(n, np.inf), None, False, {"name": "tiny-nnls", "kind": "nnls"})


def orthonormal_bvls(seed: int, m: int, n: int) -> Problem:
    """A with orthonormal columns (A^T A = I, Prop. 2 case 2 geometry)."""
    rng = rng_for(33, seed, m, n)
    Q, _ = np.linalg.qr(rng.standard_normal((m, n)))
    A = _colmajor(Q, np.float64)
    l = -rng.random(n)
    u = rng.random(n)
    y = 1.5 * rng.standard_normal(m)
    return Problem(A, y, l, u, None, False, {"name": "orth-bvls", "kind": "bvls"})


# --------------------------------------------------------------------------
# Translation direction for signed matrices (an input of the NNLS solver)
# --------------------------------------------------------------------------
def interior_direction(A: np.ndarray, margin_floor: float = 1e-9):
    """A direction t with A^T t < 0 (t in Int(F_D) for NNLS, Sec. 4.2
    eq. interior_FD), found by the linear program
        max s  s.t.  A^T w + s <= 0,  -1 <= w_i <= 1,  s <= 1
    (SciPy HiGHS).  Returns t scaled so that max_j a_j^T t = -1, or None when
    no such direction exists (0 in conv{a_j}, Remark 4)."""
    from scipy.optimize import linprog
    A64 = np.asarray(A, dtype=np.float64)
    m, n = A64.shape
    c = np.zeros(m + 1)
    c[-1] = -1.0
    A_ub = np.hstack([A64.T, np.ones((n, 1))])
    b_ub = np.zeros(n)
    bounds = [(-1.0, 1.0)] * m + [(None, 1.0)]
    res = linprog(c, A_ub=A_ub, b_ub=b_ub, bounds=bounds, method="highs")
    if res.status != 0 or -res.fun <= margin_floor:
        return None
    t = res.x[:m]
    w = A64.T @ t
    if not np.all(w < 0):
        return None
    return t / (-np.max(w))
