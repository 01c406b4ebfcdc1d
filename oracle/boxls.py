"""Plain FP64 reference for box-constrained least squares with Gap-safe screening.

TEST INFRASTRUCTURE ONLY (see the package docstring): never imported by the
product path.

Problem (Sec. 2, eq. LR, with the least-squares fidelity of Sec. 5):
    minimise  P(x) = sum_i f([Ax]_i; y_i),  f(z; y) = 1/2 (z - y)^2,
    subject to l <= x <= u,   l finite, u_j in R or +inf.
Non-negative LS is l = 0, u = +inf; bounded-variable LS has every u_j finite.

A second fidelity with a Lipschitz gradient, the case of eq. GAP_Safe_sph
with alpha = 1 / L (Sec. 3.3): the Huber function of the residual,
    f(z; y) = h_delta(y - z),  h_delta(s) = s^2 / 2 for |s| <= delta,
                                          delta |s| - delta^2 / 2 otherwise,
whose derivative psi_delta(s) = clip(s, -delta, delta) is 1-Lipschitz, so
alpha = 1 as for LS.  The keyword ``delta`` selects it; delta = +inf is LS.

Conventions: A is an (m, n) array (any memory order), vectors are 1-D FP64
arrays, J_inf = {j : u_j = +inf}.  For the negative and positive parts we use
[z]^- = min(0, z) and [z]^+ = max(0, z) (Sec. 1, Notations).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

INF = math.inf


# ---------------------------------------------------------------------------
# Objectives (Sec. 2 eq. LR; Sec. 3.1 eqs. Dual_obj and Dual_set; Sec. 5)
# ---------------------------------------------------------------------------
def huber(s, delta=INF):
    """h_delta(s) entrywise: s^2 / 2 for |s| <= delta, delta |s| - delta^2 / 2
    beyond (delta = +inf: s^2 / 2)."""
    s = np.asarray(s, dtype=np.float64)
    a = np.abs(s)
    out = 0.5 * s * s
    big = a > delta
    if np.any(big):
        out = np.where(big, 0.0, out)
        out[big] = delta * a[big] - 0.5 * delta * delta
    return out


def huber_grad(s, delta=INF):
    """psi_delta(s) = h_delta'(s) = clip(s, -delta, delta)."""
    return np.clip(np.asarray(s, dtype=np.float64), -delta, delta)


def huber_conj(v, delta=INF):
    """h_delta*(v) = v^2 / 2 for |v| <= delta, +inf otherwise (entrywise)."""
    v = np.asarray(v, dtype=np.float64)
    return np.where(np.abs(v) <= delta, 0.5 * v * v, INF)


def primal(A, y, x, delta=INF) -> float:
    """P(x) = sum_i f([Ax]_i; y_i): 1/2 ||Ax - y||^2 for LS (eq. LR with the
    LS fidelity of Sec. 5), sum_i h_delta(y_i - [Ax]_i) for the Huber one."""
    r = y - np.asarray(A, dtype=np.float64) @ x
    if not math.isfinite(delta):
        return 0.5 * float(r @ r)
    return float(np.sum(huber(r, delta)))


def fconj(v, y, delta=INF):
    """Fenchel conjugate of f(.; y) = h_delta(y - .), entrywise:
    f*(v; y) = sup_z v z - h_delta(y - z) = v y + h_delta*(-v); for LS
    (delta = +inf) this is 1/2 ((y + v)^2 - y^2) (Sec. 5)."""
    if not math.isfinite(delta):
        return 0.5 * ((y + v) ** 2 - y ** 2)
    return v * y + huber_conj(-v, delta)


def dual(A, y, l, u, theta, delta=INF) -> float:
    """Dual objective, eq. Dual_obj (Sec. 3.1):
    D(theta) = - sum_i f*(-theta_i; y_i) - sum_j l_j [A^T theta]^-_j
               - sum_{j not in J_inf} u_j [A^T theta]^+_j.
    Evaluated as written; feasibility (eq. Dual_set, and |theta_i| <= delta
    for the Huber fidelity, where f* is finite) is a separate check."""
    A = np.asarray(A, dtype=np.float64)
    c = A.T @ theta
    fin = np.isfinite(u)
    val = -float(np.sum(fconj(-theta, y, delta)))
    val -= float(np.sum(l * np.minimum(c, 0.0)))
    val -= float(np.sum(u[fin] * np.maximum(c[fin], 0.0)))
    return val


def dual_feasible(A, u, theta, tol: float = 0.0) -> bool:
    """Membership in F_D, eq. Dual_set: a_j^T theta <= 0 for every j in J_inf."""
    A = np.asarray(A, dtype=np.float64)
    J = ~np.isfinite(u)
    if not np.any(J):
        return True
    return bool(np.all(A[:, J].T @ theta <= tol))


def duality_gap(A, y, l, u, x, theta, delta=INF) -> float:
    """Gap(x, theta) = P(x) - D(theta), eq. Dual_Gap (Sec. 3.3)."""
    return primal(A, y, x, delta) - dual(A, y, l, u, theta, delta)


def gap_per_coordinate(A, y, l, u, x, theta, delta=INF) -> float:
    """Gap(x, theta) = P(x) - D(theta) (eq. Dual_Gap) rewritten as a sum of
    per-coordinate terms, the form the screening loop evaluates.

    From eq. Dual_obj with f* of Sec. 5,
        -sum_i f*(-theta_i; y_i) = 1/2 ||y||^2 - 1/2 ||y - theta||^2,
    and with rho = y - Ax, y - theta = Ax + (rho - theta), so that
        P(x) - D(theta) = sum_j (-x_j c_j + l_j [c_j]^- + u_j [c_j]^+) + 1/2 ||rho - theta||^2,
    c = A^T theta, the u_j term only for finite u_j (eq. Dual_obj).  Per
    coordinate, for l_j <= x_j <= u_j:
        finite u_j:  (u_j - x_j) [c_j]^+ + (x_j - l_j) [-c_j]^+        (>= 0)
        u_j = +inf:  (x_j - l_j) [-c_j]^+ - x_j [c_j]^+                 (>= 0 on F_D)
    No two large numbers are subtracted, so rounding cannot drive the value
    toward zero while a coordinate inside the box still has a correlation of
    its own (its term keeps the radius sqrt(2 Gap) above that correlation),
    unlike P - D, whose two sides are each of the size of 1/2 ||y||^2.

    Huber fidelity: the same derivation with f*(v; y) = v y + h*(-v) gives
    the row terms h(rho_i) + h*(theta_i) - theta_i rho_i (>= 0, the
    Fenchel-Young gap) in place of 1/2 (rho_i - theta_i)^2.  For |rho_i| <=
    delta they are 1/2 (rho_i - theta_i)^2 again; beyond, with s = sign(rho_i),
    1/2 (theta_i - s delta)^2 + (|rho_i| - delta)(delta - s theta_i), two
    non-negative parts for |theta_i| <= delta (no cancellation either)."""
    A = np.asarray(A, dtype=np.float64)
    rho = y - A @ x
    c = A.T @ theta
    pos, neg = np.maximum(c, 0.0), np.maximum(-c, 0.0)
    fin = np.isfinite(u)
    terms = (x - l) * neg
    terms[fin] += (u[fin] - x[fin]) * pos[fin]
    terms[~fin] -= x[~fin] * pos[~fin]
    d = rho - theta
    if not math.isfinite(delta):
        return float(np.sum(terms)) + 0.5 * float(d @ d)
    if np.any(np.abs(theta) > delta):
        return INF                                  # theta outside dom h*
    rows = 0.5 * d * d
    out = np.abs(rho) > delta
    if np.any(out):
        sg, th, ar = np.sign(rho[out]), theta[out], np.abs(rho[out])
        rows[out] = 0.5 * (th - sg * delta) ** 2 + (ar - delta) * (delta - sg * th)
    return float(np.sum(terms)) + float(np.sum(rows))


# ---------------------------------------------------------------------------
# Dual points (Sec. 4)
# ---------------------------------------------------------------------------
def residual_dual_point(A, y, x, delta=INF):
    """Theta(x) = -grad F(Ax; y) (eq. BVLR_dual_up, Sec. 4.1): y - Ax for
    the LS fidelity, psi_delta(y - Ax) for the Huber one."""
    r = y - np.asarray(A, dtype=np.float64) @ x
    return r if not math.isfinite(delta) else huber_grad(r, delta)


def translate(A, z, t, J):
    """Dual translation Xi_t(z) = z + (max_{j in J} (a_j^T z)^+ / |a_j^T t|) t
    (eq. BVLR_dual_up2, Sec. 4.2).  J selects the columns whose dual constraint
    is active (J_inf).  Returns (theta, eps)."""
    A = np.asarray(A, dtype=np.float64)
    if not np.any(J):
        return z.copy(), 0.0
    AJ = A[:, J]
    num = np.maximum(AJ.T @ z, 0.0)
    den = np.abs(AJ.T @ t)
    eps = float(np.max(num / den))
    return z + eps * t, eps


def interior_direction_ok(A, u, t) -> bool:
    """t in Int(F_D) (Sec. 4.2, eq. interior_FD): a_j^T t < 0 for every
    j in J_inf."""
    A = np.asarray(A, dtype=np.float64)
    J = ~np.isfinite(u)
    if not np.any(J):
        return True
    return bool(np.all(A[:, J].T @ t < 0.0))


def translation_direction(A, choice: str):
    """Translation directions t for the dual update (Sec. 4.2) computed from A
    (Prop. 2 and the choices compared in Sec. 5.1, Fig. 2), with the columns
    normalised, b_k = a_k / ||a_k||:
      "neg_mean_column":       t = -(1/n) sum_k b_k    (Prop. 2, case 2: a negative
                               combination of the columns of an orthogonal A)
      "neg_most_correlated":   t = -b_+, "neg_least_correlated": t = -b_-, where
                               b_+ (b_-) maximises (minimises) the summed correlation
                               with the other columns, sum_{k != j} b_j^T b_k
                               (Prop. 2, case 4, when that column of A^T A is positive);
      "normal_equations":      Prop. 2, case 1 (rank(A) = n <= m): the solution of
                               A^T t = -1 in the range of A, t = A (A^T A)^{-1} (-1)
                               (unnormalised columns), so that A^T t = -1 exactly;
    ties go to the smallest index.  Returns (t, j) with j = -1 for the mean and
    the normal-equations direction."""
    A = np.asarray(A, dtype=np.float64)
    if choice == "normal_equations":
        m, n = A.shape
        if n > m:
            raise ValueError("Prop. 2, case 1 needs rank(A) = n <= m")
        v = np.linalg.solve(A.T @ A, -np.ones(n))
        return A @ v, -1
    nrm = np.sqrt(np.sum(A * A, axis=0))
    B = A / np.where(nrm > 0, nrm, 1.0)
    if choice == "neg_mean_column":
        return -np.sum(B, axis=1) / A.shape[1], -1
    G = B.T @ B                                    # correlations of the normalised columns
    score = np.sum(G, axis=1) - np.diag(G)         # leave out the k = j term
    if choice == "neg_most_correlated":
        j = int(np.argmax(score))                  # first maximiser: smallest index on ties
    elif choice == "neg_least_correlated":
        j = int(np.argmin(score))
    else:
        raise ValueError(choice)
    return -B[:, j].copy(), j


def dual_point(A, y, u, x, t, delta=INF):
    """The dual update Theta(x) used by the screening loop.

    * No infinite upper bound (BVLR): theta = -grad F(Ax; y) (Sec. 4.1).
    * Otherwise dual translation of y - Ax along t (Sec. 4.2) over J_inf.
    * If t is not in Int(F_D) for this matrix (possible for signed A, where
      Prop. 2 offers no direction), the always-feasible theta = 0 is used
      (D(0) = 0), so the gap equals P(x) and nothing can be screened.
    * Huber fidelity with some u_j = +inf: theta = 0 as well (a translation
      along t can leave the box |theta_i| <= delta where f* is finite).
    Returns (theta, eps, t_valid)."""
    z = residual_dual_point(A, y, x, delta)
    J = ~np.isfinite(u)
    if not np.any(J):
        return z, 0.0, True
    if math.isfinite(delta) or not interior_direction_ok(A, u, t):
        return np.zeros_like(z), 0.0, False
    theta, eps = translate(A, z, t, J)
    return theta, eps, True


# ---------------------------------------------------------------------------
# Gap-safe sphere and rule (Sec. 3.3, eqs. GAP_Safe_sph and safe_rule)
# ---------------------------------------------------------------------------
def safe_radius(gap: float, alpha: float = 1.0) -> float:
    """r = sqrt(2 Gap / alpha) (eq. GAP_Safe_sph); alpha = 1 for LS since f''=1.
    A gap that rounds below zero is taken as zero.  Plain FP64 without
    rounding margins."""
    return math.sqrt(2.0 * max(gap, 0.0) / alpha)


def safe_rule(A, theta, radius, u):
    """eq. safe_rule: a_j^T theta < -r ||a_j||  =>  x*_j = l_j ;
                      a_j^T theta >  r ||a_j||  =>  x*_j = u_j (u_j finite).
    Returns boolean masks (lower, upper)."""
    A = np.asarray(A, dtype=np.float64)
    c = A.T @ theta
    nrm = np.sqrt(np.sum(A * A, axis=0))
    lower = c < -radius * nrm
    upper = (c > radius * nrm) & np.isfinite(u)
    return lower, upper


# ---------------------------------------------------------------------------
# Primal solvers (Sec. 5: projected gradient [Polyak 2015]; coordinate
# descent [Franc et al. 2005]).  Neither algorithm is printed in the paper.
# ---------------------------------------------------------------------------
def project(x, l, u):
    """Euclidean projection on the box [l, u]."""
    return np.minimum(np.maximum(x, l), u)


def pg_step(A, y, l, u, x, eta, delta=INF):
    """One projected-gradient step x <- Pi_[l,u](x - eta grad P(x)) with
    grad P(x) = -A^T (y - Ax) (eq. grad, Sec. 4.1), -A^T psi_delta(y - Ax)
    for the Huber fidelity."""
    A = np.asarray(A, dtype=np.float64)
    r = y - A @ x
    g = A.T @ (r if not math.isfinite(delta) else huber_grad(r, delta))
    return project(x + eta * g, l, u)


def cp_step(A, y, l, u, x, v, tau, sigma, delta=INF):
    """One Chambolle-Pock primal-dual iteration (Chambolle & Pock 2011, the
    paper's second BVLS solver in Sec. 5) on min_x F(Ax) + G(x) with
    F(z) = 1/2 ||z - y||^2 and G the indicator of [l, u], in the order primal
    step, extrapolation, dual step:
        x+ = Pi_[l,u](x - tau A^T v)
        xb = 2 x+ - x
        v+ = prox_{sigma F*}(v + sigma A xb) = (v + sigma (A xb - y)) / (1 + sigma)
    since F*(v) = 1/2 ||v||^2 + v^T y.  Converges for tau sigma ||A||_2^2 < 1;
    at a saddle point v = A x* - y, the negated dual optimum of eq. Dual_obj.
    Huber fidelity, F(z) = sum_i h_delta(z_i - y_i): F*(v) = v^T y +
    sum_i h_delta*(v_i) adds the box |v_i| <= delta to the same separable
    quadratic, so its prox is the same point clipped to [-delta, delta].
    Returns (x+, v+)."""
    A = np.asarray(A, dtype=np.float64)
    xn = project(x - tau * (A.T @ v), l, u)
    xb = 2.0 * xn - x
    vn = (v + sigma * (A @ xb - y)) / (1.0 + sigma)
    if math.isfinite(delta):
        vn = np.clip(vn, -delta, delta)
    return xn, vn


def cd_sweep(A, y, l, u, x):
    """One cyclic sweep of exact coordinate minimisation, j = 0..n-1 in order:
    x_j <- Pi_[l_j,u_j](x_j + a_j^T r / ||a_j||^2), r <- r - delta_j a_j,
    with r = y - Ax kept current.  Zero columns are skipped (P does not depend
    on those coordinates)."""
    A = np.asarray(A, dtype=np.float64)
    x = x.copy()
    r = y - A @ x
    for j in range(A.shape[1]):
        a = A[:, j]
        d = float(a @ a)
        if d == 0.0:
            continue
        xj = min(max(x[j] + float(a @ r) / d, l[j]), u[j])
        delta = xj - x[j]
        if delta != 0.0:
            x[j] = xj
            r -= delta * a
    return x


def lipschitz(A) -> float:
    """L = ||A||_2^2, the Lipschitz constant of grad P (largest singular value
    squared, from an SVD)."""
    return float(np.linalg.norm(np.asarray(A, dtype=np.float64), 2) ** 2)


def lipschitz_power(A, iters: int = 100, seed: int = 0) -> float:
    """Power-iteration estimate of ||A||_2^2 (lower bound) for matrices too
    large for an SVD."""
    A = np.asarray(A, dtype=np.float64)
    v = np.random.default_rng(seed).standard_normal(A.shape[1])
    v /= np.linalg.norm(v)
    lam = 0.0
    for _ in range(iters):
        w = A.T @ (A @ v)
        lam = float(np.linalg.norm(w))
        v = w / lam
    return lam


def lipschitz_lanczos(A, steps: int, u0) -> float:
    """Lanczos estimate of ||A||_2^2 from the unit vector u0 / ||u0|| in R^m:
    the largest eigenvalue of the steps x steps tridiagonal matrix T that the
    three-term Lanczos recurrence builds for M = A A^T (Golub & Van Loan,
    Matrix Computations, Sec. 10.1):
        w = M q_k,  alpha_k = q_k^T w,  w -= alpha_k q_k + beta_{k-1} q_{k-1},
        beta_k = ||w||,  q_{k+1} = w / beta_k  (0 once beta_k = 0).
    It is a Rayleigh-Ritz value of M, hence at most ||A||_2^2, and it is exact
    once the Krylov space is invariant.  (The step rule eta = 1 / L of the PG
    solver needs only an estimate of L; this is the estimate the GPU library
    makes, written plainly.)"""
    A = np.asarray(A, dtype=np.float64)
    q = np.asarray(u0, dtype=np.float64)
    q = q / np.linalg.norm(q)
    q_prev = np.zeros_like(q)
    b_prev = 0.0
    alpha, beta = [], []
    for _ in range(steps):
        w = A @ (A.T @ q)
        a = float(q @ w)
        w = w - a * q - b_prev * q_prev
        b = float(np.linalg.norm(w))
        alpha.append(a)
        beta.append(b)
        q_prev, q = q, (w / b if b > 0.0 else np.zeros_like(w))
        b_prev = b
    T = np.diag(alpha) + np.diag(beta[:-1], 1) + np.diag(beta[:-1], -1)
    return float(np.linalg.eigvalsh(T)[-1])


# ---------------------------------------------------------------------------
# The screening loop (Alg. 1; Alg. 2 is its l = 0, u = +inf case)
# ---------------------------------------------------------------------------
@dataclass
class Result:
    x: np.ndarray
    sat: np.ndarray            # int8: -1 screened at l, +1 screened at u, 0 kept
    status: str                # "ok" (gap < eps_gap) or "maxiter"
    gap: float
    primal: float
    dual: float
    radius: float
    iters: int
    passes: int
    t_valid: bool
    history: list = field(default_factory=list)


def oracle_dual_point(A, u, theta_star, t):
    """The dual point of the oracle-dual experiment of Sec. 5.1 (Fig. 3): a
    known dual optimum theta* takes the place of the residual y' - Ax as the
    point the dual update starts from.  For columns with u_j = +inf the
    translation of eq. BVLR_dual_up2 is applied to it as to the residual (it
    only moves theta* when a_j^T theta* > 0, i.e. by its rounding error).
    Returns (theta, eps, t_valid) like dual_point."""
    z = np.asarray(theta_star, dtype=np.float64).copy()
    J = ~np.isfinite(u)
    if not np.any(J):
        return z, 0.0, True
    if not interior_direction_ok(A, u, t):
        return np.zeros_like(z), 0.0, False
    theta, eps = translate(A, z, t, J)
    return theta, eps, True


def solve(A, y, l, u, *, solver: str = "pg", K: int = 10, eps_gap: float = 1e-6,
          max_iter: int = 100000, step: float | None = None, t=None,
          screening: bool = True, x0=None, keep_theta: bool = False, theta_star=None,
          huber_delta: float = INF) -> Result:
    """Alg. 1 with the least-squares simplification of Remark 3.

    Each pass:
      1. K primal iterations (PG steps, or CD sweeps) on the reduced problem
         min 1/2 ||A_P x_P - y'||^2 over the preserved set P (Alg. 1,
         PrimalUpdate on F(A_P . + z)), where y' = y - A_S x_S folds the fixed
         coordinates into the data (Remark 3);
      2. dual update theta = Theta(x) on the reduced problem (Sec. 4);
      3. gap of the reduced problem and safe radius (eqs. Dual_Gap,
         GAP_Safe_sph); the gap is evaluated in its per-coordinate form
         (``gap_per_coordinate``), which equals P - D but has no cancellation,
         so the rule stays meaningful down to FP64's rounding floor (with
         P - D, rounding noise of the size u * 1/2||y||^2 can replace the gap
         once the true gap is that small, and a radius built on noise screens
         free coordinates);
      4. stop if the gap is below eps_gap (the returned x is the one whose gap
         was just measured);
      5. otherwise (screening on) apply the safe rule on P, fix the screened
         coordinates at their bound, fold them into y' and remove them from P.

    ``screening=False`` is the unscreened baseline: the same iterations and the
    same gap evaluation for stopping, but step 5 is skipped.
    ``step`` defaults to 1/||A||_2^2 (PG); for Chambolle-Pock (solver "cp",
    Sec. 5's primal-dual BVLS solver, ``cp_step``) it is tau = sigma, default
    1/(1.05 ||A||_2); its dual iterate v is kept across screening passes (it
    lives in R^m, which the reduction does not change), while the dual point
    of the screening test is the residual one of Sec. 4 as for every solver.
    ``t`` defaults to -1 (Sec. 5).
    ``keep_theta`` stores each pass's dual point, iterate and preserved set in
    the history (for the safe-sphere checks).
    ``theta_star`` (a known dual optimum) replaces the dual update by
    ``oracle_dual_point`` at every pass: the experiment of Sec. 5.1 that
    measures how much screening the dual update leaves undone (Fig. 3).
    ``huber_delta`` (finite) selects the Huber fidelity (module docstring)
    with the PG or CP solver: its gradient (PG) or dual prox (CP), dual
    point, objectives and gap; the radius keeps alpha = 1."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    y = np.asarray(y, dtype=np.float64)
    l = np.asarray(l, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    t = -np.ones(m) if t is None else np.asarray(t, dtype=np.float64)
    if solver not in ("pg", "cd", "cp"):
        raise ValueError(solver)
    hd = float(huber_delta)
    if math.isfinite(hd) and (solver == "cd" or theta_star is not None or not hd > 0.0):
        raise ValueError("the Huber fidelity runs with the PG and CP solvers and the usual dual update, delta > 0")
    if solver == "cp":
        # tau = sigma = step, default 1 / (1.05 ||A||_2): tau sigma ||A||^2 < 1
        eta = (1.0 / (1.05 * np.sqrt(lipschitz(A)))) if step is None else float(step)
    else:
        eta = (1.0 / lipschitz(A)) if step is None else float(step)
    x = project(np.zeros(n) if x0 is None else np.asarray(x0, dtype=np.float64), l, u)
    # Chambolle-Pock dual iterate: the dual step from x0 with v = 0
    v = eta * (A @ x - y) / (1.0 + eta) if solver == "cp" else None
    if v is not None and math.isfinite(hd):
        v = np.clip(v, -hd, hd)
    sat = np.zeros(n, dtype=np.int8)
    P = np.arange(n)
    yp = y.copy()
    iters = passes = 0
    hist = []
    status = "maxiter"
    gap = prim = dl = rad = float("nan")
    t_valid = True
    while True:
        AP, lP, uP = A[:, P], l[P], u[P]
        xP = x[P]
        kk = min(K, max_iter - iters)
        for _ in range(kk):
            if solver == "pg":
                xP = pg_step(AP, yp, lP, uP, xP, eta, hd)
            elif solver == "cd":
                xP = cd_sweep(AP, yp, lP, uP, xP)
            else:
                xP, v = cp_step(AP, yp, lP, uP, xP, v, eta, eta, hd)
        iters += kk
        x[P] = xP
        if theta_star is None:
            theta, eps, t_valid = dual_point(AP, yp, uP, xP, t, hd)
        else:
            theta, eps, t_valid = oracle_dual_point(AP, uP, theta_star, t)
        prim = primal(AP, yp, xP, hd)
        dl = dual(AP, yp, lP, uP, theta, hd)
        gap = gap_per_coordinate(AP, yp, lP, uP, xP, theta, hd)
        rad = safe_radius(gap)
        passes += 1
        hist.append({"iters": iters, "gap": gap, "gap_pd": prim - dl, "radius": rad, "n_active": int(P.size),
                     "eps": eps, "primal": prim, "t_valid": t_valid})
        if keep_theta:
            hist[-1]["theta"] = theta.copy()
            hist[-1]["x"] = x.copy()
            hist[-1]["active"] = P.copy()
        if gap < eps_gap:
            status = "ok"
            break
        if iters >= max_iter:
            break
        if screening and P.size:
            lo, hi = safe_rule(AP, theta, rad, uP)
            S = lo | hi
            if np.any(S):
                x[P[lo]] = l[P[lo]]
                x[P[hi]] = u[P[hi]]
                sat[P[lo]] = -1
                sat[P[hi]] = 1
                yp = yp - A[:, P[S]] @ x[P[S]]
                P = P[~S]
    return Result(x, sat, status, gap, prim, dl, rad, iters, passes, t_valid, hist)


# ---------------------------------------------------------------------------
# Exact optima and optimality checks (Sec. 3.2, eqs. optimality1-2; App. C)
# ---------------------------------------------------------------------------
def kkt_violation(A, y, l, u, x, delta=INF) -> float:
    """Largest violation of the optimality conditions eqs. optimality1-2 at x
    with theta = -grad F(Ax; y) (y - Ax for LS, psi_delta(y - Ax) for Huber):
    |a_j^T theta| on free coordinates, (a_j^T theta)^+ at lower bounds,
    (-a_j^T theta)^+ at upper bounds, plus box infeasibility."""
    A = np.asarray(A, dtype=np.float64)
    g = A.T @ residual_dual_point(A, y, x, delta)
    at_l = x <= l
    at_u = (x >= u) & np.isfinite(u)
    free = ~(at_l | at_u)
    v = 0.0
    if np.any(free):
        v = max(v, float(np.max(np.abs(g[free]))))
    if np.any(at_l):
        v = max(v, float(np.max(np.maximum(g[at_l], 0.0))))
    if np.any(at_u):
        v = max(v, float(np.max(np.maximum(-g[at_u], 0.0))))
    v = max(v, float(np.max(np.maximum(l - x, 0.0), initial=0.0)))
    v = max(v, float(np.max(np.maximum(x - u, 0.0), initial=0.0)))
    return v


def polish(A, y, l, u, x):
    """Exact optimum from an approximate one: keep the saturation pattern of x
    (coordinates exactly on a bound), solve the unconstrained least squares on
    the free set F for the folded data y - A_S x_S, and accept the result when
    it lies strictly inside the box on F and satisfies the sign conditions of
    eq. optimality2 on the saturated set.  Returns (x_exact, accepted)."""
    A = np.asarray(A, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64).copy()
    F = (x > l) & (x < u)
    S = ~F
    yF = y - A[:, S] @ x[S]
    if np.any(F):
        sol, *_ = np.linalg.lstsq(A[:, F], yF, rcond=None)
        x[F] = sol
    ok = bool(np.all(x[F] > l[F]) and np.all(x[F] < u[F]))
    g = A.T @ (y - A @ x)
    scale = 1e-9 * max(1.0, float(np.max(np.abs(g), initial=0.0)))
    at_l = S & (x <= l)
    at_u = S & (x >= u)
    ok = ok and bool(np.all(g[at_l] <= scale)) and bool(np.all(g[at_u] >= -scale))
    return x, ok
