/*
 * boxscreen.h -- C ABI of the gfx950 (MI355X) Gap-safe screening library for
 * box-constrained least squares:
 *
 *     minimise  P(x) = 1/2 ||A x - y||^2   subject to   l <= x <= u,
 *
 * the least-squares instance (Sec. 5) of the box-constrained linear regression
 * problem eq. LR (Sec. 2) of Dantas, Soubies and Fevotte, "Accelerating
 * Non-Negative and Bounded-Variable Linear Regression Algorithms with Safe
 * Screening" (arXiv:2202.07258).  l is finite; u_j may be +INFINITY (the
 * non-negative case l = 0, u = +inf and mixed constraints are covered).
 *
 * Every solver runs the dynamic screening loop of Alg. 1 (Alg. 2 for NNLS):
 * a few primal iterations on the preserved set, a dual point built from the
 * residual (dual scaling for finite boxes, Sec. 4.1; dual translation along t
 * for columns with u_j = +inf, Sec. 4.2), the duality gap (eq. Dual_Gap), the
 * Gap-safe radius (eq. GAP_Safe_sph), the saturation test (eq. safe_rule),
 * and removal of the screened columns, until the gap is below eps_gap.
 *
 * Conventions shared by every entry point
 *  - All array arguments are DEVICE pointers on the current HIP device, owned
 *    by the caller.  The library never frees caller memory.  Inputs (A, y, l,
 *    u, t) are read only; x, sat and explicit outputs are written.
 *  - A is column-major: element (i, j) is at A[i + j*lda], lda >= m.  Its
 *    element type is given by a_dtype; the problem solved is the one defined
 *    by the stored values (FP32 storage is promoted exactly to FP64).
 *  - Vectors are FP64 unless stated otherwise.  Every matrix-vector product
 *    accumulates in FP64; the gap, dual point and screening test are FP64 and
 *    carry an explicit rounding margin, so a screened coordinate is provably
 *    saturated at the optimum of the stored problem.
 *  - Work is enqueued on opts->stream (NULL: the default stream).  A call
 *    returns after the solve has finished and info has been filled.
 *  - Errors are reported by the return code; no exception crosses the ABI.
 *    Argument and shape checks happen before any launch.  Checks that need the
 *    device data (non-finite values, l > u) run on the device before the
 *    first iteration: a failing problem does not iterate, the call returns
 *    the error once every other problem of the call has finished, and x and
 *    sat are unspecified.  bxs_last_error() describes the last
 *    failure of the calling thread.
 *  - Calls are not re-entrant on the same workspace; distinct calls with
 *    distinct workspaces may run concurrently on different streams.
 */
#ifndef BOXSCREEN_H
#define BOXSCREEN_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BXS_OK            = 0,  /* gap < eps_gap reached                              */
    BXS_ERR_ARG       = 1,  /* NULL pointer, bad enum or option value              */
    BXS_ERR_SHAPE     = 2,  /* m, n < 1, lda < m, or m above the supported maximum */
    BXS_ERR_NONFINITE = 3,  /* NaN/Inf in A, y, x0, t, or NaN in l/u               */
    BXS_ERR_BOUNDS    = 4,  /* l_j = -inf, u_j = -inf or l_j > u_j                 */
    BXS_ERR_DEVICE    = 5,  /* HIP runtime error (message in bxs_last_error)       */
    BXS_ERR_NOMEM     = 6,  /* workspace too small or allocation failure           */
    BXS_MAXITER       = 7,  /* max_iter reached first: x = last iterate, info set  */
    BXS_SINGULAR      = 8   /* adjoint: a free-set normal matrix is singular       */
} bxs_status;

/* projected gradient / cyclic coordinate descent / Chambolle-Pock primal-dual
 * (Sec. 5: x+ = Pi(x - tau A^T v), v+ = (v + sigma (A (2 x+ - x) - y)) / (1 + sigma),
 * tau = sigma = opts->step or 1 / (1.05 sqrt(L_est)); the screening test uses
 * the residual dual point of Sec. 4 like the other solvers) */
typedef enum { BXS_PG = 0, BXS_CD = 1, BXS_CP = 2 } bxs_solver;
/* Data-fidelity term f of eq. LR.  BXS_FID_LS: f(z; y) = 1/2 (z - y)^2.
 * BXS_FID_HUBER: f(z; y) = h(y - z) with h(s) = s^2/2 for |s| <= delta and
 * delta |s| - delta^2/2 beyond (delta = opts->huber_delta), a fidelity whose
 * gradient is 1-Lipschitz, so eq. GAP_Safe_sph keeps alpha = 1 (Sec. 3.3).
 * Its dual update (Sec. 4.1) is theta = clip(y' - Ax, -delta, delta), which
 * lies where f* is finite; the PG gradient is -A^T theta, and the
 * Chambolle-Pock dual step is the least-squares one clipped to
 * [-delta, delta] (the prox of the Huber F*).  It runs with the PG and CP
 * solvers of solve_bvls, solve_nnls, solve_bvls_varbatch and
 * solve_bvls_noalloc, without opts->theta_star (not with CD, whose exact
 * coordinate step has no closed form for it).  A preserved column with
 * u_j = +inf makes the pass use theta = 0 (no translation: it could leave the
 * box |theta_i| <= delta), so such problems are solved but not screened
 * (info.t_valid = 0).  Fidelities that need the local strong-concavity bounds
 * Sec. 3.3 mentions (KL, beta-divergences) are not built. */
typedef enum { BXS_FID_LS = 0, BXS_FID_HUBER = 1 } bxs_fidelity;
/* Storage type of A.  Every element is promoted exactly to FP64 before it is
 * used, so the problem solved is the one the stored values define; BXS_BF16
 * (bfloat16: 8-bit significand) halves the bytes of FP32 storage for the
 * single-problem and uneven-batch solvers (not the shared-matrix solver). */
typedef enum { BXS_F64 = 0, BXS_F32 = 1, BXS_BF16 = 2 } bxs_dtype;
/* Arithmetic of the primal iterations of the batched shared-matrix solver
 * (the certification pass is FP64 in both cases). */
typedef enum { BXS_ITER_F64 = 0, BXS_ITER_BF16X3 = 1 } bxs_iter_precision;

/* Translation direction t of the dual update for u_j = +inf columns
 * (Sec. 4.2), computed by the library from A (Prop. 2 and the choices of
 * Sec. 5.1, Fig. 2); columns are taken normalised, a_k / ||a_k||:
 *   BXS_T_GIVEN                 opts->t, or -1 when it is NULL (Prop. 2, case 3)
 *   BXS_T_NEG_MEAN_COLUMN       t = -(1/n) sum_k a_k / ||a_k||   (case 2 for orthogonal A)
 *   BXS_T_NEG_MOST_CORRELATED   t = -a_+ / ||a_+||, a_+ the column whose summed correlation
 *                               sum_{k != j} a_j^T a_k / (||a_j|| ||a_k||) with the others is
 *                               largest (case 4 when that column of A^T A is positive)
 *   BXS_T_NEG_LEAST_CORRELATED  t = -a_- / ||a_-||, the smallest summed correlation
 *   BXS_T_NORMAL_EQUATIONS      t = A v with A^T A v = -1, so A^T t = -1 (case 1, rank(A) = n <= m;
 *                               BXS_ERR_ARG when n > m); v by FP64 conjugate gradients to a
 *                               residual norm of 1e-11 sqrt(n) or 2000 iterations, with a host
 *                               synchronisation every 16 iterations (setup only)
 * Ties go to the smallest column index.  The computed t goes through the
 * same interior check as a given one (info.t_valid).  solve_bvls / solve_nnls
 * / solve_bvls_noalloc only (one problem per call). */
typedef enum { BXS_T_GIVEN = 0, BXS_T_NEG_MEAN_COLUMN = 1, BXS_T_NEG_MOST_CORRELATED = 2,
               BXS_T_NEG_LEAST_CORRELATED = 3, BXS_T_NORMAL_EQUATIONS = 4 } bxs_translation;

/* Largest number of rows a single instance may have. */
#define BXS_MAX_ROWS 16384

/* One record per screening pass (Alg. 1 loop body), written to opts->history. */
typedef struct {
    long   iters;      /* primal iterations (PG steps or CD sweeps) done before this pass */
    long   n_active;   /* size of the preserved set when the gap was evaluated            */
    double gap;        /* certified duality gap of the reduced problem (eq. Dual_Gap)      */
    double radius;     /* Gap-safe radius sqrt(2 gap) (eq. GAP_Safe_sph, alpha = 1)         */
    double eps;        /* dual-translation coefficient (0 for finite boxes)                 */
    double primal;     /* 1/2 ||r||^2 of the reduced problem                                */
    long   n_screened; /* coordinates removed by this pass                                   */
} bxs_pass_record;

typedef struct {
    int     solver;          /* bxs_solver                                                      */
    int     screening;       /* 1: dynamic Gap-safe screening; 0: unscreened baseline (same
                                iterations and gap evaluations, nothing is removed)            */
    int     screen_every;    /* K >= 1: PG steps or CD sweeps between two screening passes     */
    long    max_iter;        /* >= 1: iteration budget (PG steps or CD sweeps)                  */
    double  eps_gap;         /* >= 0: absolute gap tolerance (stop when gap < eps_gap)          */
    double  step;            /* PG step; <= 0 selects 1/(1.05 L_est), see power_iters          */
    int     power_iters;     /* steps of the estimate of L = ||A||_2^2 when step <= 0, at most 64.
                                solve_bvls / solve_nnls / solve_bvls_varbatch: Lanczos steps on
                                A A^T, each one pass over A (<= 0: 8); the step is
                                1 / (1.05 L_est) with L_est the largest Ritz value (<= L).
                                Batched shared-matrix solver: power iterations (<= 0: 20).    */
    const double* t;         /* device m-vector translation direction for the u_j = +inf
                                columns (Sec. 4.2); NULL means t = -1 (Sec. 5).  If some
                                preserved column has a_j^T t >= 0 the library falls back to
                                the always-feasible dual point theta = 0 and nothing is
                                screened (info.t_valid = 0).                                    */
    void*   stream;          /* hipStream_t or NULL                                             */
    void*   workspace;       /* device scratch of workspace_bytes, or NULL (library allocates) */
    size_t  workspace_bytes;
    bxs_pass_record* history;/* HOST array for per-pass records, or NULL                        */
    long    history_cap;     /* capacity of history (records beyond it are dropped)            */
    int     profile;         /* 1: time every primal-iteration sweep with HIP events recorded on
                                opts->stream and report it in info.sweep_ms / sweep_launches  */
    int     iter_precision;  /* bxs_iter_precision; only the batched shared-matrix solver      */
    int     graph;           /* 1: every regular screening pass (K iterations, not the last) of
                                solve_bvls / solve_nnls / solve_bvls_varbatch is captured once
                                as a HIP graph and replayed; 0 (default): direct launches,
                                which measured faster on MI355X (ROCm 7.2) for every size
                                tried, since the host stays a pass ahead of the device.
                                Profile mode always launches directly.                         */
    const double* theta_star;/* device m-vector or NULL.  Diagnostic of the dual update's
                                headroom (Sec. 5.1, oracle dual point of Fig. 3): every screening
                                pass of solve_bvls / solve_nnls / solve_bvls_varbatch uses this
                                vector, a known dual optimum y - A x* (translated along t for
                                u_j = +inf columns if rounding left some a_j^T theta_star > 0),
                                in place of the point built from the residual; the gap, radius
                                and test are computed from it with the same rounding margins.
                                Screening stays safe for any dual-feasible vector; a vector that
                                is not the optimum only weakens it.  Same vector for every
                                problem of a batch.                                           */
    int     t_choice;        /* bxs_translation; with BXS_T_GIVEN opts->t applies, otherwise
                                opts->t must be NULL                                           */
    int     fidelity;        /* bxs_fidelity                                                    */
    int     deterministic;   /* 0 or 1.  Every reduction of the library sums in a fixed order
                                and no kernel uses floating-point atomics, so results repeat
                                bit for bit on the same device, inputs and options either way */
    double  huber_delta;     /* delta > 0, finite, of BXS_FID_HUBER; ignored for BXS_FID_LS    */
} bxs_opts;

typedef struct {
    int    status;      /* bxs_status of this instance                                  */
    int    t_valid;     /* 0 when the theta = 0 fallback was used                       */
    long   iters;       /* primal iterations done                                       */
    long   passes;      /* screening passes done                                        */
    long   n_active;    /* preserved coordinates at exit                                */
    long   n_lower;     /* coordinates screened at l                                    */
    long   n_upper;     /* coordinates screened at u                                    */
    double gap;         /* certified gap at the returned x                              */
    double primal;      /* P(x) at the returned x: 1/2 ||Ax - y||^2, or the Huber sum    */
    double radius;      /* last safe radius                                             */
    double eps;         /* last translation coefficient                                 */
    double step;        /* PG step used                                                 */
    double lipschitz;   /* estimate of ||A||_2^2, a lower bound (0 if step was given)   */
    double ms_setup;    /* device time of the setup phase (column norms, A^T t, L)      */
    double ms_solve;    /* device time of the iterations and screening passes           */
    long   col_iters;   /* sum over primal iterations of the preserved-set size         */
    double sweep_ms;    /* opts->profile: summed duration of the primal-iteration sweep
                           launches (PG: fused A^T r / update / A x, all but the first
                           of each screening pass, which returns at once when the
                           previous pass already took that step; CD: the sweep;
                           batched solver: the pair of iteration GEMMs)               */
    long   sweep_launches; /* opts->profile: number of timed sweep launches             */
    double event_overhead_ms; /* opts->profile: average HIP-event elapsed time around an
                           empty kernel on the same stream (dispatch latency included in
                           every timed launch); measured once per process and device    */
    long   t_column;    /* column whose negative is t (BXS_T_NEG_MOST/LEAST_CORRELATED),
                           else -1                                                      */
    double dual;        /* primal - gap: the dual objective of the last pass (eq. Dual_obj),
                           a certified lower bound of the optimal value                   */
    double max_margin;  /* last pass: rounding margin of a correlation a_j^T theta per unit
                           ||a_j|| (the band inside which no coordinate is screened)       */
    long   n_free;      /* coordinates strictly inside the box at the returned x           */
} bxs_info;

/* Fill *opts with defaults: PG, screening on, K = 10, max_iter = 100000,
 * eps_gap = 1e-6, step from power iteration, t = -1, default stream. */
void bxs_default_opts(bxs_opts* opts);

/* Bytes of device workspace a call with these sizes needs (m, n per instance). */
bxs_status bxs_workspace_size(long m, long n, const bxs_opts* opts, size_t* bytes);
bxs_status bxs_workspace_size_batch(long count, const long* m, const long* n,
                                    const bxs_opts* opts, size_t* bytes);

/* Bounded-variable / mixed LS (Alg. 1).
 *   A    [lda*n] a_dtype, column-major            y [m]
 *   l, u [n] bounds (u_j may be +inf)             x [n] in: start point (clipped
 *   sat  [n] signed char out: -1 screened at l,      to the box), out: solution
 *        +1 screened at u, 0 kept in the preserved set
 *   info host, may be NULL.  Returns BXS_OK, BXS_MAXITER or an error code. */
bxs_status solve_bvls(long m, long n, int a_dtype, const void* A, long lda,
                      const double* y, const double* l, const double* u,
                      double* x, signed char* sat, const bxs_opts* opts, bxs_info* info);

/* Allocation-free variant of solve_bvls, for callers that cannot allocate
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, kernels and results as solve_bvls, but the
 * call makes no device or pinned-host allocation and creates no event or
 * graph: its workspace is a fixed device array of BXS_NOALLOC_SCRATCH_BYTES
 * inside the library (one copy per GPU, held until the process ends), the
 * device tables go up from a fixed host area, and the host waits for each
 * screening pass with a stream synchronisation (one host round trip per
 * pass, so it is slower than solve_bvls on small problems).
 *   - opts->workspace must be NULL, opts->graph and opts->profile 0
 *     (BXS_ERR_ARG otherwise).
 *   - A problem whose workspace (bxs_workspace_size) exceeds
 *     BXS_NOALLOC_SCRATCH_BYTES returns BXS_ERR_NOMEM before any launch.
 *   - Calls share each GPU's array and keep its last contents; every value a
 *     solve reads is written by that solve first.  Calls are serialised
 *     within the process; calls from different processes on one GPU use
 *     different copies.
 *   - info->ms_setup is 0 and info->ms_solve is the host's wall time of the
 *     call. */
#define BXS_NOALLOC_SCRATCH_BYTES (32L << 20)
bxs_status solve_bvls_noalloc(long m, long n, int a_dtype, const void* A, long lda,
                              const double* y, const double* l, const double* u,
                              double* x, signed char* sat, const bxs_opts* opts, bxs_info* info);

/* Non-negative LS (Alg. 2): solve_bvls with l = 0, u = +inf, dual translation
 * along opts->t (default -1, valid for A >= 0 with no zero column, Prop. 2). */
bxs_status solve_nnls(long m, long n, int a_dtype, const void* A, long lda,
                      const double* y, double* x, signed char* sat,
                      const bxs_opts* opts, bxs_info* info);

/* One independent problem of a batch (pointers are device pointers). */
typedef struct {
    long m, n, lda;
    const void* A;       /* column-major, element type a_dtype of the call */
    const double* y;     /* [m]                                            */
    const double* l;     /* [n] or NULL (l = 0)                            */
    const double* u;     /* [n] or NULL (u = +inf)                         */
    double* x;           /* [n] in/out                                     */
    signed char* sat;    /* [n] out                                        */
} bxs_problem;

/* Uneven batch: `count` independent problems of different shapes solved
 * together, every kernel launch covering all unfinished problems.  probs and
 * infos are HOST arrays of length count; infos may be NULL.  opts->history is
 * ignored.  Returns BXS_OK when every problem reached its gap, BXS_MAXITER
 * when at least one did not, or the first error. */
bxs_status solve_bvls_varbatch(long count, int a_dtype, const bxs_problem* probs,
                               const bxs_opts* opts, bxs_info* infos);

/* Kernel-shape tuning.  The column sweeps come in several compiled shapes
 * ("variants": threads per column, column groups per workgroup, rows per
 * thread, columns per round).  Each problem is assigned a row class, the
 * smallest default variant that holds its m rows; bxs_set_sweep_variant
 * selects which variant later calls use for a class (v < 0 restores the
 * default).  These settings are process-wide and must not change while a
 * solve is running; they apply to FP32 and FP64 storage (bfloat16 storage
 * keeps the library's own table).  Used by the autotuner, which times the
 * candidates. */
int        bxs_num_sweep_variants(void);
bxs_status bxs_sweep_variant_info(int v, int* tpc, int* ng, int* rows, int* cbi, int* pd, long* capacity);
int        bxs_row_class(long m);            /* -1 if m > BXS_MAX_ROWS */
int        bxs_sweep_variant_for_rows(long m); /* variant later calls use for m rows, -1 if none */
bxs_status bxs_set_sweep_variant(int row_class, int v);
/* Tuning: the work items of an instance (blocks of preserved columns, one
 * workgroup each, one partial product each) are spread over scale x the
 * chip's resident workgroups, shared among the instances of a call in
 * proportion to m*n.  A smaller scale gives fewer, longer items (less
 * partial-product traffic, less parallelism).  scale in [1/64, 4], default 1;
 * process-wide per row class; set before the solve that should use it.
 * Returns BXS_ERR_ARG for a bad class or scale. */
bxs_status bxs_set_group_scale(int row_class, double scale);
double bxs_group_scale(int row_class);   /* current scale, 0 for a bad class */

/* Coordinate descent of a single problem (solve_bvls / solve_nnls with
 * BXS_CD) runs block-sequentially by default: blocks of 128 preserved
 * coordinates, their correlations A_J^T r over many workgroups, the
 * coordinate updates of the block in order from the Gram block A_J^T A_J
 * (c_p = a_p^T r - sum_{q < p in J} a_p^T a_q delta_q, the same iterates as one
 * coordinate at a time up to rounding), then r -= A_J delta_J.  Its
 * workspace (bxs_workspace_size counts it) adds 2 * 128 doubles per column
 * (the Gram blocks and the cross blocks A_Jk^T A_J(k-1)).  enable = 0 runs
 * every sweep in one workgroup instead, as batches and solve_bvls_noalloc
 * always do.  Process-wide; BXS_ERR_ARG for enable outside {0, 1}. */
bxs_status bxs_set_cd_block(int enable);

/* Batched non-negative LS with one shared matrix (Alg. 2 for every column
 * y_b of Y):  min 1/2 ||A x_b - y_b||^2  s.t. x_b >= 0,  b = 0..B-1.
 * Projected gradient for all right-hand sides at once, the matrix products
 * as GEMMs: FP64 (opts->iter_precision = BXS_ITER_F64) or hand-written
 * gfx950 MFMA GEMMs on bf16 hi/lo splits of the FP32 operands with FP32
 * accumulation and fused residual / projected-step epilogues
 * (BXS_ITER_BF16X3).  Every screen_every iterations an FP64 pass computes
 * the residuals and correlations from the stored matrix, the translated
 * dual point (along opts->t, default -1), the certified gap per right-hand
 * side, the safe radius and the saturation test; right-hand sides whose
 * gap is below eps_gap stop and leave the active set.
 *   A [lda*n] (a_dtype)   Y [ldy*B] FP64   X [ldx*B] FP64 in: x0, out: x
 *   sat [ldsat*B] out (-1 screened at 0, else 0)   infos host [B] or NULL
 * Requires m, n, B >= 1 and lda >= m, ldy >= m, ldx >= n, ldsat >= n. */
bxs_status solve_nnls_batched_shared(long m, long n, long B, int a_dtype, const void* A, long lda,
                                     const double* Y, long ldy, double* X, long ldx,
                                     signed char* sat, long ldsat, const bxs_opts* opts, bxs_info* infos);
bxs_status bxs_workspace_size_batched(long m, long n, long B, const bxs_opts* opts, size_t* bytes);

/* Adjoint of the batched NNLS solution map by implicit differentiation.
 * With F_b = {j : X_jb > 0} the free set of right-hand side b, the optimality
 * conditions (Sec. 3.2, eq. optimality2) give x_F = (A_F^T A_F)^{-1} A_F^T y_b,
 * so for an upstream gradient dL/dX:
 *     v_b = (A_F^T A_F)^{-1} (dL/dx_b)_F   (masked conjugate gradients, FP64)
 *     dL/dY = A V,   dL/dA = (Y - A X) V^T - (dL/dY) X^T   (summed over b)
 *     dL/dl_b = (dL/dx_b - A^T dL/dy_b) on the coordinates at 0
 * Coordinates at 0 are treated as saturated (one-sided derivative where a
 * coordinate is weakly active).  opts->max_iter bounds the CG iterations and
 * opts->eps_gap is the CG tolerance relative to ||(dL/dx_b)_F||.
 *   A [lda*n] (a_dtype)  Y [ldy*B]  X [ldx*B] (forward solution)
 *   dX [ldg*B] in   dY [lddy*B] out   dA [ldda*n] out or NULL
 *   dl [lddl*B] out or NULL: the gradient with respect to the lower bounds
 *        l = 0 of each right-hand side, dL/dl_jb = (dL/dx_b)_j - a_j^T dL/dy_b
 *        where x_jb sits on its bound and 0 on the free set (u = +inf has no
 *        gradient).
 *   cg_iters host out or NULL.  Each right-hand side runs CG until its
 *   residual is below the tolerance, or until it breaks down: p^T A_F^T A_F p
 *   at or below the rounding level 2 gamma_{m+2} ||p||^2 ||A||_F^2 of its
 *   FP64 evaluation (A_F rank deficient, e.g. more free coordinates than
 *   rows, so the forward solution is not an isolated optimum).  The
 *   columns of dY and the terms of dA of a broken-down right-hand side are 0.
 *   Returns BXS_OK; BXS_SINGULAR if at least one column broke down;
 *   BXS_MAXITER if CG did not reach the tolerance for every right-hand side;
 *   or an error code (outputs unset). */
bxs_status nnls_adjoint(long m, long n, long B, int a_dtype, const void* A, long lda,
                        const double* Y, long ldy, const double* X, long ldx,
                        const double* dX, long ldg, double* dY, long lddy, double* dA, long ldda,
                        double* dl, long lddl, const bxs_opts* opts, long* cg_iters);

/* The same adjoint for box constraints shared by the right-hand sides
 * (Sec. 3.2, eq. optimality2 with the free set F_b = {j : l_j < X_jb < u_j};
 * the coordinates on a bound stay there under small perturbations when
 * complementarity is strict):
 *     v_b = (A_F^T A_F)^{-1} (dL/dx_b)_F,  dL/dY = A V,
 *     dL/dA = (Y - A X) V^T - (dL/dY) X^T,
 *     dL/dl_jb = (dL/dx_b - A^T dL/dy_b)_j where X_jb <= l_j, else 0,
 *     dL/du_jb = the same where X_jb >= u_j, else 0.
 *   l, u: device n-vectors or NULL (NULL l: l = 0; NULL u: u = +inf, so
 *   l = u = NULL is nnls_adjoint).  du [lddu*B] out or NULL.  Every other
 *   argument, the CG and the return codes as for nnls_adjoint. */
bxs_status bvls_adjoint(long m, long n, long B, int a_dtype, const void* A, long lda,
                        const double* Y, long ldy, const double* X, long ldx,
                        const double* l, const double* u, const double* dX, long ldg,
                        double* dY, long lddy, double* dA, long ldda, double* dl, long lddl,
                        double* du, long lddu, const bxs_opts* opts, long* cg_iters);
bxs_status bxs_workspace_size_adjoint(long m, long n, long B, size_t* bytes);

/* Thread-local description of the last error (empty string if none). */
const char* bxs_last_error(void);

/* Library version string. */
const char* bxs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BOXSCREEN_H */
