// gfx950 kernels of the boxscreen library: column sweeps (the matrix-vector
// products of the projected-gradient step, the correlations A^T r, the fold of
// screened columns, products with A A^T), their deterministic partial reductions,
// per-column statistics, the screening pass (dual point, gap, safe rule,
// stream compaction) and the coordinate-descent sweep.
//
// Data layout (HBM): A column-major with leading dimension lda; every
// per-column vector (x, l, u, g, w, cn, cn2, sat) is indexed by the ORIGINAL
// column index j; the preserved set is the int32 list idx[0..n_active), kept
// in ascending j.  Removing columns only compacts idx, so A itself is never
// copied: a column stays a contiguous run of m elements and each sweep reads
// it with 16-byte vector loads.
//
// Reductions are deterministic: every sum has a fixed order that depends only
// on the launch configuration, so two runs of the same solve agree bit for bit.
#include "dev_common.h"

namespace bxs {

// ---------------------------------------------------------------------------
// Partial reduction: kRedRows rows x 64 item-groups per workgroup (many
// workgroups even for a few thousand rows), fixed summation order.  Each
// thread issues U independent branch-free global loads (clamped addresses,
// masked in the sum) before adding them in order; the 64 group sums of a row
// are then added by wave shuffles (4 groups per wave) and 16 per-wave sums.
// ---------------------------------------------------------------------------
// The reduced row's update, by mode: r = y' - sum (residual), r2 = y' - sum
// (step taken ahead), y' -= sum and r -= sum2 (fold), r = sum (product with
// A A^T), the Chambolle-Pock dual step v <- (v + sigma (sum - y')) / (1 + sigma)
// with v in r2.
template <int MODE>
__device__ __forceinline__ void reduce_apply(const Inst& I, const State& S, int row, double ypv, double tot,
                                             double tot2)
{
    if constexpr (MODE == kRedResidual) {
        I.r[row] = ypv - tot;
    } else if constexpr (MODE == kRedAhead) {
        I.r2[row] = ypv - tot;
    } else if constexpr (MODE == kRedFold) {
        I.yp[row] = ypv - tot;
        I.r[row] -= tot2;
    } else if constexpr (MODE == kRedCP) {
        // dual step of Chambolle-Pock: prox of sigma F*, F*(v) = 1/2 ||v||^2 + v^T y'
        // (least squares), restricted to |v_i| <= delta for the Huber fidelity,
        // whose prox is the same point clipped (delta = +inf: no clip)
        const double sg = S.step, hub = I.hub;
        I.r2[row] = fmin(fmax((I.r2[row] + sg * (tot - ypv)) / (1.0 + sg), -hub), hub);
    } else {
        I.r[row] = tot;
    }
}

template <int MODE>
__global__ __launch_bounds__(1024)
void k_reduce(const Inst* __restrict__ insts, State* __restrict__ st, const RItem* __restrict__ ritems, int first,
              int single)
{
    constexpr int TG = 1024 / kRedRows, U = 4, NWV = 1024 / 64;
    static_assert(kRedRows == 16, "four item-groups per wave");
    const RItem ri = single ? RItem{0, (int)blockIdx.x} : ritems[blockIdx.x];
    const Inst& I = insts[ri.inst];
    const State& S = st[ri.inst];
    const int rowl = threadIdx.x % kRedRows, tg = threadIdx.x / kRedRows;
    const int row = ri.rb * kRedRows + rowl;
    const int m = I.m;
    const int rowc = (row < m) ? row : m - 1;          // a valid row; its sum is not stored
    // The first round of loads goes out before the instance's state is read:
    // every slot below items_cap is a valid partial (the number in use, T,
    // is never larger; the others are masked below).
    const int Tcap = I.items_cap;
    double v0[U], w0[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int t = tg + u * TG;
        const size_t off = (size_t)((t < Tcap) ? t : 0) * m + rowc;
        v0[u] = gload(I.part + off);
        if (MODE == kRedFold) w0[u] = gload(I.part2 + off);
    }
    const double ypv = (MODE == kRedPow) ? 0.0 : gload(I.yp + rowc);
    if (S.done) return;
    if (MODE == kRedResidual && first && S.ahead) return;
    const int nlist = (MODE == kRedFold) ? S.n_fold : S.n_active;
    const int cb = (MODE == kRedFold) ? S.cb_fold : S.cb;
    const int T = (nlist + cb - 1) / cb;
    double s = 0.0, s2 = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const bool ok = tg + u * TG < T;
        s += ok ? v0[u] : 0.0;
        if (MODE == kRedFold) s2 += ok ? w0[u] : 0.0;
    }
    for (int t0 = tg + TG * U; t0 < T; t0 += TG * U) {
        double v[U], v2[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = t0 + u * TG;
            const size_t off = (size_t)((t < T) ? t : 0) * m + rowc;
            v[u] = gload(I.part + off);
            if (MODE == kRedFold) v2[u] = gload(I.part2 + off);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool ok = t0 + u * TG < T;
            s += ok ? v[u] : 0.0;
            if (MODE == kRedFold) s2 += ok ? v2[u] : 0.0;
        }
    }
    // the wave's four groups of the same row: lanes l, l^16, l^32, l^48
    s += __shfl_xor(s, 16, 64);
    s += __shfl_xor(s, 32, 64);
    if (MODE == kRedFold) {
        s2 += __shfl_xor(s2, 16, 64);
        s2 += __shfl_xor(s2, 32, 64);
    }
    __shared__ double sh[NWV][kRedRows], sh2[(MODE == kRedFold) ? NWV : 1][kRedRows];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane < kRedRows) {
        sh[wave][rowl] = s;
        if (MODE == kRedFold) sh2[wave][rowl] = s2;
    }
    __syncthreads();
    if (tg == 0 && row < m) {
        double tot = 0.0, tot2 = 0.0;
#pragma unroll
        for (int w = 0; w < NWV; ++w) {
            tot += sh[w][rowl];
            if (MODE == kRedFold) tot2 += sh2[w][rowl];
        }
        reduce_apply<MODE>(I, S, row, ypv, tot, tot2);
    }
}

// Partial reduction for instances with at most kRedNarrowMax work items (the
// host puts every row block of such an instance in the narrow list): one
// thread per row, kRedRowsN rows per workgroup, the partials of the row summed
// in item order.  The wide kernel above would spend a 1024-thread workgroup
// on every 16 rows whatever the number of items.
template <int MODE>
__global__ __launch_bounds__(kRedRowsN)
void k_reduce_n(const Inst* __restrict__ insts, State* __restrict__ st, const RItem* __restrict__ ritems, int first)
{
    const RItem ri = ritems[blockIdx.x];
    const Inst& I = insts[ri.inst];
    const State& S = st[ri.inst];
    if (S.done) return;
    if (MODE == kRedResidual && first && S.ahead) return;
    const int m = I.m;
    const int row = ri.rb * kRedRowsN + threadIdx.x;
    if (row >= m) return;
    const int nlist = (MODE == kRedFold) ? S.n_fold : S.n_active;
    const int cb = (MODE == kRedFold) ? S.cb_fold : S.cb;
    const int T = (nlist + cb - 1) / cb;
    const double ypv = (MODE == kRedPow) ? 0.0 : gload(I.yp + row);
    double s = 0.0, s2 = 0.0;
    for (int t = 0; t < T; ++t) {
        s += gload(I.part + (size_t)t * m + row);
        if (MODE == kRedFold) s2 += gload(I.part2 + (size_t)t * m + row);
    }
    reduce_apply<MODE>(I, S, row, ypv, s, s2);
}

// ---------------------------------------------------------------------------
// Setup: copy y, clip x0, identity preserved set, input validation.
// grid (blocks, count), State zeroed by the host beforehand.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256)
void k_init(const Inst* __restrict__ insts, State* __restrict__ st)
{
    const int i = blockIdx.y;
    const Inst& I = insts[i];
    State& S = st[i];
    int err = 0;
    const int stride = gridDim.x * blockDim.x;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < I.m; k += stride) {
        const double yv = I.y[k];
        if (!isfinite(yv)) err |= kErrNonfinite;
        I.yp[k] = yv;
        I.r[k] = 0.0;
        if (I.t && !isfinite(I.t[k])) err |= kErrNonfinite;
        if (I.ts && !isfinite(I.ts[k])) err |= kErrNonfinite;
    }
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < I.n; j += stride) {
        const double lj = lo_of(I.l, j), uj = up_of(I.u, j), xj = I.x[j];
        if (isnan(lj) || isnan(uj) || !isfinite(xj)) err |= kErrNonfinite;
        else if (isinf(lj) || (isinf(uj) && uj < 0) || lj > uj) err |= kErrBounds;
        I.x[j] = fmin(fmax(xj, lj), uj);
        I.idx[j] = j;
        I.sat[j] = 0;
        I.g[j] = 0.0;
    }
    if (err) atomicOr(&S.err, err);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        S.n_active = I.n;
        S.n_fold = 0;
        S.cb = choose_cb(I.n, I.g_target);
        S.cb_fold = kCbMin;
        S.done = 0;
        S.status = BXS_OK;
        S.t_valid = 1;
        S.passes = 0;
        S.ahead = 0;
        S.n_free = 0;
    }
}

// Input validation on the device: an instance whose data failed the checks of
// k_init or k_colstats stops here with the error as its status, so the solve
// needs no host round trip before its first iteration.
__global__ __launch_bounds__(256)
void k_validate(State* __restrict__ st, int* __restrict__ done_counter, int count)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    State& S = st[i];
    if (S.err == 0 || S.done) return;
    S.done = 1;
    S.status = (S.err & kErrNonfinite) ? BXS_ERR_NONFINITE : BXS_ERR_BOUNDS;
    atomicAdd(done_counter, 1);
}

// Copy of the stop counter into host memory (pinned, mapped): the host reads
// it once the pass's completion event has fired.
__global__ __launch_bounds__(64)
void k_publish(const int* __restrict__ src, int* __restrict__ dst)
{
    if (threadIdx.x == 0) dst[0] = src[0];
}

// ---------------------------------------------------------------------------
// Column statistics: rigorous norm bound, sum of squares, w = A^T t, and a
// finiteness check of A.  One wave per column; each lane reads V consecutive
// rows per 16-byte load (V = 1 when the columns are not 16-byte aligned) and
// keeps U loads in flight before using them.
// ---------------------------------------------------------------------------
template <typename TA, int V>
__global__ __launch_bounds__(256)
void k_colstats(const Inst* __restrict__ insts, State* __restrict__ st, const Item* __restrict__ items)
{
    constexpr int U = 8;
    const Item it = items[blockIdx.x];
    const Inst& I = insts[it.inst];
    State& S = st[it.inst];
    const int cb = S.cb;
    const int pos0 = it.t * cb;
    const int pos1 = min(pos0 + cb, I.n);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const TA* __restrict__ A = reinterpret_cast<const TA*>(I.A);
    const double* __restrict__ t = I.t;
    // each of the V chains of a lane adds at most m / (64 V) + 1 terms, then
    // V chains and the 6-level wave butterfly: depth below m / 64 + 8
    const double gm = gamma_k((double)(I.m / 64) + 8.0);
    int err = 0;
    const int m = I.m;
    const double* __restrict__ ts = I.ts;
    for (int j = pos0 + wv; j < pos1; j += 4) {
        const TA* col = A + (long long)j * I.lda;
        double s2[V], sw[V], ss[V];
#pragma unroll
        for (int e = 0; e < V; ++e) { s2[e] = 0.0; sw[e] = 0.0; ss[e] = 0.0; }
        for (int k0 = 0; k0 * 64 * V < m; k0 += U) {
            TA a[U][V];
            double tv[U][V];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int row = ((k0 + u) * 64 + lane) * V;
                load_pack_nb<TA, V>(col, row, m, a[u]);
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    const int rc = (row + e < m) ? row + e : 0;
                    tv[u][e] = t ? gload(t + rc) : -1.0;
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    const bool ok = ((k0 + u) * 64 + lane) * V + e < m;
                    const double av = ok ? (double)a[u][e] : 0.0;
                    if (ok && !isfinite(av)) err = kErrNonfinite;
                    s2[e] = fma(av, av, s2[e]);
                    sw[e] = fma(av, tv[u][e], sw[e]);
                }
            if (ts) {
                // correlations with the given dual optimum (diagnostic mode)
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int e = 0; e < V; ++e) {
                        const int row = ((k0 + u) * 64 + lane) * V + e;
                        const bool ok = row < m;
                        const double av = ok ? (double)a[u][e] : 0.0;
                        ss[e] = fma(av, ok ? ts[row] : 0.0, ss[e]);
                    }
            }
        }
        double s2l = 0.0, swl = 0.0, ssl = 0.0;
#pragma unroll
        for (int e = 0; e < V; ++e) { s2l += s2[e]; swl += sw[e]; ssl += ss[e]; }
        const double s2t = wave_sum(s2l);
        const double swt = wave_sum(swl);
        const double sst = ts ? wave_sum(ssl) : 0.0;
        if (lane == 0) {
            I.cn2[j] = s2t;
            I.cn[j] = sqrt(s2t * (1.0 + gm)) * (1.0 + 2.0 * kUnit);
            I.w[j] = swt;
            if (ts) I.gs[j] = sst;
        }
    }
    if (err) atomicOr(&S.err, err);
}

// ---------------------------------------------------------------------------
// Per-instance scalars: bounds on ||y|| and ||t||, step from the caller, and
// the unit starting vector q_0 of the Lanczos estimate of ||A||_2^2 (when do_pow).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256)
void k_inst_scalars(const Inst* __restrict__ insts, State* __restrict__ st, int do_pow, double user_step)
{
    __shared__ double sh[4];
    const Inst& I = insts[blockIdx.x];
    State& S = st[blockIdx.x];
    const int m = I.m;
    double sy = 0.0, stt = 0.0, su = 0.0, sts = 0.0;
    for (int i = threadIdx.x; i < m; i += 256) {
        const double yv = I.y[i], tv = t_of(I.t, i);
        sy = fma(yv, yv, sy);
        stt = fma(tv, tv, stt);
        if (I.ts) sts = fma(I.ts[i], I.ts[i], sts);
        if (do_pow) {
            // deterministic start: 1 +- 1/4 by a multiplicative hash of the row
            const unsigned h = (unsigned)i * 2654435761u;
            const double v = 1.0 + ((h >> 31) ? 0.25 : -0.25);
            I.r[i] = v;
            su = fma(v, v, su);
        }
    }
    sy = block_sum<256>(sy, sh);
    stt = block_sum<256>(stt, sh);
    su = block_sum<256>(su, sh);
    sts = block_sum<256>(sts, sh);
    if (do_pow) {
        const double inv = 1.0 / sqrt(su);
        double* q0 = I.lz + 2 * I.lz_steps;
        for (int i = threadIdx.x; i < m; i += 256) {
            const double q = I.r[i] * inv;
            I.r[i] = q;
            q0[i] = q;
        }
    }
    if (threadIdx.x == 0) {
        const double gm = gamma_k((double)m + 32.0);
        S.ynorm = sqrt(sy * (1.0 + gm)) * (1.0 + 2.0 * kUnit);
        S.tnorm = sqrt(stt * (1.0 + gm)) * (1.0 + 2.0 * kUnit);
        S.tsnorm = sqrt(sts * (1.0 + gm)) * (1.0 + 2.0 * kUnit);
        if (!do_pow) {
            S.step = user_step;
            S.lipschitz = 0.0;
        }
    }
}

// Largest eigenvalue of the symmetric tridiagonal matrix with diagonal a[0..s)
// and off-diagonal b[0..s-1), by multisection on Sturm counts: each of the
// wave's 64 lanes counts the eigenvalues below its own point of the current
// bracket (signs of the LDL^T pivots), and the bracket shrinks 65-fold per
// round.  Called by one whole wave; every lane returns the same value, the
// upper end of the final bracket.
__device__ double tridiag_max_eig(const double* a, const double* b, int s)
{
    const int lane = threadIdx.x & 63;
    double lo = 0.0, hi = 0.0;
    for (int i = 0; i < s; ++i) {
        const double rad = (i > 0 ? fabs(b[i - 1]) : 0.0) + (i + 1 < s ? fabs(b[i]) : 0.0);
        hi = fmax(hi, a[i] + rad);
        lo = fmin(lo, a[i] - rad);
    }
    hi *= 1.0 + 4.0 * kUnit;
    for (int round = 0; round < 16 && hi - lo > 8.0 * kUnit * fabs(hi); ++round) {
        const double x = lo + (hi - lo) * (double)(lane + 1) / 65.0;
        int below = 0;
        double d = 1.0;
        for (int i = 0; i < s; ++i) {
            d = a[i] - x - (i > 0 ? b[i - 1] * b[i - 1] / d : 0.0);
            if (d == 0.0) d = -1e-300;
            below += d < 0.0;
        }
        // lanes whose point lies above every eigenvalue
        const unsigned long long above = __ballot(below == s);
        const int f = above ? __ffsll((long long)above) - 1 : 64;
        const double xf = (f < 64) ? __shfl(x, f, 64) : hi;
        const double xl = (f > 0) ? __shfl(x, f - 1, 64) : lo;
        hi = xf;
        lo = xl;
    }
    return hi;
}

// One Lanczos step on M = A A^T (three-term recurrence, Golub & Van Loan,
// Matrix Computations, Sec. 10.1).  On entry r = M q_k (column sweep and
// partial reduction of the previous launches), q_k and q_{k-1} in lz:
//   alpha_k = q_k^T r,  w = r - alpha_k q_k - beta_{k-1} q_{k-1},
//   beta_k = ||w||,  q_{k+1} = w / beta_k  (0 if beta_k = 0: the Krylov space
//   is invariant and the remaining steps add zero rows to T).
// After the last step the largest eigenvalue of the tridiagonal T (a
// Rayleigh-Ritz value of M: at most ||A||_2^2 up to rounding, and far closer
// to it than the power iteration with as many products) gives the PG step
// 1 / (1.05 L).  One workgroup per instance.
__global__ __launch_bounds__(1024)
void k_lanczos(const Inst* __restrict__ insts, State* __restrict__ st, int k, int last, int cp)
{
    constexpr int NT = 1024;
    __shared__ double sh[NT / 64];
    const Inst& I = insts[blockIdx.x];
    State& S = st[blockIdx.x];
    const int m = I.m, steps = I.lz_steps;
    double* al = I.lz;
    double* be = I.lz + steps;
    double* qc = I.lz + 2 * steps;
    double* qp = qc + m;
    const int tid = threadIdx.x;
    double a = 0.0;
    for (int i = tid; i < m; i += NT) a = fma(qc[i], I.r[i], a);
    a = block_sum<NT>(a, sh);
    const double bp = (k > 0) ? be[k - 1] : 0.0;
    double ss = 0.0;
    for (int i = tid; i < m; i += NT) {
        double w = fma(-a, qc[i], I.r[i]);
        if (k > 0) w = fma(-bp, qp[i], w);
        I.r[i] = w;
        ss = fma(w, w, ss);
    }
    ss = block_sum<NT>(ss, sh);
    const double b = sqrt(ss);
    const double inv = (b > 0.0) ? 1.0 / b : 0.0;
    for (int i = tid; i < m; i += NT) {
        const double q = I.r[i] * inv;
        qp[i] = qc[i];
        qc[i] = q;
        I.r[i] = q;
    }
    if (tid == 0) {
        al[k] = a;
        be[k] = b;
    }
    if (last) {
        __syncthreads();
        if (tid < 64) {
            const double lam = tridiag_max_eig(al, be, k + 1);
            if (tid == 0) {
                S.lipschitz = lam;
                // PG: 1 / (1.05 L); Chambolle-Pock: tau = sigma = 1 / (1.05 sqrt(L)), tau sigma L < 1
                S.step = (lam > 0.0) ? (cp ? 1.0 / (1.05 * sqrt(lam)) : 1.0 / (1.05 * lam)) : 1.0;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Screening pass (Alg. 1 body after PrimalUpdate), one workgroup per instance.
//
// Inputs: r = y' - A_P x_P (FP64), g_j = a_j^T r for j in P (FP64).
// 1. dual point: theta = r + eps t (Sec. 4.2), eps = max over P with u_j = inf
//    of (g_j)^+ / |a_j^T t|; no such column -> eps = 0 (Sec. 4.1).  If some
//    such column has a_j^T t >= 0 (t not interior) theta = 0 is used.
// 2. gap (eq. Dual_Gap) in per-coordinate form:
//      sum_j (u_j - x_j)[a_j^T theta]^+ + (x_j - l_j)[-a_j^T theta]^+
//      + 1/2 ||theta - (y - Ax)||^2,
//    with theta - (y - Ax) = eps t + (rounding error of r).
// 3. radius sqrt(2 Gap) (eq. GAP_Safe_sph, alpha = 1), test (eq. safe_rule),
//    fix x_S at its bound, list S for the fold, compact P.
// Every floating-point quantity that decides safety is bounded rigorously:
// e_j bounds |computed - exact| of a_j^T theta, delta_r bounds the residual
// error, and each rounded sum, product and square root is pushed outward.
// ---------------------------------------------------------------------------
// SK selects the pass: kScreenLS, kScreenOracleDual (the diagnostic mode
// with a given dual optimum) or kScreenHuber (the Huber fidelity), each its
// own instantiation, so the regular pass carries none of the others'
// registers.
template <int SK>
__device__ __forceinline__ void screen_pass(const Inst* __restrict__ insts, State* __restrict__ st,
                                            int* __restrict__ done_counter, double eps_gap, int screening,
                                            int final_pass, int K, int kk, int ahead)
{
    constexpr bool OD = SK == kScreenOracleDual;
    constexpr int NT = 1024;
    constexpr int E = 4;                       // consecutive preserved positions per thread per chunk
    constexpr int CH = NT * E;
    __shared__ double sh[NT / 64];
    __shared__ int wsum[NT / 64];
    const Inst& I = insts[blockIdx.x];
    State& S = st[blockIdx.x];
    if (S.done) return;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int m = I.m, n = I.n;
    const int nA = S.n_active;
    const int passes = S.passes;
    // every earlier pass ran K primal iterations (all unfinished instances of
    // a call advance together), this one kk: the arguments stay the same for
    // every regular pass, so a pass can be replayed from a captured graph
    const long long iters = (long long)passes * K + kk;
    const double tnorm = S.tnorm;
    const double u1 = kUnit;
    const bool nnls_like = (I.u == nullptr);   // every u_j = +inf
    // diagnostic mode: a given dual optimum ts replaces the residual as the
    // point the dual update starts from (correlations gs_j = a_j^T ts from
    // the setup), so the item partials of the sweep do not apply
    const double* __restrict__ ts = I.ts;
    constexpr bool oracle_dual = OD;

    // ||r||^2 and the per-item quantities written by the correlation sweep
    // (mass, interior flag of t, largest translation ratio, presence of
    // u = +inf columns, gap terms and largest screening score at eps = 0),
    // combined over the workgroup in one reduction
    double a = 0.0, a2 = 0.0;
    for (int i = tid; i < m; i += NT) {
        const double ri = I.r[i];
        a = fma(ri, ri, a);
        if (oracle_dual) {
            const double d = ri - ts[i];
            a2 = fma(d, d, a2);
        }
    }
    // ||r - ts|| bound (diagnostic mode only)
    const double rts = oracle_dual
        ? sqrt(block_sum<NT>(a2, sh) * (1.0 + gamma_k((double)(m / NT) + 24.0))) * (1.0 + 2.0 * u1) : 0.0;
    const int T = (nA + S.cb - 1) / S.cb;
    double red7[7] = {a, 0.0, 0.0, 1.0, 0.0, 0.0, -__builtin_inf()};   // rsq mass gap0 | tv | emax hasinf z0
    for (int t = tid; t < T; t += NT) {
        const double* o = I.iscal + (size_t)t * kItemScalars;
        red7[1] += o[kIsMass];
        red7[2] += o[kIsGap0];
        red7[3] = fmin(red7[3], o[kIsTv]);
        red7[4] = fmax(red7[4], o[kIsEmax]);
        red7[5] = fmax(red7[5], o[kIsHasInf]);
        red7[6] = fmax(red7[6], o[kIsZmax0]);
    }
    {
        __shared__ double sh7[7][NT / 64];
        red7[0] = wave_sum(red7[0]);
        red7[1] = wave_sum(red7[1]);
        red7[2] = wave_sum(red7[2]);
        red7[3] = wave_min(red7[3]);
        red7[4] = wave_max(red7[4]);
        red7[5] = wave_max(red7[5]);
        red7[6] = wave_max(red7[6]);
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < 7; ++k) sh7[k][wave] = red7[k];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            double tot = 0.0;
#pragma unroll
            for (int w = 0; w < NT / 64; ++w) tot += sh7[k][w];
            red7[k] = tot;
        }
        double mn = sh7[3][0], m4 = sh7[4][0], m5 = sh7[5][0], m6 = sh7[6][0];
#pragma unroll
        for (int w = 1; w < NT / 64; ++w) {
            mn = fmin(mn, sh7[3][w]);
            m4 = fmax(m4, sh7[4][w]);
            m5 = fmax(m5, sh7[5][w]);
            m6 = fmax(m6, sh7[6][w]);
        }
        red7[3] = mn; red7[4] = m4; red7[5] = m5; red7[6] = m6;
    }
    const double rsq = red7[0];
    const double rnorm = sqrt(rsq * (1.0 + gamma_k((double)(m / NT) + 24.0))) * (1.0 + 2.0 * u1);
    // error bounds of the correlations g_j (sweep kernels) and of w_j = a_j^T t
    // (column statistics), by Cauchy-Schwarz: sum_i |a_ij v_i| <= ||a_j|| ||v||
    const double gm = gamma_k(kDotDepth);
    const double gw = gamma_k((double)(m / 64) + 8.0);

    // Per-chunk gather of the preserved columns' data: each thread takes E
    // consecutive positions and issues all of its loads before using them.
    struct Col { int j; double g, w, cn, x, l, u; };
    const double* __restrict__ gsrc = oracle_dual ? I.gs : I.g;
    auto gather = [&](int base, Col (&c)[E], bool (&valid)[E]) {
        int jj[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int p = base + tid * E + e;
            valid[e] = p < nA;
            jj[e] = valid[e] ? I.idx[p] : 0;
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int j = jj[e];
            c[e].j = j;
            c[e].g = valid[e] ? gsrc[j] : 0.0;
            c[e].w = valid[e] ? I.w[j] : 0.0;
            c[e].cn = valid[e] ? I.cn[j] : 0.0;
            c[e].x = valid[e] ? (ahead ? I.xs[j] : I.x[j]) : 0.0;
            c[e].l = valid[e] ? lo_of(I.l, j) : 0.0;
            c[e].u = valid[e] ? up_of(I.u, j) : 0.0;
        }
    };

    double tv = red7[3], emax = red7[4];
    const double mass = red7[1], hasinf = red7[5], gap0 = red7[2], z0 = red7[6];
    const bool has_inf = hasinf > 0.5;
    // correlations of the given dual optimum carry the error of their setup
    // dot products (depth m/64 + 8, like w)
    const double e_ts = oracle_dual ? gw * S.tsnorm : 0.0;
    if (oracle_dual && has_inf) {
        // interior check of t and translation coefficient from gs (a plain
        // loop: this diagnostic path keeps no batch of columns in registers)
        double tvl = 1.0, eml = 0.0;
        for (int p = tid; p < nA; p += NT) {
            const int j = I.idx[p];
            if (!isinf(up_of(I.u, j))) continue;
            const double cnj = I.cn[j], wj = I.w[j], gj = I.gs[j];
            const double ewj = gw * cnj * tnorm;
            if (!(wj + ewj < 0.0)) tvl = 0.0;
            else eml = fmax(eml, fmax(gj + cnj * e_ts + 4.0 * u1 * fabs(gj), 0.0) / (-wj - ewj));
        }
        tv = block_min<NT>(tvl, sh);
        emax = block_max<NT>(eml, sh);
    }
    // Huber fidelity: no translation for u_j = +inf columns (theta + eps t
    // could leave the box |theta_i| <= delta where f* is finite), theta = 0
    // instead
    constexpr bool huber = SK == kScreenHuber;
    const double hub = huber ? I.hub : 0.0;
    const bool fallback = has_inf && (!(tv > 0.5) || huber);
    const double eps = (has_inf && !fallback) ? emax * (1.0 + 4.0 * u1) : 0.0;
    const double massall = (mass + S.mass_screened) * (1.0 + gamma_k((double)n + 64.0));
    const double delta_r = gamma_k(2.0 * n + 4.0 * passes + 64.0) * (S.ynorm + 2.0 * massall);

    // a_j^T theta for theta = r + eps t, and its rounding bound
    const double e_g = oracle_dual ? e_ts : gm * rnorm;     // per unit column norm
    auto corr = [&](const Col& c, double& cj, double& ej) {
        cj = fma(eps, c.w, c.g);
        ej = c.cn * (e_g + gw * eps * tnorm) + 4.0 * u1 * (fabs(c.g) + eps * fabs(c.w));
    };

    // Huber fidelity: its primal value sum_i h(r_i), h(s) = s^2 / 2 for
    // |s| <= delta and delta (|s| - delta / 2) beyond (reported, and the gap
    // of the theta = 0 fallback); one more pass over r
    double hsum = 0.0;
    if (huber) {
        double ah = 0.0;
        for (int i = tid; i < m; i += NT) {
            const double ri = I.r[i], ar = fabs(ri);
            ah += (ar <= hub) ? 0.5 * ri * ri : hub * (ar - 0.5 * hub);
        }
        hsum = block_sum<NT>(ah, sh);
    }
    // gap: at eps = 0 the sweep already summed the per-column terms; with a
    // translation the terms change and are summed here in one more pass
    double G, zmax = z0;
    if (fallback && huber) {
        // theta = 0: the gap is P(x) = sum_i h(r_i) at the exact residual
        // r = r~ + e, ||e|| <= delta_r; h is 1-smooth with |h'(r~_i)| <=
        // |r~_i|, so P <= sum h(r~_i) + ||r~|| delta_r + delta_r^2 / 2
        const double hb = hsum * (1.0 + gamma_k((double)(m / NT) + 24.0));
        G = (hb + rnorm * delta_r + 0.5 * delta_r * delta_r) * (1.0 + 4.0 * u1);
    } else if (fallback) {
        const double tt = rnorm + delta_r;
        G = 0.5 * tt * tt * (1.0 + 4.0 * u1);
    } else {
        double gsum = gap0;
        if (eps > 0.0 || oracle_dual) {
            double acc = 0.0, zz = -__builtin_inf();
            for (int base = 0; base < nA; base += CH) {
                Col c[E];
                bool valid[E];
                gather(base, c, valid);
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    if (!valid[e]) continue;
                    double cj, ej;
                    corr(c[e], cj, ej);
                    double term = (c[e].x - c[e].l) * fmax(ej - cj, 0.0);
                    double zs = -(cj + ej);
                    if (!isinf(c[e].u)) {
                        term += (c[e].u - c[e].x) * fmax(cj + ej, 0.0);
                        zs = fmax(zs, cj - ej);
                    }
                    acc += term;
                    if (c[e].cn > 0.0) zz = fmax(zz, zs / c[e].cn);
                }
            }
            gsum = block_sum<NT>(acc, sh);
            zmax = block_max<NT>(zz, sh);
        }
        // || (y' - A x) - theta || <= delta_r + ||r - ts|| + eps ||t||  (ts = r outside the diagnostic mode)
        const double tt = delta_r + rts + eps * tnorm;
        G = (gsum * (1.0 + 3.0 * u1) + 0.5 * tt * tt * (1.0 + 4.0 * u1)) * (1.0 + gamma_k((double)n + 64.0));
    }
    const double rad = sqrt(2.0 * G) * (1.0 + 2.0 * u1);
    const double primal = huber ? hsum : 0.5 * rsq;
    const bool stop = G < eps_gap;
    if (tid == 0) S.col_iters += (long long)nA * kk;

    // the largest screening score bounds every column's test: if it stays
    // below the radius nothing can be screened and the scan is skipped
    const bool none = !(zmax >= rad);
    if (stop || final_pass || !screening || fallback || none) {
        if (tid == 0) {
            if (passes < I.rec_cap) {
                bxs_pass_record& rc = I.rec[passes];
                rc.iters = iters; rc.n_active = nA; rc.gap = G; rc.radius = rad;
                rc.eps = eps; rc.primal = primal; rc.n_screened = 0;
            }
            S.gap = G; S.radius = rad; S.eps = eps; S.primal = primal; S.margin = e_g + gw * eps * tnorm;
            S.t_valid = fallback ? 0 : 1;
            S.passes = passes + 1;
            S.n_fold = 0;
            if (stop || final_pass) {
                S.done = 1;
                S.status = stop ? BXS_OK : BXS_MAXITER;
                S.iters = iters;
                atomicAdd(done_counter, 1);
            }
            S.ahead = (ahead && !(stop || final_pass)) ? 1 : 0;
        }
        if (ahead) {
            if (stop || final_pass) {
                // the result is the iterate the gap was computed at
                for (int p = tid; p < nA; p += NT) {
                    const int j = I.idx[p];
                    I.x[j] = I.xs[j];
                }
            } else {
                // keep the step taken ahead: its residual becomes r
                for (int i = tid; i < m; i += NT) I.r[i] = I.r2[i];
            }
        }
        return;
    }

    // pass 3: safe rule, fix, fold list, in-place compaction of idx.
    // One packed block scan per chunk: low 16 bits count kept columns, high
    // 16 bits screened ones (at most CH = 4096 of each per chunk).
    int out = 0, fout = 0;
    double nlo = 0.0, nhi = 0.0, smass = 0.0;
    for (int base = 0; base < nA; base += CH) {
        Col c[E];
        bool valid[E];
        gather(base, c, valid);
        int flag[E];                           // 0 keep, 1 lower, 2 upper, 3 invalid
        int packed = 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            flag[e] = 3;
            if (!valid[e]) continue;
            double cj, ej;
            corr(c[e], cj, ej);
            const double thr = rad * c[e].cn * (1.0 + 2.0 * u1);
            const bool lower = (cj + ej) < -thr;
            const bool upper = !lower && !isinf(c[e].u) && (cj - ej) > thr;
            flag[e] = lower ? 1 : (upper ? 2 : 0);
            packed += (flag[e] == 0) ? 1 : (1 << 16);
        }
        // inclusive wave scan, then wave offsets through LDS
        int x = packed;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(x, o, 64);
            if (lane >= o) x += t;
        }
        if (lane == 63) wsum[wave] = x;
        __syncthreads();                       // also orders every idx read of this chunk before the writes
        int woff = 0, tot = 0;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) {
            if (w < wave) woff += wsum[w];
            tot += wsum[w];
        }
        const int excl = x - packed + woff;
        int kpos = out + (excl & 0xffff);
        int spos = fout + (excl >> 16);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (flag[e] == 0) {
                I.idx[kpos++] = c[e].j;
            } else if (flag[e] == 1 || flag[e] == 2) {
                const bool lower = flag[e] == 1;
                const double b = lower ? c[e].l : c[e].u;
                I.fidx[spos] = c[e].j;
                I.fval[spos] = b;
                I.fdx[spos] = b - c[e].x;
                ++spos;
                I.x[c[e].j] = b;
                I.sat[c[e].j] = lower ? (signed char)-1 : (signed char)1;
                smass = fma(fabs(b), c[e].cn, smass);
                if (lower) nlo += 1.0; else nhi += 1.0;
            }
        }
        out += tot & 0xffff;
        fout += tot >> 16;
        __syncthreads();                       // wsum reuse
    }
    nlo = block_sum<NT>(nlo, sh);
    nhi = block_sum<NT>(nhi, sh);
    smass = block_sum<NT>(smass, sh);
    if (tid == 0) {
        if (passes < I.rec_cap) {
            bxs_pass_record& rc = I.rec[passes];
            rc.iters = iters; rc.n_active = nA; rc.gap = G; rc.radius = rad;
            rc.eps = eps; rc.primal = primal; rc.n_screened = fout;
        }
        S.gap = G; S.radius = rad; S.eps = eps; S.primal = primal; S.margin = e_g + gw * eps * tnorm;
        S.t_valid = 1;
        S.passes = passes + 1;
        S.n_active = out;
        S.n_fold = fout;
        S.cb = choose_cb(out, I.g_target);
        S.cb_fold = choose_cb(fout, I.g_target);
        S.n_lower += (int)nlo;
        S.n_upper += (int)nhi;
        S.mass_screened += smass;
        S.ahead = (ahead && fout == 0) ? 1 : 0;
    }
    if (ahead) {
        if (fout > 0) {
            // the step taken ahead used columns now fixed: return the kept
            // coordinates to the screening point (r still holds its residual)
            for (int p = tid; p < out; p += NT) {
                const int j = I.idx[p];
                I.x[j] = I.xs[j];
            }
        } else {
            for (int i = tid; i < m; i += NT) I.r[i] = I.r2[i];
        }
    }
}

// Coordinates strictly inside the box at the returned iterate (reported with
// the solve); grid (blocks, count), each block adds its count to n_free,
// which the setup cleared.
__global__ __launch_bounds__(256)
void k_count_free(const Inst* __restrict__ insts, State* __restrict__ st)
{
    __shared__ double sh[4];
    const Inst& I = insts[blockIdx.y];
    double c = 0.0;
    for (int j = blockIdx.x * 256 + threadIdx.x; j < I.n; j += gridDim.x * 256) {
        const double xj = I.x[j];
        c += (xj > lo_of(I.l, j) && xj < up_of(I.u, j)) ? 1.0 : 0.0;
    }
    c = block_sum<256>(c, sh);
    if (threadIdx.x == 0 && c > 0.0) atomicAdd(&st[blockIdx.y].n_free, (int)c);
}

hipError_t launch_count_free(const LaunchCtx& c, int count)
{
    k_count_free<<<dim3(16, count), dim3(256), 0, c.stream>>>(c.insts, c.st);
    return hipGetLastError();
}

// One workgroup per instance.  With host_done set, the last workgroup to
// finish (ticket counter next to the stop counter) also copies the stop
// counter into host memory, so no separate copy follows the pass; with
// host_gap set (single instance), it also copies the instance's gap, from
// which the host predicts whether the next pass will stop; with host_seq set
// it then stores the number of screening passes run so far (a counter after
// the ticket) with a system-scope release, so the host can wait for the pass
// by reading that word instead of a completion event.
template <int SK>
__global__ __launch_bounds__(1024)
void k_screen(const Inst* __restrict__ insts, State* __restrict__ st, int* __restrict__ done_counter,
              double eps_gap, int screening, int final_pass, int K, int kk, int ahead, int* host_done,
              double* host_gap, int* host_seq, int* host_nact)
{
    screen_pass<SK>(insts, st, done_counter, eps_gap, screening, final_pass, K, kk, ahead);
    if (host_done == nullptr) return;
    __syncthreads();
    if (threadIdx.x == 0) {
        int* ticket = done_counter + 1;
        __threadfence();
        const int t = atomicAdd(ticket, 1);
        if (t == (int)gridDim.x - 1) {
            __threadfence();
            host_done[0] = atomicAdd(done_counter, 0);
            if (host_gap) host_gap[0] = st[0].gap;
            if (host_nact) host_nact[0] = st[0].n_active;
            atomicExch(ticket, 0);
            if (host_seq) {
                const int seq = atomicAdd(done_counter + 2, 1) + 1;
                __threadfence_system();
                __hip_atomic_store(host_seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Cyclic coordinate descent, one workgroup per instance: for j in P in
// ascending order, x_j <- Pi(x_j + a_j^T r / ||a_j||^2), r -= delta a_j.
// r lives in registers across the whole sweep.  The columns are sequential
// but their loads are not: a ring of PF column buffers keeps the loads of
// the next PF - 1 columns in flight while the current one is reduced and
// applied.  The preserved-set indices are staged in LDS by chunks of 1024
// positions (two buffers, the next chunk loaded when a chunk begins), so a
// column load waits only on an LDS read of its index.  Ring slots are
// compile-time (the step loop is unrolled by PF).
// ---------------------------------------------------------------------------
template <typename TA, int TPC, int R, int V, int PF>
__global__ __launch_bounds__(TPC)
void k_cd(const Inst* __restrict__ insts, State* __restrict__ st, const int* __restrict__ inst_list, int sweeps)
{
    constexpr int RO = R / V;
    constexpr int NW = TPC / 64;
    static_assert(PF >= 2, "at least one column in flight");
    const int ii = inst_list[blockIdx.x];
    const Inst& I = insts[ii];
    const State& S = st[ii];
    if (S.done) return;
    const int L = threadIdx.x;
    const int m = I.m;
    const long long lda = I.lda;
    const TA* __restrict__ A = reinterpret_cast<const TA*>(I.A);
    const int nA = S.n_active;
    // every per-column array through a global address-space pointer held in
    // registers: a flat load also counts against the scalar-load counter, and
    // the wait for a descriptor field would then drain the prefetched columns
    const int* __restrict__ idx = I.idx;
    const double* __restrict__ cn2p = I.cn2;
    double* __restrict__ xp = I.x;
    const double* __restrict__ lp = I.l;
    const double* __restrict__ up = I.u;
    const double* __restrict__ lq = lp ? lp : cn2p;   // always a valid address
    const double* __restrict__ uq = up ? up : cn2p;
    double rl[R];
#pragma unroll
    for (int k = 0; k < RO; ++k)
#pragma unroll
        for (int e = 0; e < V; ++e) {
            const int row = (k * TPC + L) * V + e;
            rl[k * V + e] = (row < m) ? I.r[row] : 0.0;
        }
    bool rowok[R];
#pragma unroll
    for (int k = 0; k < RO; ++k)
#pragma unroll
        for (int e = 0; e < V; ++e) rowok[k * V + e] = (k * TPC + L) * V + e < m;
    __shared__ double red[2][NW];
    int buf = 0;
    // column j and its scalars; rows >= m are masked where the column is used
    struct Col { int j; double c2, x, l, u; };
    TA ab[PF][R];
    Col cs[PF];
    constexpr int CH = 1024;
    __shared__ int s_idx[2][CH];
    auto stage = [&](int c) {                  // chunk c of positions into buffer c & 1
        for (int k = L; k < CH; k += TPC) {
            const int pos = c * CH + k;
            s_idx[c & 1][k] = (pos < nA) ? gload(idx + pos) : 0;
        }
    };
    auto idx_at = [&](int pos) { return s_idx[(pos / CH) & 1][pos % CH]; };
    auto load_col = [&](int j, TA (&dst)[R], Col& nx) {
        const TA* col = A + (long long)j * lda;
#pragma unroll
        for (int k = 0; k < RO; ++k) {
            TA tmp[V];
            load_pack_nb<TA, V>(col, (k * TPC + L) * V, m, tmp);
#pragma unroll
            for (int e = 0; e < V; ++e) dst[k * V + e] = tmp[e];
        }
        nx.j = j;
        nx.c2 = gload(cn2p + j);
        nx.x = gload(xp + j);
        // raw bound values: the defaults for absent bounds are selected where
        // the column is used, so nothing here waits for these loads
        nx.l = gload(lq + j);
        nx.u = gload(uq + j);
    };
    for (int s = 0; s < sweeps; ++s) {
        if (nA == 0) break;
        stage(0);
        stage(1);
        __syncthreads();
        // prologue: columns of positions 0 .. PF-2 in slots 0 .. PF-2
#pragma unroll
        for (int q = 0; q < PF - 1; ++q)
            if (q < nA) load_col(idx_at(q), ab[q], cs[q]);
        for (int p0 = 0; p0 < nA; p0 += PF) {
#pragma unroll
            for (int q = 0; q < PF; ++q) {
                const int p = p0 + q;
                if (p >= nA) break;
                // a chunk begins: the buffer of the one before it is free (the
                // lookahead only runs forward) and takes the chunk after it
                if (p % CH == 0 && p > 0) {
                    stage(p / CH + 1);
                    __syncthreads();
                }
                // issue position p + PF - 1 into the slot freed by step p - 1
                const int s1 = (q + PF - 1) % PF;
                if (p + PF - 1 < nA) load_col(idx_at(p + PF - 1), ab[s1], cs[s1]);
                // independent of the dot product: overlaps its reduction
                const double ic2 = (cs[q].c2 > 0.0) ? 1.0 / cs[q].c2 : 0.0;
                double d = 0.0;
#pragma unroll
                for (int k = 0; k < R; ++k) d = fma(rowok[k] ? (double)ab[q][k] : 0.0, rl[k], d);
                d = wave_sum_dpp(d);
                if constexpr (NW > 1) {
                    if ((L & 63) == 0) red[buf][L >> 6] = d;
                    __syncthreads();
                    double t2 = 0.0;
#pragma unroll
                    for (int w = 0; w < NW; ++w) t2 += red[buf][w];
                    d = t2;
                    buf ^= 1;
                }
                // branch-free update (a zero column, ic2 = 0, leaves x_j and r as
                // they are); only the store of x_j is conditional
                const Col& cur = cs[q];
                const double lo = lp ? cur.l : 0.0, hi = up ? cur.u : __builtin_inf();
                const double xn = fmin(fmax(cur.x + d * ic2, lo), hi);
                const double delta = (cur.c2 > 0.0) ? xn - cur.x : 0.0;
#pragma unroll
                for (int k = 0; k < R; ++k) rl[k] = fma(-delta, rowok[k] ? (double)ab[q][k] : 0.0, rl[k]);
                if (L == 0 && delta != 0.0) gstore(xp + cur.j, xn);
            }
        }
        // the next sweep reads x_j written by lane 0 in this one
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < RO; ++k)
#pragma unroll
        for (int e = 0; e < V; ++e) {
            const int row = (k * TPC + L) * V + e;
            if (row < m) I.r[row] = rl[k * V + e];
        }
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
// Sweep variants are instantiated in separate translation units
// (sweep_<type>_<part>.hip) so that they compile in parallel.
#define BXS_SWEEP_PART_DECL(NAME) \
    hipError_t NAME(const LaunchCtx& c, int variant, int mode, const Item* items, int n_items, int first);
BXS_SWEEP_PART_DECL(sweep_f32v_0)
BXS_SWEEP_PART_DECL(sweep_f32v_1)
BXS_SWEEP_PART_DECL(sweep_f32v_2)
BXS_SWEEP_PART_DECL(sweep_f64v_0)
BXS_SWEEP_PART_DECL(sweep_f64v_1)
BXS_SWEEP_PART_DECL(sweep_f64v_2)
BXS_SWEEP_PART_DECL(sweep_f32s)
BXS_SWEEP_PART_DECL(sweep_f64s)
BXS_SWEEP_PART_DECL(sweep_bf16v_0)
BXS_SWEEP_PART_DECL(sweep_bf16v_1)
BXS_SWEEP_PART_DECL(sweep_bf16v_2)
BXS_SWEEP_PART_DECL(sweep_bf16s)
#undef BXS_SWEEP_PART_DECL

hipError_t launch_sweep(const LaunchCtx& c, int variant, int mode, const Item* items, int n_items, int first)
{
    if (n_items <= 0) return hipSuccess;
    if (variant < 0 || variant >= kNumVariants) return hipErrorInvalidValue;
    if (c.dtype == BXS_BF16) {
        if (!c.vec) return sweep_bf16s(c, variant, mode, items, n_items, first);
        switch (variant % kSweepParts) {
        case 0: return sweep_bf16v_0(c, variant, mode, items, n_items, first);
        case 1: return sweep_bf16v_1(c, variant, mode, items, n_items, first);
        default: return sweep_bf16v_2(c, variant, mode, items, n_items, first);
        }
    }
    if (c.dtype == BXS_F32) {
        if (!c.vec) return sweep_f32s(c, variant, mode, items, n_items, first);
        switch (variant % kSweepParts) {
        case 0: return sweep_f32v_0(c, variant, mode, items, n_items, first);
        case 1: return sweep_f32v_1(c, variant, mode, items, n_items, first);
        default: return sweep_f32v_2(c, variant, mode, items, n_items, first);
        }
    }
    if (!c.vec) return sweep_f64s(c, variant, mode, items, n_items, first);
    switch (variant % kSweepParts) {
    case 0: return sweep_f64v_0(c, variant, mode, items, n_items, first);
    case 1: return sweep_f64v_1(c, variant, mode, items, n_items, first);
    default: return sweep_f64v_2(c, variant, mode, items, n_items, first);
    }
}

template <typename TA, int V>
static hipError_t cd_dispatch_v(const LaunchCtx& c, int bucket, const int* list, int n_list, int sweeps)
{
// PF: columns in flight, sized to the registers each bucket's workgroup
// leaves a thread (64 and 256 threads: 512 VGPRs, 512: 256, 1024: 128)
#define BXS_CD(TPC, R, PF)                                                                              \
    {                                                                                                   \
        constexpr int VV = (V < R) ? V : R;                                                             \
        k_cd<TA, TPC, R, VV, PF><<<dim3(n_list), dim3(TPC), 0, c.stream>>>(c.insts, c.st, list, sweeps); \
        return hipGetLastError();                                                                       \
    }
    switch (bucket) {
    case 0: BXS_CD(64, 1, 8)
    case 1: BXS_CD(64, 2, 8)
    case 2: BXS_CD(64, 4, 8)
    case 3: BXS_CD(64, 8, 8)
    case 4: BXS_CD(256, 4, 8)
    case 5: BXS_CD(256, 8, 8)
    case 6: BXS_CD(256, 16, 6)
    case 7: BXS_CD(512, 16, (sizeof(TA) == 8 && V == 1) ? 2 : 3)
    case 8: BXS_CD(1024, 16, 2)
    default: return hipErrorInvalidValue;
    }
#undef BXS_CD
}

hipError_t launch_cd(const LaunchCtx& c, int bucket, const int* inst_list, int n_list, int sweeps)
{
    if (n_list <= 0) return hipSuccess;
    if (c.dtype == BXS_BF16)
        return c.vec ? cd_dispatch_v<__bf16, 8>(c, bucket, inst_list, n_list, sweeps)
                     : cd_dispatch_v<__bf16, 1>(c, bucket, inst_list, n_list, sweeps);
    if (c.dtype == BXS_F32)
        return c.vec ? cd_dispatch_v<float, 4>(c, bucket, inst_list, n_list, sweeps)
                     : cd_dispatch_v<float, 1>(c, bucket, inst_list, n_list, sweeps);
    return c.vec ? cd_dispatch_v<double, 2>(c, bucket, inst_list, n_list, sweeps)
                 : cd_dispatch_v<double, 1>(c, bucket, inst_list, n_list, sweeps);
}

hipError_t launch_reduce(const LaunchCtx& c, int mode, const RItem* ritems, int n_ritems, int first,
                         const RItem* nritems, int n_nritems)
{
    if (n_nritems > 0) {
        const dim3 g(n_nritems), b(kRedRowsN);
        switch (mode) {
        case kRedResidual: k_reduce_n<kRedResidual><<<g, b, 0, c.stream>>>(c.insts, c.st, nritems, first); break;
        case kRedFold: k_reduce_n<kRedFold><<<g, b, 0, c.stream>>>(c.insts, c.st, nritems, first); break;
        case kRedPow: k_reduce_n<kRedPow><<<g, b, 0, c.stream>>>(c.insts, c.st, nritems, first); break;
        case kRedAhead: k_reduce_n<kRedAhead><<<g, b, 0, c.stream>>>(c.insts, c.st, nritems, first); break;
        case kRedCP: k_reduce_n<kRedCP><<<g, b, 0, c.stream>>>(c.insts, c.st, nritems, first); break;
        default: return hipErrorInvalidValue;
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (n_ritems <= 0) return hipSuccess;
    dim3 grid(n_ritems), block(1024);
    switch (mode) {
    case kRedResidual: k_reduce<kRedResidual><<<grid, block, 0, c.stream>>>(c.insts, c.st, ritems, first, c.single); break;
    case kRedFold: k_reduce<kRedFold><<<grid, block, 0, c.stream>>>(c.insts, c.st, ritems, first, c.single); break;
    case kRedPow: k_reduce<kRedPow><<<grid, block, 0, c.stream>>>(c.insts, c.st, ritems, first, c.single); break;
    case kRedAhead: k_reduce<kRedAhead><<<grid, block, 0, c.stream>>>(c.insts, c.st, ritems, first, c.single); break;
    case kRedCP: k_reduce<kRedCP><<<grid, block, 0, c.stream>>>(c.insts, c.st, ritems, first, c.single); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_init(const LaunchCtx& c, int count, const double*)
{
    k_init<<<dim3(8, count), dim3(256), 0, c.stream>>>(c.insts, c.st);
    return hipGetLastError();
}

hipError_t launch_colstats(const LaunchCtx& c, int bucket, const Item* items, int n_items)
{
    (void)bucket;
    if (n_items <= 0) return hipSuccess;
    const dim3 g(n_items), b(256);
    if (c.dtype == BXS_BF16) {
        if (c.vec) k_colstats<__bf16, 8><<<g, b, 0, c.stream>>>(c.insts, c.st, items);
        else k_colstats<__bf16, 1><<<g, b, 0, c.stream>>>(c.insts, c.st, items);
    } else if (c.dtype == BXS_F32) {
        if (c.vec) k_colstats<float, 4><<<g, b, 0, c.stream>>>(c.insts, c.st, items);
        else k_colstats<float, 1><<<g, b, 0, c.stream>>>(c.insts, c.st, items);
    } else {
        if (c.vec) k_colstats<double, 2><<<g, b, 0, c.stream>>>(c.insts, c.st, items);
        else k_colstats<double, 1><<<g, b, 0, c.stream>>>(c.insts, c.st, items);
    }
    return hipGetLastError();
}

hipError_t launch_validate(const LaunchCtx& c, int count)
{
    k_validate<<<dim3((count + 255) / 256), dim3(256), 0, c.stream>>>(c.st, c.done_counter, count);
    return hipGetLastError();
}

hipError_t launch_publish(const LaunchCtx& c, int* host_dst)
{
    k_publish<<<dim3(1), dim3(64), 0, c.stream>>>(c.done_counter, host_dst);
    return hipGetLastError();
}

hipError_t launch_pow_init(const LaunchCtx& c, int count)
{
    k_inst_scalars<<<dim3(count), dim3(256), 0, c.stream>>>(c.insts, c.st, 1, 0.0);
    return hipGetLastError();
}

hipError_t launch_set_step(const LaunchCtx& c, int count, double step)
{
    k_inst_scalars<<<dim3(count), dim3(256), 0, c.stream>>>(c.insts, c.st, 0, step);
    return hipGetLastError();
}

hipError_t launch_lanczos(const LaunchCtx& c, int count, int k, int last, int cp)
{
    k_lanczos<<<dim3(count), dim3(1024), 0, c.stream>>>(c.insts, c.st, k, last, cp);
    return hipGetLastError();
}

// Chambolle-Pock start: the dual step from x0 with v = 0,
// v = sigma (A x0 - y') / (1 + sigma) = -sigma r / (1 + sigma); grid (blocks, count)
__global__ __launch_bounds__(256)
void k_cp_init(const Inst* __restrict__ insts, const State* __restrict__ st)
{
    const Inst& I = insts[blockIdx.y];
    const double sg = st[blockIdx.y].step, hub = I.hub;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < I.m; i += gridDim.x * 256)
        I.r2[i] = fmin(fmax(-sg * I.r[i] / (1.0 + sg), -hub), hub);
}

hipError_t launch_cp_init(const LaunchCtx& c, int count)
{
    k_cp_init<<<dim3(16, count), dim3(256), 0, c.stream>>>(c.insts, c.st);
    return hipGetLastError();
}

hipError_t launch_screen(const LaunchCtx& c, int count, double eps_gap, int screening, int final_pass,
                         int K, int kk, int ahead, int* host_done, double* host_gap, int* host_seq,
                         int kind, int* host_nact)
{
    const dim3 g(count), b(1024);
    if (kind == kScreenOracleDual)
        k_screen<kScreenOracleDual><<<g, b, 0, c.stream>>>(c.insts, c.st, c.done_counter, eps_gap, screening,
                                                           final_pass, K, kk, ahead, host_done, host_gap, host_seq,
                                                           host_nact);
    else if (kind == kScreenHuber)
        k_screen<kScreenHuber><<<g, b, 0, c.stream>>>(c.insts, c.st, c.done_counter, eps_gap, screening,
                                                      final_pass, K, kk, ahead, host_done, host_gap, host_seq,
                                                      host_nact);
    else
        k_screen<kScreenLS><<<g, b, 0, c.stream>>>(c.insts, c.st, c.done_counter, eps_gap, screening,
                                                   final_pass, K, kk, ahead, host_done, host_gap, host_seq,
                                                   host_nact);
    return hipGetLastError();
}

}  // namespace bxs
