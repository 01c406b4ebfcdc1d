// gfx950 kernels of the boxscreen library: column sweeps (the matrix-vector
// products of the projected-gradient step, the correlations A^T r, the fold of
// screened columns, power iteration), their deterministic partial reductions,
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
#include "bxs_internal.h"

#include <type_traits>

namespace bxs {

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double lo_of(const double* l, int j) { return l ? l[j] : 0.0; }
__device__ __forceinline__ double up_of(const double* u, int j) { return u ? u[j] : __builtin_inf(); }
__device__ __forceinline__ double t_of(const double* t, int i) { return t ? t[i] : -1.0; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}

// Block-wide reductions with a fixed summation order; every thread gets the
// result.  `sh` must hold NT/64 doubles; the trailing barrier makes it
// reusable immediately.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[wave] = v;
    __syncthreads();
    double tot = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) tot += sh[w];
    __syncthreads();
    return tot;
}
template <int NT>
__device__ __forceinline__ double block_max(double v, double* sh) {
    v = wave_max(v);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[wave] = v;
    __syncthreads();
    double tot = sh[0];
#pragma unroll
    for (int w = 1; w < NT / 64; ++w) tot = fmax(tot, sh[w]);
    __syncthreads();
    return tot;
}
template <int NT>
__device__ __forceinline__ double block_min(double v, double* sh) {
    v = wave_min(v);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[wave] = v;
    __syncthreads();
    double tot = sh[0];
#pragma unroll
    for (int w = 1; w < NT / 64; ++w) tot = fmin(tot, sh[w]);
    __syncthreads();
    return tot;
}

__host__ __device__ __forceinline__ int choose_cb(int n_list, int g_target) {
    int cb = (n_list + g_target - 1) / g_target;
    return cb < kCbMin ? kCbMin : (cb > kCbMax ? kCbMax : cb);
}

// Load V consecutive elements of a column starting at row `row` (row % V == 0)
// as doubles; rows >= m read as 0.  With V > 1 the caller guarantees that
// lda % V == 0 and that the column start is 16-byte aligned, so the vector
// never crosses the column's lda-element storage.
template <typename TA, int V>
struct alignas(sizeof(TA) * V) Pack { TA v[V]; };

template <typename TA, int V>
__device__ __forceinline__ void load_pack(const TA* __restrict__ col, int row, int m, TA (&o)[V]) {
    if (row < m) {
        if constexpr (V == 1) {
            o[0] = col[row];
        } else {
            const Pack<TA, V> pk = *reinterpret_cast<const Pack<TA, V>*>(col + row);
#pragma unroll
            for (int e = 0; e < V; ++e) o[e] = (row + e < m) ? pk.v[e] : TA(0);
        }
    } else {
#pragma unroll
        for (int e = 0; e < V; ++e) o[e] = TA(0);
    }
}

// ---------------------------------------------------------------------------
// Column sweep.  One workgroup = one work item (instance, block of cb
// consecutive positions of the preserved-set list, or of the fold list).
// NG groups of TPC threads each take every NG-th column of the item; thread
// L of a group owns rows {(k*TPC + L)*V + e}, k < R/V, e < V, and keeps the
// residual rows and its share of the partial product in registers.
// ---------------------------------------------------------------------------
template <typename TA, int TPC, int NG, int R, int V, int MODE>
__global__ __launch_bounds__(TPC * NG)
void k_sweep(const Inst* __restrict__ insts, State* __restrict__ st, const Item* __restrict__ items)
{
    constexpr int RO = R / V;
    constexpr int CBI = (R >= 16) ? 2 : ((R >= 8) ? 4 : 8);
    constexpr bool DOT = (MODE == kModePG || MODE == kModeCorr || MODE == kModePow);
    constexpr bool ACC = (MODE != kModeCorr);
    constexpr int NW = TPC / 64;
    static_assert(R % V == 0, "rows per thread must be a multiple of the vector width");

    const Item it = items[blockIdx.x];
    const Inst& I = insts[it.inst];
    State& S = st[it.inst];
    if (S.done) return;
    const int nlist = (MODE == kModeFold) ? S.n_fold : S.n_active;
    const int cb = (MODE == kModeFold) ? S.cb_fold : S.cb;
    const int pos0 = it.t * cb;
    if (pos0 >= nlist) return;
    const int pos1 = min(pos0 + cb, nlist);

    const int tid = threadIdx.x;
    const int grp = (NG > 1) ? tid / TPC : 0;
    const int L = (NG > 1) ? tid % TPC : tid;
    const int m = I.m;
    const long long lda = I.lda;
    const TA* __restrict__ A = reinterpret_cast<const TA*>(I.A);
    const int* __restrict__ list = (MODE == kModeFold) ? I.fidx : I.idx;
    const double eta = (MODE == kModePG) ? S.step : 0.0;

    double rl[R];
    if constexpr (DOT) {
#pragma unroll
        for (int k = 0; k < RO; ++k)
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const int row = (k * TPC + L) * V + e;
                rl[k * V + e] = (row < m) ? I.r[row] : 0.0;
            }
    }
    double p[R];
    double p2[(MODE == kModeFold) ? R : 1];
#pragma unroll
    for (int k = 0; k < R; ++k) p[k] = 0.0;
    if constexpr (MODE == kModeFold) {
#pragma unroll
        for (int k = 0; k < R; ++k) p2[k] = 0.0;
    }
    double gsq = 0.0;

    __shared__ double red[2][(NW > 1) ? NW : 1][CBI];
    int buf = 0;

    // software pipeline: columns of the next round (and their per-column
    // scalars) are loaded while the current round is reduced and applied.
    // Reading x_j before the round's barrier also orders it before the write
    // of x_j by lane 0 of the group.
    TA av[CBI][R];
    int jc[CBI];
    bool vc[CBI];
    double xs[CBI], ls[CBI], us[CBI];
    auto load_round = [&](int rs, TA (&dst)[CBI][R], int (&jj)[CBI], bool (&vv)[CBI],
                          double (&xo)[CBI], double (&lo)[CBI], double (&uo)[CBI]) {
#pragma unroll
        for (int c = 0; c < CBI; ++c) {
            const int q = rs + c * NG + grp;
            vv[c] = q < pos1;
            jj[c] = vv[c] ? list[q] : 0;
            xo[c] = 0.0; lo[c] = 0.0; uo[c] = 0.0;
            if (vv[c]) {
                if constexpr (MODE == kModePG) {
                    xo[c] = I.x[jj[c]]; lo[c] = lo_of(I.l, jj[c]); uo[c] = up_of(I.u, jj[c]);
                } else if constexpr (MODE == kModeAx) {
                    xo[c] = I.x[jj[c]];
                } else if constexpr (MODE == kModeFold) {
                    xo[c] = I.fval[q]; lo[c] = I.fdx[q];
                }
            }
            const TA* col = A + (long long)jj[c] * lda;
#pragma unroll
            for (int k = 0; k < RO; ++k) {
                TA tmp[V];
                if (vv[c]) {
                    load_pack<TA, V>(col, (k * TPC + L) * V, m, tmp);
                } else {
#pragma unroll
                    for (int e = 0; e < V; ++e) tmp[e] = TA(0);
                }
#pragma unroll
                for (int e = 0; e < V; ++e) dst[c][k * V + e] = tmp[e];
            }
        }
    };

    load_round(pos0, av, jc, vc, xs, ls, us);
    for (int rs = pos0; rs < pos1; rs += NG * CBI) {
        TA an[CBI][R];
        int jn[CBI];
        bool vn[CBI];
        double xn_[CBI], ln_[CBI], un_[CBI];
        const int rs_next = rs + NG * CBI;
        if (rs_next < pos1) {
            load_round(rs_next, an, jn, vn, xn_, ln_, un_);
        }

        double coef[CBI], coef2[CBI];
        if constexpr (DOT) {
            double d[CBI];
#pragma unroll
            for (int c = 0; c < CBI; ++c) {
                double s = 0.0;
#pragma unroll
                for (int k = 0; k < R; ++k) s = fma((double)av[c][k], rl[k], s);
                d[c] = s;
            }
#pragma unroll
            for (int c = 0; c < CBI; ++c) d[c] = wave_sum(d[c]);
            if constexpr (NW > 1) {
                const int wv = tid >> 6;
                if ((tid & 63) == 0) {
#pragma unroll
                    for (int c = 0; c < CBI; ++c) red[buf][wv][c] = d[c];
                }
                __syncthreads();
#pragma unroll
                for (int c = 0; c < CBI; ++c) {
                    double s = 0.0;
#pragma unroll
                    for (int w = 0; w < NW; ++w) s += red[buf][w][c];
                    d[c] = s;
                }
                buf ^= 1;
            }
#pragma unroll
            for (int c = 0; c < CBI; ++c) {
                coef[c] = 0.0;
                if (!vc[c]) continue;
                const int j = jc[c];
                if constexpr (MODE == kModePG) {
                    const double xn = fmin(fmax(xs[c] + eta * d[c], ls[c]), us[c]);
                    coef[c] = xn;
                    if (L == 0) I.x[j] = xn;
                } else if constexpr (MODE == kModeCorr) {
                    if (L == 0) I.g[j] = d[c];
                } else {  // power iteration
                    coef[c] = d[c];
                    gsq += d[c] * d[c];
                }
            }
        } else {
#pragma unroll
            for (int c = 0; c < CBI; ++c) {
                coef[c] = vc[c] ? xs[c] : 0.0;                          // x_j, or b_j for the fold
                coef2[c] = (MODE == kModeFold && vc[c]) ? ls[c] : 0.0;  // b_j - x_j (fold)
            }
        }
        if constexpr (ACC) {
#pragma unroll
            for (int c = 0; c < CBI; ++c)
#pragma unroll
                for (int k = 0; k < R; ++k) p[k] = fma((double)av[c][k], coef[c], p[k]);
            if constexpr (MODE == kModeFold) {
#pragma unroll
                for (int c = 0; c < CBI; ++c)
#pragma unroll
                    for (int k = 0; k < R; ++k) p2[k] = fma((double)av[c][k], coef2[c], p2[k]);
            }
        }
        if (rs_next < pos1) {
#pragma unroll
            for (int c = 0; c < CBI; ++c) {
                jc[c] = jn[c];
                vc[c] = vn[c];
                xs[c] = xn_[c]; ls[c] = ln_[c]; us[c] = un_[c];
#pragma unroll
                for (int k = 0; k < R; ++k) av[c][k] = an[c][k];
            }
        }
    }

    if constexpr (!ACC) return;

    // combine the NG groups' partial products (fixed order) and store
    if constexpr (NG > 1) {
        __shared__ double comb[(NG > 1) ? (NG - 1) * TPC * R : 1];
        __shared__ double gs[NG];
        if (grp > 0) {
#pragma unroll
            for (int k = 0; k < R; ++k) comb[((grp - 1) * R + k) * TPC + L] = p[k];
        }
        if (MODE == kModePow && L == 0) gs[grp] = gsq;
        __syncthreads();
        if (grp == 0) {
#pragma unroll
            for (int g2 = 1; g2 < NG; ++g2)
#pragma unroll
                for (int k = 0; k < R; ++k) p[k] += comb[((g2 - 1) * R + k) * TPC + L];
            if (MODE == kModePow && L == 0) {
                double s = 0.0;
                for (int g2 = 0; g2 < NG; ++g2) s += gs[g2];
                gsq = s;
            }
        }
        if constexpr (MODE == kModeFold) {
            __syncthreads();
            if (grp > 0) {
#pragma unroll
                for (int k = 0; k < R; ++k) comb[((grp - 1) * R + k) * TPC + L] = p2[k];
            }
            __syncthreads();
            if (grp == 0) {
#pragma unroll
                for (int g2 = 1; g2 < NG; ++g2)
#pragma unroll
                    for (int k = 0; k < R; ++k) p2[k] += comb[((g2 - 1) * R + k) * TPC + L];
            }
        }
        if (grp != 0) return;
    }
    double* __restrict__ out = I.part + (size_t)it.t * m;
#pragma unroll
    for (int k = 0; k < RO; ++k)
#pragma unroll
        for (int e = 0; e < V; ++e) {
            const int row = (k * TPC + L) * V + e;
            if (row < m) out[row] = p[k * V + e];
        }
    if constexpr (MODE == kModeFold) {
        double* __restrict__ out2 = I.part2 + (size_t)it.t * m;
#pragma unroll
        for (int k = 0; k < RO; ++k)
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const int row = (k * TPC + L) * V + e;
                if (row < m) out2[row] = p2[k * V + e];
            }
    }
    if constexpr (MODE == kModePow) {
        if (L == 0) I.iscal[it.t] = gsq;
    }
}

// ---------------------------------------------------------------------------
// Partial reduction: 64 rows x 4 item-groups per workgroup, fixed order.
// ---------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(256)
void k_reduce(const Inst* __restrict__ insts, State* __restrict__ st, const RItem* __restrict__ ritems)
{
    const RItem ri = ritems[blockIdx.x];
    const Inst& I = insts[ri.inst];
    const State& S = st[ri.inst];
    if (S.done) return;
    const int nlist = (MODE == kRedFold) ? S.n_fold : S.n_active;
    const int cb = (MODE == kRedFold) ? S.cb_fold : S.cb;
    const int T = (nlist + cb - 1) / cb;
    const int rowl = threadIdx.x & 63, tg = threadIdx.x >> 6;
    const int row = ri.rb * 64 + rowl;
    const int m = I.m;
    double s = 0.0, s2 = 0.0;
    if (row < m) {
        for (int t = tg; t < T; t += 4) {
            s += I.part[(size_t)t * m + row];
            if (MODE == kRedFold) s2 += I.part2[(size_t)t * m + row];
        }
    }
    __shared__ double sh[4][64], sh2[4][64];
    sh[tg][rowl] = s;
    sh2[tg][rowl] = s2;
    __syncthreads();
    if (tg == 0 && row < m) {
        const double tot = ((sh[0][rowl] + sh[1][rowl]) + sh[2][rowl]) + sh[3][rowl];
        if constexpr (MODE == kRedResidual) {
            I.r[row] = I.yp[row] - tot;
        } else if constexpr (MODE == kRedFold) {
            const double tot2 = ((sh2[0][rowl] + sh2[1][rowl]) + sh2[2][rowl]) + sh2[3][rowl];
            I.yp[row] -= tot;
            I.r[row] -= tot2;
        } else {
            I.r[row] = tot;
        }
    }
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
    }
}

// ---------------------------------------------------------------------------
// Column statistics: rigorous norm bound, sum of squares, w = A^T t, and a
// finiteness check of A.  One wave per column.
// ---------------------------------------------------------------------------
template <typename TA>
__global__ __launch_bounds__(256)
void k_colstats(const Inst* __restrict__ insts, State* __restrict__ st, const Item* __restrict__ items)
{
    const Item it = items[blockIdx.x];
    const Inst& I = insts[it.inst];
    State& S = st[it.inst];
    const int cb = S.cb;
    const int pos0 = it.t * cb;
    const int pos1 = min(pos0 + cb, I.n);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const TA* __restrict__ A = reinterpret_cast<const TA*>(I.A);
    const double gm = gamma_k((double)(I.m / 64) + 8.0);   // summation depth of this kernel
    int err = 0;
    for (int j = pos0 + wv; j < pos1; j += 4) {
        const TA* col = A + (long long)j * I.lda;
        double s2 = 0.0, sw = 0.0;
        for (int i = lane; i < I.m; i += 64) {
            const double a = (double)col[i];
            if (!isfinite(a)) err = kErrNonfinite;
            s2 = fma(a, a, s2);
            sw = fma(a, t_of(I.t, i), sw);
        }
        s2 = wave_sum(s2);
        sw = wave_sum(sw);
        if (lane == 0) {
            I.cn2[j] = s2;
            I.cn[j] = sqrt(s2 * (1.0 + gm)) * (1.0 + 2.0 * kUnit);
            I.w[j] = sw;
        }
    }
    if (err) atomicOr(&S.err, err);
}

// ---------------------------------------------------------------------------
// Per-instance scalars: bounds on ||y|| and ||t||, step from the caller, and
// the starting vector of the power iteration (when do_pow).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256)
void k_inst_scalars(const Inst* __restrict__ insts, State* __restrict__ st, int do_pow, double user_step)
{
    __shared__ double sh[4];
    const Inst& I = insts[blockIdx.x];
    State& S = st[blockIdx.x];
    const int m = I.m;
    double sy = 0.0, stt = 0.0, su = 0.0;
    for (int i = threadIdx.x; i < m; i += 256) {
        const double yv = I.y[i], tv = t_of(I.t, i);
        sy = fma(yv, yv, sy);
        stt = fma(tv, tv, stt);
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
    if (do_pow) {
        const double inv = 1.0 / sqrt(su);
        for (int i = threadIdx.x; i < m; i += 256) I.r[i] *= inv;
    }
    if (threadIdx.x == 0) {
        const double gm = gamma_k((double)m + 32.0);
        S.ynorm = sqrt(sy * (1.0 + gm)) * (1.0 + 2.0 * kUnit);
        S.tnorm = sqrt(stt * (1.0 + gm)) * (1.0 + 2.0 * kUnit);
        if (!do_pow) {
            S.step = user_step;
            S.lipschitz = 0.0;
        }
    }
}

// Power iteration on A A^T: after the sweep and reduction r = A A^T u, with
// iscal holding the pieces of ||A^T u||^2 (the Rayleigh quotient of A A^T at
// the unit vector u).  Normalise r; on the last round set the step.
__global__ __launch_bounds__(256)
void k_pow_normalize(const Inst* __restrict__ insts, State* __restrict__ st, int last, double user_step)
{
    __shared__ double sh[4];
    const Inst& I = insts[blockIdx.x];
    State& S = st[blockIdx.x];
    const int m = I.m;
    double s = 0.0;
    for (int i = threadIdx.x; i < m; i += 256) s = fma(I.r[i], I.r[i], s);
    s = block_sum<256>(s, sh);
    const int T = (S.n_active + S.cb - 1) / S.cb;
    double lam = 0.0;
    for (int t = threadIdx.x; t < T; t += 256) lam += I.iscal[t];
    lam = block_sum<256>(lam, sh);
    const double inv = (s > 0.0) ? 1.0 / sqrt(s) : 0.0;
    for (int i = threadIdx.x; i < m; i += 256) I.r[i] *= inv;
    if (threadIdx.x == 0) {
        S.lipschitz = lam;
        if (last) S.step = (user_step > 0.0) ? user_step : ((lam > 0.0) ? 1.0 / (1.05 * lam) : 1.0);
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
__global__ __launch_bounds__(1024)
void k_screen(const Inst* __restrict__ insts, State* __restrict__ st, int* __restrict__ done_counter,
              double eps_gap, int screening, int final_pass, long long iters, int kk)
{
    constexpr int NT = 1024;
    __shared__ double sh[NT / 64];
    __shared__ int wk[NT / 64], ws[NT / 64];
    const Inst& I = insts[blockIdx.x];
    State& S = st[blockIdx.x];
    if (S.done) return;
    const int tid = threadIdx.x;
    const int m = I.m, n = I.n;
    const int nA = S.n_active;
    const int passes = S.passes;
    const double tnorm = S.tnorm;
    const double u1 = kUnit;

    double a = 0.0;
    for (int i = tid; i < m; i += NT) a = fma(I.r[i], I.r[i], a);
    const double rsq = block_sum<NT>(a, sh);
    const double rnorm = sqrt(rsq * (1.0 + gamma_k((double)(m / NT) + 24.0))) * (1.0 + 2.0 * u1);
    // error bounds of the correlations g_j (sweep kernels) and of w_j = a_j^T t
    // (column statistics), by Cauchy-Schwarz: sum_i |a_ij v_i| <= ||a_j|| ||v||
    const double gm = gamma_k(kDotDepth);
    const double gw = gamma_k((double)(m / 64) + 8.0);

    // pass 1: interior check of t, translation coefficient, absolute mass
    double tv = 1.0, emax = 0.0, mass = 0.0, hasinf = 0.0;
    for (int p = tid; p < nA; p += NT) {
        const int j = I.idx[p];
        const double cnj = I.cn[j];
        mass = fma(fabs(I.x[j]), cnj, mass);
        if (isinf(up_of(I.u, j))) {
            hasinf = 1.0;
            const double ewj = gw * cnj * tnorm;
            const double egj = gm * cnj * rnorm;
            const double wj = I.w[j];
            if (!(wj + ewj < 0.0)) {
                tv = 0.0;
            } else {
                const double num = fmax(I.g[j] + egj, 0.0);
                const double den = -wj - ewj;
                emax = fmax(emax, num / den);
            }
        }
    }
    tv = block_min<NT>(tv, sh);
    emax = block_max<NT>(emax, sh);
    mass = block_sum<NT>(mass, sh);
    hasinf = block_max<NT>(hasinf, sh);
    const bool has_inf = hasinf > 0.5;
    const bool fallback = has_inf && !(tv > 0.5);
    const double eps = (has_inf && !fallback) ? emax * (1.0 + 4.0 * u1) : 0.0;
    const double massall = (mass + S.mass_screened) * (1.0 + gamma_k((double)n + 64.0));
    const double delta_r = gamma_k(2.0 * n + 4.0 * passes + 64.0) * (S.ynorm + 2.0 * massall);

    // pass 2: gap
    double G;
    if (!fallback) {
        double acc = 0.0;
        for (int p = tid; p < nA; p += NT) {
            const int j = I.idx[p];
            const double cnj = I.cn[j], gj = I.g[j], wj = I.w[j];
            const double cj = fma(eps, wj, gj);
            const double ej = cnj * (gm * rnorm + gw * eps * tnorm) + 4.0 * u1 * (fabs(gj) + eps * fabs(wj));
            const double xj = I.x[j], lj = lo_of(I.l, j), uj = up_of(I.u, j);
            double term = (xj - lj) * fmax(ej - cj, 0.0);
            if (!isinf(uj)) term += (uj - xj) * fmax(cj + ej, 0.0);
            acc += term;
        }
        const double gsum = block_sum<NT>(acc, sh);
        const double tt = delta_r + eps * tnorm;
        G = (gsum * (1.0 + 3.0 * u1) + 0.5 * tt * tt * (1.0 + 4.0 * u1)) * (1.0 + gamma_k((double)n + 64.0));
    } else {
        const double tt = rnorm + delta_r;
        G = 0.5 * tt * tt * (1.0 + 4.0 * u1);
    }
    const double rad = sqrt(2.0 * G) * (1.0 + 2.0 * u1);
    const double primal = 0.5 * rsq;
    const bool stop = G < eps_gap;
    if (tid == 0) S.col_iters += (long long)nA * kk;

    if (stop || final_pass || !screening || fallback) {
        if (tid == 0) {
            if (passes < I.rec_cap) {
                bxs_pass_record& rc = I.rec[passes];
                rc.iters = iters; rc.n_active = nA; rc.gap = G; rc.radius = rad;
                rc.eps = eps; rc.primal = primal; rc.n_screened = 0;
            }
            S.gap = G; S.radius = rad; S.eps = eps; S.primal = primal;
            S.t_valid = fallback ? 0 : 1;
            S.passes = passes + 1;
            S.n_fold = 0;
            if (stop || final_pass) {
                S.done = 1;
                S.status = stop ? BXS_OK : BXS_MAXITER;
                S.iters = iters;
                atomicAdd(done_counter, 1);
            }
        }
        return;
    }

    // pass 3: safe rule, fix, fold list, in-place compaction of idx
    const int lane = tid & 63, wave = tid >> 6;
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int out = 0, fout = 0;
    double nlo = 0.0, nhi = 0.0, smass = 0.0;
    for (int base = 0; base < nA; base += NT) {
        const int p = base + tid;
        bool lower = false, upper = false, keep = false;
        int j = 0;
        double xj = 0.0, lj = 0.0, uj = 0.0, cnj = 0.0;
        if (p < nA) {
            j = I.idx[p];
            cnj = I.cn[j];
            const double gj = I.g[j], wj = I.w[j];
            const double cj = fma(eps, wj, gj);
            const double ej = cnj * (gm * rnorm + gw * eps * tnorm) + 4.0 * u1 * (fabs(gj) + eps * fabs(wj));
            const double thr = rad * cnj * (1.0 + 2.0 * u1);
            xj = I.x[j]; lj = lo_of(I.l, j); uj = up_of(I.u, j);
            lower = (cj + ej) < -thr;
            upper = !lower && !isinf(uj) && (cj - ej) > thr;
            keep = !(lower || upper);
        }
        const bool scr = lower || upper;
        const unsigned long long mk = __ballot(keep);
        const unsigned long long ms = __ballot(scr);
        if (lane == 0) {
            wk[wave] = __popcll(mk);
            ws[wave] = __popcll(ms);
        }
        __syncthreads();
        int kb = 0, sb = 0, kt = 0, stot = 0;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) {
            if (w < wave) { kb += wk[w]; sb += ws[w]; }
            kt += wk[w];
            stot += ws[w];
        }
        if (keep) I.idx[out + kb + __popcll(mk & lt)] = j;
        if (scr) {
            const int k = fout + sb + __popcll(ms & lt);
            const double b = lower ? lj : uj;
            I.fidx[k] = j;
            I.fval[k] = b;
            I.fdx[k] = b - xj;
            I.x[j] = b;
            I.sat[j] = lower ? (signed char)-1 : (signed char)1;
            smass = fma(fabs(b), cnj, smass);
            if (lower) nlo += 1.0; else nhi += 1.0;
        }
        out += kt;
        fout += stot;
        __syncthreads();
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
        S.gap = G; S.radius = rad; S.eps = eps; S.primal = primal;
        S.t_valid = 1;
        S.passes = passes + 1;
        S.n_active = out;
        S.n_fold = fout;
        S.cb = choose_cb(out, I.g_target);
        S.cb_fold = choose_cb(fout, I.g_target);
        S.n_lower += (int)nlo;
        S.n_upper += (int)nhi;
        S.mass_screened += smass;
    }
}

// ---------------------------------------------------------------------------
// Cyclic coordinate descent, one workgroup per instance: for j in P in
// ascending order, x_j <- Pi(x_j + a_j^T r / ||a_j||^2), r -= delta a_j.
// r lives in registers across the whole sweep; the next column is loaded
// while the current dot product is reduced.
// ---------------------------------------------------------------------------
template <typename TA, int TPC, int R, int V>
__global__ __launch_bounds__(TPC)
void k_cd(const Inst* __restrict__ insts, State* __restrict__ st, const int* __restrict__ inst_list, int sweeps)
{
    constexpr int RO = R / V;
    constexpr int NW = TPC / 64;
    const int ii = inst_list[blockIdx.x];
    const Inst& I = insts[ii];
    const State& S = st[ii];
    if (S.done) return;
    const int L = threadIdx.x;
    const int m = I.m;
    const long long lda = I.lda;
    const TA* __restrict__ A = reinterpret_cast<const TA*>(I.A);
    const int nA = S.n_active;
    double rl[R];
#pragma unroll
    for (int k = 0; k < RO; ++k)
#pragma unroll
        for (int e = 0; e < V; ++e) {
            const int row = (k * TPC + L) * V + e;
            rl[k * V + e] = (row < m) ? I.r[row] : 0.0;
        }
    __shared__ double red[2][NW];
    int buf = 0;
    auto load_col = [&](int j, TA (&dst)[R]) {
        const TA* col = A + (long long)j * lda;
#pragma unroll
        for (int k = 0; k < RO; ++k) {
            TA tmp[V];
            load_pack<TA, V>(col, (k * TPC + L) * V, m, tmp);
#pragma unroll
            for (int e = 0; e < V; ++e) dst[k * V + e] = tmp[e];
        }
    };
    for (int s = 0; s < sweeps; ++s) {
        if (nA == 0) break;
        TA av[R];
        int j = I.idx[0];
        load_col(j, av);
        for (int p = 0; p < nA; ++p) {
            TA an[R];
            int jn = 0;
            if (p + 1 < nA) {
                jn = I.idx[p + 1];
                load_col(jn, an);
            }
            double d = 0.0;
#pragma unroll
            for (int k = 0; k < R; ++k) d = fma((double)av[k], rl[k], d);
            d = wave_sum(d);
            if constexpr (NW > 1) {
                if ((L & 63) == 0) red[buf][L >> 6] = d;
                __syncthreads();
                double t2 = 0.0;
#pragma unroll
                for (int w = 0; w < NW; ++w) t2 += red[buf][w];
                d = t2;
                buf ^= 1;
            }
            const double c2 = I.cn2[j];
            if (c2 > 0.0) {
                const double xj = I.x[j];
                const double xn = fmin(fmax(xj + d / c2, lo_of(I.l, j)), up_of(I.u, j));
                const double delta = xn - xj;
                if (delta != 0.0) {
#pragma unroll
                    for (int k = 0; k < R; ++k) rl[k] = fma(-delta, (double)av[k], rl[k]);
                    if constexpr (NW > 1) __syncthreads();  // every lane has read x_j
                    if (L == 0) I.x[j] = xn;
                }
            }
            if (p + 1 < nA) {
                j = jn;
#pragma unroll
                for (int k = 0; k < R; ++k) av[k] = an[k];
            }
        }
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
template <typename TA, int V>
static hipError_t sweep_dispatch_v(const LaunchCtx& c, int bucket, int mode, const Item* items, int n_items)
{
#define BXS_SWEEP(TPC, NG, R)                                                                     \
    {                                                                                             \
        constexpr int VV = (V < R) ? V : R;                                                       \
        dim3 grid(n_items), block(TPC * NG);                                                      \
        switch (mode) {                                                                           \
        case kModePG: k_sweep<TA, TPC, NG, R, VV, kModePG><<<grid, block, 0, c.stream>>>(c.insts, c.st, items); break;     \
        case kModeCorr: k_sweep<TA, TPC, NG, R, VV, kModeCorr><<<grid, block, 0, c.stream>>>(c.insts, c.st, items); break; \
        case kModeAx: k_sweep<TA, TPC, NG, R, VV, kModeAx><<<grid, block, 0, c.stream>>>(c.insts, c.st, items); break;     \
        case kModeFold: k_sweep<TA, TPC, NG, R, VV, kModeFold><<<grid, block, 0, c.stream>>>(c.insts, c.st, items); break; \
        default: k_sweep<TA, TPC, NG, R, VV, kModePow><<<grid, block, 0, c.stream>>>(c.insts, c.st, items); break;         \
        }                                                                                         \
        return hipGetLastError();                                                                 \
    }
    switch (bucket) {
    case 0: BXS_SWEEP(64, 4, 1)
    case 1: BXS_SWEEP(64, 4, 2)
    case 2: BXS_SWEEP(64, 4, 4)
    case 3: BXS_SWEEP(64, 4, 8)
    case 4: BXS_SWEEP(256, 1, 4)
    case 5: BXS_SWEEP(256, 1, 8)
    case 6: BXS_SWEEP(256, 1, 16)
    case 7: BXS_SWEEP(512, 1, 16)
    case 8: BXS_SWEEP(1024, 1, 16)
    default: return hipErrorInvalidValue;
    }
#undef BXS_SWEEP
}

hipError_t launch_sweep(const LaunchCtx& c, int bucket, int mode, const Item* items, int n_items)
{
    if (n_items <= 0) return hipSuccess;
    if (c.dtype == BXS_F32)
        return c.vec ? sweep_dispatch_v<float, 4>(c, bucket, mode, items, n_items)
                     : sweep_dispatch_v<float, 1>(c, bucket, mode, items, n_items);
    return c.vec ? sweep_dispatch_v<double, 2>(c, bucket, mode, items, n_items)
                 : sweep_dispatch_v<double, 1>(c, bucket, mode, items, n_items);
}

template <typename TA, int V>
static hipError_t cd_dispatch_v(const LaunchCtx& c, int bucket, const int* list, int n_list, int sweeps)
{
#define BXS_CD(TPC, R)                                                                              \
    {                                                                                               \
        constexpr int VV = (V < R) ? V : R;                                                         \
        k_cd<TA, TPC, R, VV><<<dim3(n_list), dim3(TPC), 0, c.stream>>>(c.insts, c.st, list, sweeps); \
        return hipGetLastError();                                                                   \
    }
    switch (bucket) {
    case 0: BXS_CD(64, 1)
    case 1: BXS_CD(64, 2)
    case 2: BXS_CD(64, 4)
    case 3: BXS_CD(64, 8)
    case 4: BXS_CD(256, 4)
    case 5: BXS_CD(256, 8)
    case 6: BXS_CD(256, 16)
    case 7: BXS_CD(512, 16)
    case 8: BXS_CD(1024, 16)
    default: return hipErrorInvalidValue;
    }
#undef BXS_CD
}

hipError_t launch_cd(const LaunchCtx& c, int bucket, const int* inst_list, int n_list, int sweeps)
{
    if (n_list <= 0) return hipSuccess;
    if (c.dtype == BXS_F32)
        return c.vec ? cd_dispatch_v<float, 4>(c, bucket, inst_list, n_list, sweeps)
                     : cd_dispatch_v<float, 1>(c, bucket, inst_list, n_list, sweeps);
    return c.vec ? cd_dispatch_v<double, 2>(c, bucket, inst_list, n_list, sweeps)
                 : cd_dispatch_v<double, 1>(c, bucket, inst_list, n_list, sweeps);
}

hipError_t launch_reduce(const LaunchCtx& c, int mode, const RItem* ritems, int n_ritems)
{
    if (n_ritems <= 0) return hipSuccess;
    dim3 grid(n_ritems), block(256);
    switch (mode) {
    case kRedResidual: k_reduce<kRedResidual><<<grid, block, 0, c.stream>>>(c.insts, c.st, ritems); break;
    case kRedFold: k_reduce<kRedFold><<<grid, block, 0, c.stream>>>(c.insts, c.st, ritems); break;
    default: k_reduce<kRedPow><<<grid, block, 0, c.stream>>>(c.insts, c.st, ritems); break;
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
    if (c.dtype == BXS_F32)
        k_colstats<float><<<dim3(n_items), dim3(256), 0, c.stream>>>(c.insts, c.st, items);
    else
        k_colstats<double><<<dim3(n_items), dim3(256), 0, c.stream>>>(c.insts, c.st, items);
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

hipError_t launch_pow_normalize(const LaunchCtx& c, int count, int last, double user_step)
{
    k_pow_normalize<<<dim3(count), dim3(256), 0, c.stream>>>(c.insts, c.st, last, user_step);
    return hipGetLastError();
}

hipError_t launch_screen(const LaunchCtx& c, int count, double eps_gap, int screening, int final_pass,
                         long long iters, int kk)
{
    k_screen<<<dim3(count), dim3(1024), 0, c.stream>>>(c.insts, c.st, c.done_counter, eps_gap, screening,
                                                        final_pass, iters, kk);
    return hipGetLastError();
}

}  // namespace bxs
