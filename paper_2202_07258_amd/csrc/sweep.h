// Column-sweep kernel of the boxscreen library (gfx950): the fused
// matrix-vector products of the projected-gradient step, the correlations
// A^T r with the screening partials, the fold of screened columns and the
// products with A A^T.  Included by the translation units that instantiate
// its variants (sweep_*.hip).
#pragma once

#include "dev_common.h"

#include <type_traits>

namespace bxs {

// ---------------------------------------------------------------------------
// Column sweep.  One workgroup = one work item (instance, block of cb
// consecutive positions of the preserved-set list, or of the fold list).
// NG groups of TPC threads each take every NG-th column of the item, CBI
// columns per round; thread L of a group owns rows {(k*TPC + L)*V + e},
// k < R/V, e < V, and keeps those residual rows and its share of the partial
// product in registers.  Columns of the next round are loaded before the
// current round's dot products are reduced (software pipeline), so a barrier
// never drains the memory queue.
//
// kModePGS reads every column once for both the screening test at the
// current iterate x (correlations g = A^T r and the per-column gap terms)
// and the next projected-gradient step from x, which needs the same g: the
// step is taken ahead of the test.  x is kept in xs and the new residual goes
// to r2, so the screening pass can either keep the step (nothing screened,
// no stop) or return to x.  kModePG1 (the first iteration of the next pass)
// then returns at once; so do the two-pass forms' kernels launched with
// first = 1.  For the shapes too large to keep the residual and the partial
// product in registers the residual is staged in LDS and the products run as
// a dot pass and a product pass (two_pass_shape).
// ---------------------------------------------------------------------------
template <typename TA, int TPC, int NG, int R, int V, int CBI, int PD, int MODE>
__global__ __launch_bounds__(TPC * NG)
void k_sweep(const Inst* __restrict__ insts, State* __restrict__ st, const Item* __restrict__ items, int first,
             int single)
{
    constexpr int RO = R / V;
    constexpr bool SCR = (MODE == kModeCorr || MODE == kModePGS || MODE == kModeStepS);  // screening at x
    constexpr bool CPM = (MODE == kModeCP || MODE == kModeStepCP);   // Chambolle-Pock: v in r2
    constexpr bool STP = (MODE == kModePG || MODE == kModePG1 || MODE == kModePGS || MODE == kModeStep ||
                          MODE == kModeStepS || CPM);
    constexpr bool KEEPX = (MODE == kModePGS || MODE == kModeStepS);  // x kept in xs
    constexpr bool DOT = (STP || SCR || MODE == kModePow || MODE == kModePowG);
    constexpr bool ACC = !(MODE == kModeCorr || MODE == kModeStep || MODE == kModeStepS || MODE == kModePowG ||
                           MODE == kModeStepCP);
    constexpr bool COEF = (MODE == kModeAx || MODE == kModeAg || MODE == kModeAxS);  // partial += A c, c staged
    // residual rows staged in LDS (shapes too large for it to stay in registers)
    constexpr bool RLDS = DOT && two_pass_shape(TPC, R);
    constexpr int NW = TPC / 64;
    static_assert(R % V == 0, "rows per thread must be a multiple of the vector width");
    static_assert(TPC % 64 == 0, "a column group is whole waves");
    static_assert(dot_depth(TPC, R) <= (int)kDotDepth, "correlation sums deeper than the screening margin assumes");

    // a single instance's items are {0, blockIdx.x}: no table load on the
    // critical path of the launch
    const Item it = single ? Item{0, (int)blockIdx.x} : items[blockIdx.x];
    const Inst& I = insts[it.inst];
    State& S = st[it.inst];
    if (S.done) return;
    if ((MODE == kModePG1 || ((MODE == kModeStep || MODE == kModeAx) && first)) && S.ahead) return;
    const int nlist = (MODE == kModeFold) ? S.n_fold : S.n_active;
    const int cb = (MODE == kModeFold) ? S.cb_fold : S.cb;
    const int pos0 = it.t * cb;
    if (pos0 >= nlist) return;
    const int pos1 = min(pos0 + cb, nlist);

    const int tid = threadIdx.x;
    const int grp = (NG > 1) ? tid / TPC : 0;
    const int L = (NG > 1) ? tid % TPC : tid;
    const int lane = tid & 63;
    const int wig = L >> 6;                       // wave index inside the group
    const int myc = col_of_lane<CBI>(lane);       // column this lane finalises
    const bool owner = (lane & ((64 >> Log2C<CBI>::v) - 1)) == 0 && wig == 0;
    const int m = I.m;
    const long long lda = I.lda;
    const TA* __restrict__ A = reinterpret_cast<const TA*>(I.A);
    const int* __restrict__ list = (MODE == kModeFold) ? I.fidx : I.idx;
    // PG ascends along A^T r; Chambolle-Pock descends along A^T v
    const double eta = STP ? (CPM ? -S.step : S.step) : 0.0;
    const double* __restrict__ rsrc = CPM ? I.r2 : I.r;
    // Huber fidelity: the gradient and the dual point use psi(r) =
    // clip(r, -delta, delta) (delta = +inf for least squares: r itself)
    constexpr bool HUB = (STP || SCR) && !CPM;
    const double hub = HUB ? I.hub : 0.0;
    const double tnorm_c = SCR ? S.tnorm : 0.0;

    bool rowok[R];
#pragma unroll
    for (int k = 0; k < RO; ++k)
#pragma unroll
        for (int e = 0; e < V; ++e) rowok[k * V + e] = (k * TPC + L) * V + e < m;
    double rl[(DOT && !RLDS) ? R : 1];
    __shared__ double s_r[RLDS ? TPC * R : 1];
    auto rv = [&](int k) -> double {
        if constexpr (RLDS) return s_r[k * TPC + L]; else return rl[k];
    };
    if constexpr (DOT) {
#pragma unroll
        for (int k = 0; k < RO; ++k)
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const int row = (k * TPC + L) * V + e;
                double v = (row < m) ? rsrc[row] : 0.0;
                if constexpr (HUB) v = fmin(fmax(v, -hub), hub);
                if constexpr (RLDS) s_r[(k * V + e) * TPC + L] = v; else rl[k * V + e] = v;
            }
    }
    // CORR: bound on ||r|| (every workgroup sums the same registers in the
    // same order, so all items of an instance agree bit for bit) and the
    // per-column screening quantities accumulated by the owner lanes.
    double rnorm_c = 0.0;
    double a_mass = 0.0, a_tv = 1.0, a_emax = 0.0, a_inf = 0.0, a_gap = 0.0, a_z = -__builtin_inf();
    if constexpr (SCR) {
        double sq = 0.0;
#pragma unroll
        for (int k = 0; k < R; ++k) sq = fma(rv(k), rv(k), sq);
        sq = wave_sum(sq);
        __shared__ double s_sq[(TPC * NG) / 64];
        if (lane == 0) s_sq[tid >> 6] = sq;
        __syncthreads();
        double tot = 0.0;
        if (NG == 1) {
#pragma unroll
            for (int w = 0; w < (TPC * NG) / 64; ++w) tot += s_sq[w];
        } else {
#pragma unroll
            for (int w = 0; w < TPC / 64; ++w) tot += s_sq[w];   // group 0 holds every row once
        }
        rnorm_c = sqrt(tot * (1.0 + gamma_k((double)R + 24.0))) * (1.0 + 2.0 * kUnit);
    }
    double p[ACC ? R : 1];
    double p2[(MODE == kModeFold) ? R : 1];
#pragma unroll
    for (int k = 0; k < (ACC ? R : 1); ++k) p[k] = 0.0;
#pragma unroll
    for (int k = 0; k < ((MODE == kModeFold) ? R : 1); ++k) p2[k] = 0.0;

    __shared__ double red[2][NG][(NW > 1) ? NW : 1][CBI];
    int buf = 0;

    // Two column buffers used in ping-pong: while one round is reduced and
    // applied, the next round's columns are already in flight.
    //  DOT modes keep the scalars of the lane's own column (x, l, u);
    //  AX / FOLD keep the coefficient of every column of the round.
    constexpr int NC1 = DOT ? 1 : CBI;
    constexpr int NC2 = (MODE == kModeFold) ? CBI : 1;
    TA a0[CBI][R], a1[CBI][R];
    int j0 = 0, j1 = 0;
    bool v0 = false, v1 = false;
    double x0 = 0.0, l0 = 0.0, u0 = 0.0, x1 = 0.0, l1 = 0.0, u1 = 0.0;
    double c10[NC1], c20[NC2], c11[NC1], c21[NC2];

    // Stage the item's column indices and per-column scalars in LDS once, so
    // that a round's column loads never wait on a dependent index load.
    __shared__ int s_j[kCbMax];
    __shared__ double s_x[(STP || SCR || COEF || MODE == kModeFold) ? kCbMax : 1];
    __shared__ double s_l[(STP || SCR || MODE == kModeFold) ? kCbMax : 1];
    __shared__ double s_u[(STP || SCR) ? kCbMax : 1];
    __shared__ double s_cn[SCR ? kCbMax : 1];
    __shared__ double s_w[SCR ? kCbMax : 1];
    for (int k = tid; k < pos1 - pos0; k += TPC * NG) {
        const int q = pos0 + k;
        const int j = list[q];
        s_j[k] = j;
        if constexpr (SCR) {
            s_x[k] = I.x[j];
            s_l[k] = lo_of(I.l, j);
            s_u[k] = up_of(I.u, j);
            s_cn[k] = I.cn[j];
            s_w[k] = I.w[j];
        } else if constexpr (STP) {
            s_x[k] = I.x[j];
            s_l[k] = lo_of(I.l, j);
            s_u[k] = up_of(I.u, j);
        } else if constexpr (MODE == kModeAx) {
            s_x[k] = I.x[j];
        } else if constexpr (MODE == kModeAg) {
            s_x[k] = I.g[j];
        } else if constexpr (MODE == kModeAxS) {
            s_x[k] = I.xs[j];
        } else if constexpr (MODE == kModeFold) {
            s_x[k] = I.fval[q];
            s_l[k] = I.fdx[q];
        }
    }
    __syncthreads();

    auto load_round = [&](int rs, TA (&a)[CBI][R], int& jo, bool& vo, double& xo, double& lo, double& uo,
                          double (&c1)[NC1], double (&c2)[NC2]) {
#pragma unroll
        for (int c = 0; c < CBI; ++c) {
            const int q = rs + c * NG + grp;
            const bool vv = q < pos1;
            // a slot past the item's end reads the item's first column; its
            // dot product is discarded and its update coefficient is 0
            const int jj = s_j[vv ? q - pos0 : 0];
            const TA* col = A + (long long)jj * lda;
#pragma unroll
            for (int k = 0; k < RO; ++k) {
                TA tmp[V];
                load_pack_nb<TA, V>(col, (k * TPC + L) * V, m, tmp);
#pragma unroll
                for (int e = 0; e < V; ++e) a[c][k * V + e] = tmp[e];
            }
            if constexpr (COEF) {
                c1[c] = vv ? s_x[q - pos0] : 0.0;
            } else if constexpr (MODE == kModeFold) {
                c1[c] = vv ? s_x[q - pos0] : 0.0;
                c2[c] = vv ? s_l[q - pos0] : 0.0;
            }
        }
        if constexpr (DOT) {
            // jo: slot of the lane's own column in the staged arrays
            const int q = rs + myc * NG + grp;
            vo = q < pos1;
            jo = vo ? q - pos0 : 0;
            if constexpr (STP) {
                xo = vo ? s_x[jo] : 0.0;
                lo = vo ? s_l[jo] : 0.0;
                uo = vo ? s_u[jo] : 0.0;
            }
        }
    };

    auto compute_round = [&](const TA (&a)[CBI][R], int jo, bool vo, double xo, double lo, double uo,
                             const double (&c1)[NC1], const double (&c2)[NC2]) {
        if constexpr (DOT) {
            double d[CBI];
#pragma unroll
            for (int c = 0; c < CBI; ++c) {
                double s = 0.0;
#pragma unroll
                for (int k = 0; k < R; ++k) s = fma(rowok[k] ? (double)a[c][k] : 0.0, rv(k), s);
                d[c] = s;
            }
            double tot = wave_reduce_scatter<CBI>(d, lane);
            if constexpr (NW > 1) {
                if ((lane & ((64 >> Log2C<CBI>::v) - 1)) == 0) red[buf][grp][wig][myc] = tot;
                __syncthreads();
                double s = 0.0;
#pragma unroll
                for (int w = 0; w < NW; ++w) s += red[buf][grp][w][myc];
                tot = s;
                buf ^= 1;
            }
            double cown = 0.0;
            if (vo) {
                if constexpr (STP) {
                    const double xn = fmin(fmax(xo + eta * tot, lo), uo);
                    // Chambolle-Pock multiplies A by the extrapolated point 2 x+ - x
                    cown = CPM ? 2.0 * xn - xo : xn;
                    if (owner) gstore(I.x + s_j[jo], xn);
                    if (KEEPX && owner) gstore(I.xs + s_j[jo], xo);
                    if (MODE == kModeStepCP && owner) gstore(I.xs + s_j[jo], cown);
                }
                if constexpr (SCR) {
                    if (owner) {
                        gstore(I.g + s_j[jo], tot);
                        // screening quantities of this column at eps = 0
                        const int k = jo;
                        const double cnj = s_cn[k], wj = s_w[k], xj = s_x[k], lj = s_l[k], uj = s_u[k];
                        const double gm = gamma_k(kDotDepth);
                        const double gw = gamma_k((double)(m / 64) + 8.0);
                        a_mass = fma(fabs(xj), cnj, a_mass);
                        const double ej = cnj * gm * rnorm_c + 4.0 * kUnit * fabs(tot);
                        double term = (xj - lj) * fmax(ej - tot, 0.0);
                        double zs = -(tot + ej);
                        if (isinf(uj)) {
                            a_inf = 1.0;
                            const double ewj = gw * cnj * tnorm_c;
                            if (!(wj + ewj < 0.0)) a_tv = 0.0;
                            else a_emax = fmax(a_emax, fmax(tot + cnj * gm * rnorm_c, 0.0) / (-wj - ewj));
                        } else {
                            term += (uj - xj) * fmax(tot + ej, 0.0);
                            zs = fmax(zs, tot - ej);
                        }
                        a_gap += term;
                        if (cnj > 0.0) a_z = fmax(a_z, zs / cnj);
                    }
                }
                if constexpr (MODE == kModePow) cown = tot;
                if constexpr (MODE == kModePowG) {
                    if (owner) gstore(I.g + s_j[jo], tot);
                }
            }
            if constexpr (ACC) {
#pragma unroll
                for (int c = 0; c < CBI; ++c) {
                    const double cf = __shfl(cown, lane_of_col<CBI>(c), 64);
#pragma unroll
                    for (int k = 0; k < R; ++k) p[k] = fma((double)opaque(a[c][k]), cf, p[k]);
                }
            }
        } else {
#pragma unroll
            for (int c = 0; c < CBI; ++c)
#pragma unroll
                for (int k = 0; k < R; ++k) p[k] = fma((double)a[c][k], c1[c], p[k]);
            if constexpr (MODE == kModeFold) {
#pragma unroll
                for (int c = 0; c < CBI; ++c)
#pragma unroll
                    for (int k = 0; k < R; ++k) p2[k] = fma((double)a[c][k], c2[c], p2[k]);
            }
        }
    };

    constexpr int STEP = NG * CBI;
    if constexpr (PD == 1) {
        // prefetch distance one round: two buffers.  Every compute that has a
        // next round is preceded, on every path, by that round's loads, so
        // the wait before it leaves the prefetch in flight; the last round of
        // the item leaves the loop through its own exit.
        load_round(pos0, a0, j0, v0, x0, l0, u0, c10, c20);
        int rs = pos0;
        while (true) {
            if (rs + STEP >= pos1) {
                compute_round(a0, j0, v0, x0, l0, u0, c10, c20);
                break;
            }
            load_round(rs + STEP, a1, j1, v1, x1, l1, u1, c11, c21);
            compute_round(a0, j0, v0, x0, l0, u0, c10, c20);
            rs += STEP;
            if (rs + STEP >= pos1) {
                compute_round(a1, j1, v1, x1, l1, u1, c11, c21);
                break;
            }
            load_round(rs + STEP, a0, j0, v0, x0, l0, u0, c10, c20);
            compute_round(a1, j1, v1, x1, l1, u1, c11, c21);
            rs += STEP;
        }
    } else {
        // prefetch distance two rounds: three buffers in rotation
        TA a2[CBI][R];
        int j2 = 0;
        bool v2 = false;
        double x2 = 0.0, l2 = 0.0, u2 = 0.0;
        double c12[NC1], c22[NC2];
        load_round(pos0, a0, j0, v0, x0, l0, u0, c10, c20);
        if (pos0 + STEP < pos1) load_round(pos0 + STEP, a1, j1, v1, x1, l1, u1, c11, c21);
        for (int rs = pos0; rs < pos1; rs += 3 * STEP) {
            if (rs + 2 * STEP < pos1) load_round(rs + 2 * STEP, a2, j2, v2, x2, l2, u2, c12, c22);
            compute_round(a0, j0, v0, x0, l0, u0, c10, c20);
            if (rs + STEP >= pos1) break;
            if (rs + 3 * STEP < pos1) load_round(rs + 3 * STEP, a0, j0, v0, x0, l0, u0, c10, c20);
            compute_round(a1, j1, v1, x1, l1, u1, c11, c21);
            if (rs + 2 * STEP >= pos1) break;
            if (rs + 4 * STEP < pos1) load_round(rs + 4 * STEP, a1, j1, v1, x1, l1, u1, c11, c21);
            compute_round(a2, j2, v2, x2, l2, u2, c12, c22);
        }
    }

    if constexpr (SCR) {
        // combine the owner lanes' screening quantities over the workgroup
        constexpr int NWB = (TPC * NG) / 64;
        __shared__ double s_red[6][NWB];
        double vals[6] = {a_mass, a_tv, a_emax, a_inf, a_gap, a_z};
        vals[0] = wave_sum(vals[0]);
        vals[1] = wave_min(vals[1]);
        vals[2] = wave_max(vals[2]);
        vals[3] = wave_max(vals[3]);
        vals[4] = wave_sum(vals[4]);
        vals[5] = wave_max(vals[5]);
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < 6; ++k) s_red[k][tid >> 6] = vals[k];
        }
        __syncthreads();
        if (tid == 0) {
            double r0 = 0.0, r1 = 1.0, r2 = 0.0, r3 = 0.0, r4 = 0.0, r5 = -__builtin_inf();
            for (int w = 0; w < NWB; ++w) {
                r0 += s_red[0][w]; r1 = fmin(r1, s_red[1][w]); r2 = fmax(r2, s_red[2][w]);
                r3 = fmax(r3, s_red[3][w]); r4 += s_red[4][w]; r5 = fmax(r5, s_red[5][w]);
            }
            double* o = I.iscal + (size_t)it.t * kItemScalars;
            o[kIsMass] = r0; o[kIsTv] = r1; o[kIsEmax] = r2; o[kIsHasInf] = r3; o[kIsGap0] = r4; o[kIsZmax0] = r5;
        }
    }
    if constexpr (!ACC) return;

    // combine the NG groups' partial products (fixed order) and store
    if constexpr (NG > 1) {
        __shared__ double comb[(NG > 1) ? (NG - 1) * TPC * R : 1];
        if (grp > 0) {
#pragma unroll
            for (int k = 0; k < R; ++k) comb[((grp - 1) * R + k) * TPC + L] = p[k];
        }
        __syncthreads();
        if (grp == 0) {
#pragma unroll
            for (int g2 = 1; g2 < NG; ++g2)
#pragma unroll
                for (int k = 0; k < R; ++k) p[k] += comb[((g2 - 1) * R + k) * TPC + L];
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
            if (row < m) gstore(out + row, p[k * V + e]);
        }
    if constexpr (MODE == kModeFold) {
        double* __restrict__ out2 = I.part2 + (size_t)it.t * m;
#pragma unroll
        for (int k = 0; k < RO; ++k)
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const int row = (k * TPC + L) * V + e;
                if (row < m) gstore(out2 + row, p2[k * V + e]);
            }
    }
}

template <typename TA, int V, int TPC, int NG, int R, int CBI, int PD>
static hipError_t sweep_launch_t(const LaunchCtx& c, int mode, const Item* items, int n_items, int first)
{
    constexpr int VV = (V < R) ? V : R;
    dim3 grid(n_items), block(TPC * NG);
#define BXS_SW(MD) k_sweep<TA, TPC, NG, R, VV, CBI, PD, MD><<<grid, block, 0, c.stream>>>(c.insts, c.st, items, first, c.single)
    // the fused forms are built only for shapes that hold them in registers,
    // the two-pass forms only for the others
    constexpr bool TWO = two_pass_shape(TPC, R);
    switch (mode) {
    case kModeCorr: BXS_SW(kModeCorr); break;
    case kModeAx: BXS_SW(kModeAx); break;
    case kModeFold: BXS_SW(kModeFold); break;
    case kModePG: if constexpr (!TWO) { BXS_SW(kModePG); break; } else { return hipErrorInvalidValue; }
    case kModePG1: if constexpr (!TWO) { BXS_SW(kModePG1); break; } else { return hipErrorInvalidValue; }
    case kModePow: if constexpr (!TWO) { BXS_SW(kModePow); break; } else { return hipErrorInvalidValue; }
    case kModePGS: if constexpr (!TWO) { BXS_SW(kModePGS); break; } else { return hipErrorInvalidValue; }
    case kModeCP: if constexpr (!TWO) { BXS_SW(kModeCP); break; } else { return hipErrorInvalidValue; }
    case kModeStepCP: if constexpr (TWO) { BXS_SW(kModeStepCP); break; } else { return hipErrorInvalidValue; }
    case kModeAxS: if constexpr (TWO) { BXS_SW(kModeAxS); break; } else { return hipErrorInvalidValue; }
    case kModeStep: if constexpr (TWO) { BXS_SW(kModeStep); break; } else { return hipErrorInvalidValue; }
    case kModeStepS: if constexpr (TWO) { BXS_SW(kModeStepS); break; } else { return hipErrorInvalidValue; }
    case kModePowG: if constexpr (TWO) { BXS_SW(kModePowG); break; } else { return hipErrorInvalidValue; }
    case kModeAg: if constexpr (TWO) { BXS_SW(kModeAg); break; } else { return hipErrorInvalidValue; }
    default: return hipErrorInvalidValue;
    }
#undef BXS_SW
    return hipGetLastError();
}

// The sweep variants of one element type and load width, split into NPART
// translation units (variant id modulo NPART) that compile in parallel.
template <typename TA, int V, int NPART, int PART>
hipError_t sweep_dispatch_part(const LaunchCtx& c, int variant, int mode, const Item* items, int n_items, int first)
{
    switch (variant) {
#define BXS_V(ID, TPC, NG, R, CBI, PD)                                                         \
    case ID:                                                                                   \
        if constexpr (ID % NPART == PART)                                                      \
            return sweep_launch_t<TA, V, TPC, NG, R, CBI, PD>(c, mode, items, n_items, first); \
        else                                                                                   \
            return hipErrorInvalidValue;
    BXS_SWEEP_VARIANTS(BXS_V)
#undef BXS_V
    default: return hipErrorInvalidValue;
    }
}

}  // namespace bxs
