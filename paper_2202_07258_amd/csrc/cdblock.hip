// Block-sequential cyclic coordinate descent for one large instance (the
// exact form of the cyclic sweep that spreads over the chip).  The preserved
// list is cut into blocks J_0, J_1, ... of kCdbB consecutive positions and the
// blocks are taken in order.  With r^(k) the residual after blocks 0..k-1:
//   g_k = A_{J_k}^T r^(k),
//   for p in J_k ascending: c_p = g_p - sum_{q < p in J_k} (a_p^T a_q) delta_q,
//                           x_p <- Pi(x_p + c_p / ||a_p||^2), delta_p = change,
//   r^(k+1) = r^(k) - A_{J_k} delta_k.
// Since a_p^T (r - sum_{q<p} delta_q a_q) = g_p - sum_{q<p} delta_q a_p^T a_q,
// the iterates are those of the one-coordinate-at-a-time sweep (Alg. 1 with
// the CD solver of Sec. 5) up to rounding.
//
// Launch k of a sweep does two independent things at once:
//   * the row workgroups apply r^(k-1) = r^(k-2) - A_{J_{k-2}} delta_{k-2} and
//     form their rows' share of A_{J_k}^T r^(k-1);
//   * one more workgroup runs the sequential update of block k-1 from
//     g_{k-1} = A_{J_{k-1}}^T r^(k-2) - (A_{J_{k-1}}^T A_{J_{k-2}}) delta_{k-2}:
//     the cross-Gram block accounts for the previous block's update, which the
//     row workgroups apply to r only in this same launch.
// A sweep of nb blocks is nb + 2 launches.  The Gram blocks A_J^T A_J and the
// cross blocks A_{J_k}^T A_{J_{k-1}} of the preserved list are formed when the
// list has changed (a screening pass that removed columns, or a new solve).
// Every sum runs in a fixed order.
#include "dev_common.h"

#include <algorithm>
#include <type_traits>

namespace bxs {

namespace {

__device__ __forceinline__ double readlane_d(double v, int lane)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

struct double4v {
    double x, y, z, w;
};
__device__ __forceinline__ double4v ld4(const double* s, int p)
{
    return double4v{s[4 * p], s[4 * p + 1], s[4 * p + 2], s[4 * p + 3]};
}

// The Gram blocks are valid for the preserved list of this many columns (+1,
// so that 0 means none yet): the list only shrinks, keeping its order, so its
// length names it.
__device__ __forceinline__ int gram_tag(int n_active) { return n_active + 1; }

}  // namespace

// ---------------------------------------------------------------------------
// Gram blocks.  blockIdx.z = 0: gram[k] = A_{J_k}^T A_{J_k}; z = 1 (k >= 1):
// gram[nbh + k] = A_{J_k}^T A_{J_{k-1}}; both column-major B x B, element
// (a, b) at b * B + a with rows a from J_k, zero outside the blocks' sizes.
// On the FP64 matrix cores (v_mfma_f64_16x16x4_f64): grid (nbh, 4, 2), a
// 64 x 64 quadrant of a block pair per workgroup, 4 waves of 32 x 32 outputs (2 x 2 blocks of 16 x 16).
// Rows of A go through LDS 32 at a time (K-major: a fragment read is 16
// consecutive doubles per quarter-wave), promoted exactly to FP64 on load;
// the next 32 rows are loaded into registers while the current ones are
// multiplied.  Each element is the sum over the row steps, in order, of
// 4-term MFMA partial sums (deterministic for a given m).
// ---------------------------------------------------------------------------
typedef double cdb_d4 __attribute__((ext_vector_type(4)));

template <typename TA>
__global__ __launch_bounds__(256)
void k_cdb_gram_mfma(const Inst* __restrict__ insts, const State* __restrict__ st, double* __restrict__ gram, int nbh)
{
    constexpr int B = kCdbB, Q = 64, KS = 32, PAD = 2;
    const Inst& I = insts[0];
    const State& S = st[0];
    if (S.done || S.cdb_n == gram_tag(S.n_active)) return;
    const int nA = S.n_active;
    const int k = blockIdx.x, cross = blockIdx.z;
    const int p0 = k * B;
    if (p0 >= nA || (cross && k == 0)) return;
    const int bs = min(B, nA - p0);
    const int pb = cross ? p0 - B : p0, bsb = cross ? B : bs;
    const int ta = blockIdx.y >> 1, tb = blockIdx.y & 1;
    const int m = I.m;
    const long long lda = I.lda;
    const TA* __restrict__ A = reinterpret_cast<const TA*>(I.A);
    __shared__ double sA[KS][Q + PAD], sB[KS][Q + PAD];
    __shared__ int ja[Q], jb[Q];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    if (tid < Q) {
        const int qa = ta * Q + tid, qb = tb * Q + tid;
        ja[tid] = (qa < bs) ? I.idx[p0 + qa] : -1;
        jb[tid] = (qb < bsb) ? I.idx[pb + qb] : -1;
    }
    __syncthreads();
    // one row step: 2048 elements per operand, a pair of consecutive rows of
    // one column per thread and chunk (16 threads cover a column's 32 rows)
    double ra[8], rb[8];
    auto load = [&](int r0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = tid + 256 * q, col = c >> 4, rr = (c & 15) * 2;
            const int i = r0 + rr;
            const int ca = ja[col], cb = jb[col];
            const TA* pa = A + (long long)(ca < 0 ? 0 : ca) * lda + i;
            const TA* pbp = A + (long long)(cb < 0 ? 0 : cb) * lda + i;
            ra[2 * q] = (ca >= 0 && i < m) ? (double)pa[0] : 0.0;
            ra[2 * q + 1] = (ca >= 0 && i + 1 < m) ? (double)pa[1] : 0.0;
            rb[2 * q] = (cb >= 0 && i < m) ? (double)pbp[0] : 0.0;
            rb[2 * q + 1] = (cb >= 0 && i + 1 < m) ? (double)pbp[1] : 0.0;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = tid + 256 * q, col = c >> 4, rr = (c & 15) * 2;
            sA[rr][col] = ra[2 * q];
            sA[rr + 1][col] = ra[2 * q + 1];
            sB[rr][col] = rb[2 * q];
            sB[rr + 1][col] = rb[2 * q + 1];
        }
    };
    cdb_d4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[a][c] = cdb_d4{0.0, 0.0, 0.0, 0.0};
    const int kq = lane >> 4, kr = lane & 15;
    const int nk = (m + KS - 1) / KS;
    load(0);
    store();
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        if (kt + 1 < nk) load((kt + 1) * KS);
#pragma unroll
        for (int ks = 0; ks < KS / 4; ++ks) {
            double fa[2], fb[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) fa[a] = sA[ks * 4 + kq][wm * 32 + a * 16 + kr];
#pragma unroll
            for (int c = 0; c < 2; ++c) fb[c] = sB[ks * 4 + kq][wn * 32 + c * 16 + kr];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    acc[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(fb[c], fa[a], acc[a][c], 0, 0, 0);
        }
        __syncthreads();
        if (kt + 1 < nk) {
            store();
            __syncthreads();
        }
    }
    // register r of lane l holds element (row a-index l % 16, column 4 r + l / 16)
    // of its 16 x 16 block: G[gb * B + ga], rows ga from J_k
    double* __restrict__ G = gram + ((size_t)cross * nbh + k) * B * B;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int ga = ta * Q + wm * 32 + a * 16 + kr, gb = tb * Q + wn * 32 + c * 16 + 4 * r + kq;
                G[(size_t)gb * B + ga] = (ga < bs && gb < bsb) ? acc[a][c][r] : 0.0;
            }
}

// ---------------------------------------------------------------------------
// Launch k of a sweep (k = 0 .. nb + 1), 512 threads per workgroup.
//
// Workgroups 0 .. nchunks-1, kCdbRows rows each (64 rows x 8 groups):
//   k >= 2:  r -= A_{J_{k-2}} delta_{k-2} over the workgroup's rows;
//   k < nb:  pg[k & 1][chunk][q] = sum over the rows of a_{J_k[q]} r, one
//            column per 8 lanes (lane `part` takes rows part, part + 8, ...),
//            then a 3-step butterfly over the 8 lanes.
// Workgroup nchunks, for block b = k - 1 (1 <= k <= nb): stages the Gram
// block in LDS (128 KB), forms g_b from the chunk partials minus the cross
// block times delta_{b-1}, then one wave runs the in-block sequential update.
// Lane l holds c for positions l and l + 64; at step p every lane reads c_p
// with v_readlane and takes the same step, so delta_p is uniform and each lane
// updates its c values with column p of the Gram block.  delta_b goes to
// delta[b & 1] and the new x of the block's columns to x.
// ---------------------------------------------------------------------------
template <typename TA>
__global__ __launch_bounds__(512)
void k_cdb_step(const Inst* __restrict__ insts, State* __restrict__ st, int k, int nchunks, int nbh,
                double* __restrict__ pg, const double* __restrict__ gram, double* __restrict__ delta)
{
    constexpr int B = kCdbB, RW = kCdbRows;
    static_assert(B == 128 && RW == 64, "two positions per lane, 64 rows per workgroup");
    const Inst& I = insts[0];
    State& S = st[0];
    if (S.done) return;
    const int nA = S.n_active;
    const int nb = (nA + B - 1) / B;
    const int tid = threadIdx.x;
    __shared__ __align__(16) double smem[B * B + 21 * B];
    __shared__ int sj[2 * B];

    if (blockIdx.x == nchunks) {
        // ---- sequential update of block b ----
        const int b = k - 1;
        if (b < 0 || b >= nb) {
            if (k == nb + 1 && tid == 0) S.cdb_n = gram_tag(nA);  // this sweep's blocks are the current list's
            return;
        }
        // the per-step scalars first, at LDS addresses a read's immediate
        // offset reaches; the Gram block last
        double* sq = smem;                  // [B][4] x, l, u, 1 / ||a||^2
        double* sxn = sq + 4 * B;           // [B] new x of each position
        double* sg = sxn + B;               // [8][B] chunk-group sums of g
        double* sc = sg + 8 * B;            // [8][B] cross-term partials
        double* G = sc + 8 * B;             // [B][B] Gram block
        const int p0 = b * B, bs = min(B, nA - p0);
        int nn_form = 1;
        {
            // Every global read of the prologue is issued before its results
            // are used: the Gram block and the cross block as 16-byte loads,
            // the chunk partials in batches of independent loads.  Thread
            // (pair q2, group cg) covers positions 2 q2 and 2 q2 + 1; each
            // group's sums run in a fixed order.
            const int q2 = tid & 63, cg = tid >> 6, q = 2 * q2;
            const double2* __restrict__ Gb2 = reinterpret_cast<const double2*>(gram + (size_t)b * B * B);
            double2 gv[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) gv[i] = Gb2[tid + 512 * i];
            double2 t2 = make_double2(0.0, 0.0);
            if (b >= 1) {
                // the previous block is full; its delta is in delta[(b - 1) & 1]
                const double2* __restrict__ Cb2 = reinterpret_cast<const double2*>(gram + ((size_t)nbh + b) * B * B);
                const double* __restrict__ dp = delta + (size_t)((b - 1) & 1) * B;
                // a column of the cross block is read only for a position that
                // moved (late in a solve most stay on their bound)
                double2 cv[16];
                double dv[16];
#pragma unroll
                for (int i = 0; i < 16; ++i) dv[i] = dp[cg + 8 * i];
#pragma unroll
                for (int i = 0; i < 16; ++i)
                    cv[i] = (dv[i] != 0.0) ? Cb2[(cg + 8 * i) * (B / 2) + q2] : make_double2(0.0, 0.0);
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    t2.x = fma(cv[i].x, dv[i], t2.x);
                    t2.y = fma(cv[i].y, dv[i], t2.y);
                }
            }
            const double2* __restrict__ pg2 =
                reinterpret_cast<const double2*>(pg + (size_t)(b & 1) * nchunks * B) + q2;
            double2 s2 = make_double2(0.0, 0.0);
            int ch = cg;
            for (; ch + 8 * 7 < nchunks; ch += 8 * 8) {
                double2 v[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) v[i] = pg2[(size_t)(ch + 8 * i) * (B / 2)];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    s2.x += v[i].x;
                    s2.y += v[i].y;
                }
            }
            for (; ch < nchunks; ch += 8) {
                const double2 v = pg2[(size_t)ch * (B / 2)];
                s2.x += v.x;
                s2.y += v.y;
            }
            sg[cg * B + q] = s2.x;
            sg[cg * B + q + 1] = s2.y;
            sc[cg * B + q] = t2.x;
            sc[cg * B + q + 1] = t2.y;
            double2* G2 = reinterpret_cast<double2*>(G);
#pragma unroll
            for (int i = 0; i < 16; ++i) G2[tid + 512 * i] = gv[i];
            if (tid < B) {
                const bool v = tid < bs;
                const int j = v ? I.idx[p0 + tid] : 0;
                const double c2 = v ? I.cn2[j] : 0.0;
                const double lj = v ? lo_of(I.l, j) : 0.0, uj = v ? up_of(I.u, j) : HUGE_VAL;
                sj[tid] = j;
                sq[4 * tid + 0] = v ? I.x[j] : 0.0;
                sq[4 * tid + 1] = lj;
                sq[4 * tid + 2] = uj;
                sq[4 * tid + 3] = (c2 > 0.0) ? 1.0 / c2 : 0.0;
                nn_form = (lj == 0.0 && uj == HUGE_VAL) ? 1 : 0;
            }
        }
        // every position of the block has l = 0 and u = +inf (the NNLS form):
        // the projection is then max(t, 0), one operation on the step chain
        const int all_nn = __syncthreads_and(nn_form);
        if (tid >= 64) return;
        const int lane = tid, q0 = lane, q1 = lane + 64;
        auto sum8 = [&](const double* a, int qq) {
            return ((a[qq] + a[B + qq]) + (a[2 * B + qq] + a[3 * B + qq])) +
                   ((a[4 * B + qq] + a[5 * B + qq]) + (a[6 * B + qq] + a[7 * B + qq]));
        };
        double c0 = sum8(sg, q0) - sum8(sc, q0);
        double c1 = sum8(sg, q1) - sum8(sc, q1);
        // The step-to-step chain is kept to five dependent operations (four
        // for a block in the NNLS form, whose projection is max(t, 0)): c_p is
        // finished as a uniform value, c_p = c'_p - G[p-1][p] delta_{p-1},
        // where c'_p (every update up to delta_{p-2}) was read from its lane
        // one step earlier, before that lane's own update with delta_{p-1};
        // then the projected step and delta_p = x_new - x.  The lanes'
        // updates c_q -= G[p][q] delta_p and the reads run beside the chain.
        // G[p-1][p] delta_{p-1} is the same fma that lane p does, so c_p is
        // the value it would hold.  Column p of the Gram block and position
        // p's scalars are read four steps ahead into a ring of four register
        // sets (the loop is unrolled by four, so no set is copied); lane 0
        // records the four new x values of a turn in LDS.  A zero
        // column has 1 / ||a||^2 = 0 and c_p = 0: its step x + 0 is x (x stays
        // inside the box), delta = 0.
        const double x0 = sq[4 * q0], x1 = sq[4 * q1];
        auto run = [&](auto nn) {
            struct Buf {
                double g0, g1, gu;
                double4v s;
            };
            auto fetch = [&](Buf& f, int p) {
                const int pc = min(p, B - 1);
                f.g0 = G[pc * B + q0];
                f.g1 = G[pc * B + q1];
                f.gu = G[max(pc - 1, 0) * B + pc];
                f.s = ld4(sq, pc);
                // keep the reads here, ahead of the steps that use them
                __builtin_amdgcn_sched_barrier(0);
            };
            double cpo = readlane_d(c0, 0), dprev = 0.0;
            // one step: returns the new x of position p (uniform)
            auto step = [&](const Buf& f, int p, bool lo_half) {
                const double cp = fma(-f.gu, dprev, cpo);
                double xn;
                if constexpr (decltype(nn)::value) xn = fmax(f.s.x + cp * f.s.w, 0.0);
                else xn = fmin(fmax(f.s.x + cp * f.s.w, f.s.y), f.s.z);
                const double d = xn - f.s.x;
                cpo = readlane_d(lo_half ? c0 : c1, (p + 1) & 63);
                if (lo_half) c0 = fma(-f.g0, d, c0);
                c1 = fma(-f.g1, d, c1);
                dprev = d;
                return xn;
            };
            // four steps of the ring, their new x recorded by lane 0 afterwards
            auto turn = [&](Buf& fa, Buf& fb, Buf& fc, Buf& fd, int p, bool lo_half) {
                const double xa = step(fa, p, lo_half);
                fetch(fa, p + 4);
                const double xb = step(fb, p + 1, lo_half);
                fetch(fb, p + 5);
                const double xc = step(fc, p + 2, lo_half);
                fetch(fc, p + 6);
                const double xd = step(fd, p + 3, lo_half);
                fetch(fd, p + 7);
                if (lane == 0) {
                    sxn[p] = xa;
                    sxn[p + 1] = xb;
                    sxn[p + 2] = xc;
                    sxn[p + 3] = xd;
                }
            };
            auto tail = [&](Buf& fa, Buf& fb, Buf& fc, int p, int end, bool lo_half) {
                const double xa = step(fa, p, lo_half);
                const double xb = (p + 1 < end) ? step(fb, p + 1, lo_half) : 0.0;
                const double xc = (p + 2 < end) ? step(fc, p + 2, lo_half) : 0.0;
                if (lane == 0) {
                    sxn[p] = xa;
                    if (p + 1 < end) sxn[p + 1] = xb;
                    if (p + 2 < end) sxn[p + 2] = xc;
                }
            };
            Buf f0, f1, f2, f3;
            fetch(f0, 0);
            fetch(f1, 1);
            fetch(f2, 2);
            fetch(f3, 3);
            const int n0 = min(bs, 64);
            int p = 0;
            for (; p + 3 < n0; p += 4) turn(f0, f1, f2, f3, p, true);
            if (p < n0) {              // bs < 64: the block ends within this ring turn
                tail(f0, f1, f2, p, n0, true);
            } else if (bs > 64) {
                // position 64 is lane 0 of c1, already updated with delta_63
                cpo = readlane_d(c1, 0);
                dprev = 0.0;
                for (; p + 3 < bs; p += 4) turn(f0, f1, f2, f3, p, false);
                if (p < bs) tail(f0, f1, f2, p, bs, false);
            }
        };
        if (all_nn) run(std::true_type{});
        else run(std::false_type{});
        const double xo0 = (q0 < bs) ? sxn[q0] : x0, xo1 = (q1 < bs) ? sxn[q1] : x1;
        // delta = x_new - x, the same subtraction as in the step
        const double d0 = xo0 - x0, d1 = xo1 - x1;
        double* __restrict__ db = delta + (size_t)(b & 1) * B;
        if (q0 < bs) {
            db[q0] = d0;
            if (d0 != 0.0) I.x[sj[q0]] = xo0;
        }
        if (q1 < bs) {
            db[q1] = d1;
            if (d1 != 0.0) I.x[sj[q1]] = xo1;
        }
        return;
    }

    // ---- row workgroup: apply block k-2's update, form block k's partials ----
    const bool upd = k >= 2 && k - 2 < nb;
    const bool dot = k < nb;
    if (!upd && !dot) return;
    const int m = I.m;
    const long long lda = I.lda;
    const TA* __restrict__ A = reinterpret_cast<const TA*>(I.A);
    double* sdl = smem;                 // [B] delta_{k-2}
    double* sr = sdl + B;               // [RW] updated residual rows
    double* sp = sr + RW;               // [8][RW] update partials
    int* sip = sj;                      // [B] columns of block k-2
    int* sic = sj + B;                  // [B] columns of block k
    const int qs = upd ? min(B, nA - (k - 2) * B) : 0;
    const int bs = dot ? min(B, nA - k * B) : 0;
    if (tid < B) {
        sip[tid] = (tid < qs) ? I.idx[(k - 2) * B + tid] : 0;
        sdl[tid] = (tid < qs) ? delta[(size_t)(k & 1) * B + tid] : 0.0;
    } else if (tid < 2 * B) {
        const int t = tid - B;
        sic[t] = (t < bs) ? I.idx[k * B + t] : 0;
    }
    const int r0 = blockIdx.x * RW;
    const int row = tid & (RW - 1), grp = tid >> 6;
    const int i = r0 + row;
    const bool rok = i < m;
    const int ic = rok ? i : 0;
    __syncthreads();
    double rv = rok ? I.r[i] : 0.0;
    // Both phases' reads of A are issued before either is used (the dot
    // phase reads A_{J_k}, which does not depend on the residual update).
    const int part = tid & 7, slot = tid >> 3;
    double av[B / 8];                   // update: row i, columns grp + 8 t of block k-2
    double bv[2][8];                    // dot: column slot + 64 h, rows part + 8 e
    if (upd && qs == B) {               // every block but the last; columns that did not move are not read
#pragma unroll
        for (int t = 0; t < B / 8; ++t)
            av[t] = (sdl[grp + 8 * t] != 0.0) ? (double)A[(long long)sip[grp + 8 * t] * lda + ic] : 0.0;
    }
    if (dot) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const long long base = (long long)sic[min(slot + 64 * h, bs - 1)] * lda;
#pragma unroll
            for (int e = 0; e < 8; ++e) bv[h][e] = (double)A[base + min(r0 + part + 8 * e, m - 1)];
        }
    }
    if (upd) {
        double s = 0.0;
        if (qs == B) {
#pragma unroll
            for (int t = 0; t < B / 8; ++t) s = fma(av[t], sdl[grp + 8 * t], s);
        } else {
#pragma unroll 4
            for (int q = grp; q < qs; q += 8) s = fma((double)A[(long long)sip[q] * lda + ic], sdl[q], s);
        }
        sp[grp * RW + row] = s;
        __syncthreads();
        if (grp == 0) {
            const double* t = sp + row;
            rv -= ((t[0] + t[RW]) + (t[2 * RW] + t[3 * RW])) + ((t[4 * RW] + t[5 * RW]) + (t[6 * RW] + t[7 * RW]));
            if (rok) I.r[i] = rv;
        }
    }
    if (!dot) return;
    if (grp == 0) sr[row] = rok ? rv : 0.0;
    __syncthreads();
    double* __restrict__ pgk = pg + (size_t)(k & 1) * nchunks * B + (size_t)blockIdx.x * B;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int q = slot + 64 * h;
        double v = 0.0;
#pragma unroll
        for (int e = 0; e < 8; ++e) v = fma(bv[h][e], sr[part + 8 * e], v);
        v += dpp_move<0xB1, 0xF>(v);     // quad_perm [1,0,3,2]
        v += dpp_move<0x4E, 0xF>(v);     // quad_perm [2,3,0,1]
        v += dpp_move<0x141, 0xF>(v);    // row_half_mirror: the two quads of 8 lanes
        if (part == 0 && q < bs) pgk[q] = v;
    }
}

size_t cdb_gram_doubles(long n) { return (size_t)2 * ((n + kCdbB - 1) / kCdbB) * kCdbB * kCdbB; }
size_t cdb_pg_doubles(long m) { return (size_t)2 * ((m + kCdbRows - 1) / kCdbRows) * kCdbB; }

hipError_t launch_cdb_gram(const LaunchCtx& c, long n, double* gram)
{
    const int nbh = (int)((n + kCdbB - 1) / kCdbB);
    const dim3 g((unsigned)nbh, 4, 2), b(256);
    if (c.dtype == BXS_BF16) k_cdb_gram_mfma<__bf16><<<g, b, 0, c.stream>>>(c.insts, c.st, gram, nbh);
    else if (c.dtype == BXS_F32) k_cdb_gram_mfma<float><<<g, b, 0, c.stream>>>(c.insts, c.st, gram, nbh);
    else k_cdb_gram_mfma<double><<<g, b, 0, c.stream>>>(c.insts, c.st, gram, nbh);
    return hipGetLastError();
}

// One sweep: launches 0 .. nb + 1 with nb = ceil(n_bound / B), n_bound an
// upper bound of the device's preserved-list length (the list only shrinks;
// launches past the device's block count return at once).  n is the
// problem's column count, which sets the layout of the cross blocks.
hipError_t launch_cdb_sweep(const LaunchCtx& c, long m, long n, long n_bound, double* pg, const double* gram,
                            double* delta)
{
    const int nbh = (int)((n + kCdbB - 1) / kCdbB);
    const int nbl = (int)((std::min(n, std::max(n_bound, 0L)) + kCdbB - 1) / kCdbB);
    const int chunks = (int)((m + kCdbRows - 1) / kCdbRows);
    for (int k = 0; k <= nbl + 1; ++k) {
        if (c.dtype == BXS_BF16)
            k_cdb_step<__bf16><<<chunks + 1, 512, 0, c.stream>>>(c.insts, c.st, k, chunks, nbh, pg, gram, delta);
        else if (c.dtype == BXS_F32)
            k_cdb_step<float><<<chunks + 1, 512, 0, c.stream>>>(c.insts, c.st, k, chunks, nbh, pg, gram, delta);
        else
            k_cdb_step<double><<<chunks + 1, 512, 0, c.stream>>>(c.insts, c.st, k, chunks, nbh, pg, gram, delta);
    }
    return hipGetLastError();
}

}  // namespace bxs
