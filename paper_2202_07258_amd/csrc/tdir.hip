// Translation directions for the dual update of the non-negative / mixed
// problems computed by the library (Sec. 4.2, Prop. 2 and Sec. 5.1, Fig. 2):
//
//   BXS_T_NEG_MEAN_COLUMN       t = -(1/n) sum_k a_k / ||a_k||
//   BXS_T_NEG_MOST_CORRELATED   t = -a_+ / ||a_+||
//   BXS_T_NEG_LEAST_CORRELATED  t = -a_- / ||a_-||
//
//   BXS_T_NORMAL_EQUATIONS      t = A v with A^T A v = -1        (Prop. 2, case 1)
//
// where a_+ (a_-) is the column whose summed correlation with all other
// columns, score_j = sum_{k != j} a_j^T a_k / (||a_j|| ||a_k||), is largest
// (smallest); ties go to the smallest index.  For a tall matrix of full
// column rank, A^T t = -1 < 0 makes t interior (case 1); v comes from
// conjugate gradients on the normal equations (FP64, fixed-order sums),
// run until ||A^T A v + 1||_2 <= 1e-11 sqrt(n) or 2000 iterations.  A negative combination of the
// columns is interior for an orthogonal matrix (Prop. 2, case 2), -a_j is
// interior when the j-th column of A^T A is positive (case 4); whether the
// choice is interior for the given A is checked by the solve like any t.
//
// One instance: the normalised column sum s = sum_k a_k / ||a_k|| by chunks
// of 128 columns (row-parallel, coalesced) and a fixed-order sum of the
// chunks, the scores a_j^T s / ||a_j|| - 1 (one wave per column), and the
// pick.  ||a_k|| is the column statistics' rigorous norm bound (the run
// recomputes them, and w = A^T t, after t is set).
#include "dev_common.h"

#include <algorithm>

namespace bxs {

constexpr int kTdChunk = 128;

template <typename TA>
__global__ __launch_bounds__(256)
void k_tdir_colsum(const Inst* __restrict__ insts, double* __restrict__ partial)
{
    const Inst& I = insts[0];
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int c = blockIdx.y;
    const int m = I.m, n = I.n;
    if (i >= m) return;
    const TA* __restrict__ A = reinterpret_cast<const TA*>(I.A);
    const int j0 = c * kTdChunk, j1 = min(j0 + kTdChunk, n);
    double s = 0.0;
    for (int j = j0; j < j1; ++j) {
        const double cn = I.cn[j];
        if (cn > 0.0) s += (double)A[(long long)j * I.lda + i] / cn;
    }
    partial[(long long)c * m + i] = s;
}

__global__ __launch_bounds__(256)
void k_tdir_rowsum(const Inst* __restrict__ insts, const double* __restrict__ partial, int chunks,
                   double* __restrict__ s)
{
    const int m = insts[0].m;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    double v = 0.0;
    for (int c = 0; c < chunks; ++c) v += partial[(long long)c * m + i];
    s[i] = v;
}

template <typename TA>
__global__ __launch_bounds__(256)
void k_tdir_score(const Inst* __restrict__ insts, const double* __restrict__ s, double* __restrict__ score)
{
    const Inst& I = insts[0];
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (j >= I.n) return;
    const TA* __restrict__ col = reinterpret_cast<const TA*>(I.A) + (long long)j * I.lda;
    double d = 0.0;
    for (int i = lane; i < I.m; i += 64) d = fma((double)col[i], s[i], d);
    d = wave_sum(d);
    if (lane == 0) {
        const double cn = I.cn[j];
        // the k = j term of the sum is ||a_j||^2 / ||a_j||^2 = 1
        score[j] = (cn > 0.0) ? d / cn - I.cn2[j] / (cn * cn) : 0.0;
    }
}

// One workgroup: argmax / argmin of the scores (smallest index on ties),
// then t; choice 1 writes -s / n.  *picked receives the column index (-1 for
// the mean column).
template <typename TA>
__global__ __launch_bounds__(1024)
void k_tdir_pick(const Inst* __restrict__ insts, const double* __restrict__ s, const double* __restrict__ score,
                 int choice, double* __restrict__ t, int* __restrict__ picked)
{
    const Inst& I = insts[0];
    const int m = I.m, n = I.n, tid = threadIdx.x;
    __shared__ double sv[16];
    __shared__ int si[16];
    __shared__ int jstar;
    if (choice == BXS_T_NEG_MEAN_COLUMN) {
        for (int i = tid; i < m; i += 1024) t[i] = -s[i] / (double)n;
        if (tid == 0) *picked = -1;
        return;
    }
    const bool most = choice == BXS_T_NEG_MOST_CORRELATED;
    double best = most ? -__builtin_inf() : __builtin_inf();
    int bj = 0x7fffffff;
    for (int j = tid; j < n; j += 1024) {
        const double v = score[j];
        if ((most ? v > best : v < best) || (v == best && j < bj)) { best = v; bj = j; }
    }
    // wave, then block argmax / argmin with index tie-break
    for (int off = 32; off >= 1; off >>= 1) {
        const double ov = __shfl_xor(best, off, 64);
        const int oj = __shfl_xor(bj, off, 64);
        if ((most ? ov > best : ov < best) || (ov == best && oj < bj)) { best = ov; bj = oj; }
    }
    if ((tid & 63) == 0) { sv[tid >> 6] = best; si[tid >> 6] = bj; }
    __syncthreads();
    if (tid == 0) {
        double b = sv[0];
        int jj = si[0];
        for (int w = 1; w < 16; ++w)
            if ((most ? sv[w] > b : sv[w] < b) || (sv[w] == b && si[w] < jj)) { b = sv[w]; jj = si[w]; }
        jstar = jj;
        *picked = jj;
    }
    __syncthreads();
    const int j = jstar;
    const TA* __restrict__ col = reinterpret_cast<const TA*>(I.A) + (long long)j * I.lda;
    const double cn = I.cn[j];
    for (int i = tid; i < m; i += 1024) t[i] = (cn > 0.0) ? -(double)col[i] / cn : -1.0;
}

// --- Prop. 2, case 1: conjugate gradients on A^T A v = -1 -------------------
// w = A p by chunks of 128 columns (then k_tdir_rowsum), q = A^T w one wave
// per column, and the vector updates in one workgroup.

template <typename TA>
__global__ __launch_bounds__(256)
void k_ne_colsum(const Inst* __restrict__ insts, const double* __restrict__ p, double* __restrict__ partial)
{
    const Inst& I = insts[0];
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int c = blockIdx.y;
    const int m = I.m, n = I.n;
    if (i >= m) return;
    const TA* __restrict__ A = reinterpret_cast<const TA*>(I.A);
    const int j0 = c * kTdChunk, j1 = min(j0 + kTdChunk, n);
    double s = 0.0;
    for (int j = j0; j < j1; ++j) s = fma((double)A[(long long)j * I.lda + i], p[j], s);
    partial[(long long)c * m + i] = s;
}

__global__ void k_set_int(int* __restrict__ p, int v) { *p = v; }

// sc: [0] r^T r, [1] 1 once converged (later iterations return at once)
__global__ __launch_bounds__(1024)
void k_ne_init(int n, double* __restrict__ v, double* __restrict__ r, double* __restrict__ p, double* __restrict__ sc)
{
    for (int j = threadIdx.x; j < n; j += 1024) { v[j] = 0.0; r[j] = -1.0; p[j] = -1.0; }
    if (threadIdx.x == 0) { sc[0] = (double)n; sc[1] = 0.0; }
}

__global__ __launch_bounds__(1024)
void k_ne_update(int n, double tol2, double* __restrict__ v, double* __restrict__ r, double* __restrict__ p,
                 const double* __restrict__ q, double* __restrict__ sc)
{
    __shared__ double sh[16];
    if (sc[1] != 0.0) return;
    const double rr = sc[0];
    double pq = 0.0;
    for (int j = threadIdx.x; j < n; j += 1024) pq = fma(p[j], q[j], pq);
    pq = block_sum<1024>(pq, sh);
    if (!(pq > 0.0)) {                       // breakdown (rank-deficient A): stop at the current v
        if (threadIdx.x == 0) sc[1] = 1.0;
        return;
    }
    const double alpha = rr / pq;
    double rn = 0.0;
    for (int j = threadIdx.x; j < n; j += 1024) {
        v[j] = fma(alpha, p[j], v[j]);
        const double rj = fma(-alpha, q[j], r[j]);
        r[j] = rj;
        rn = fma(rj, rj, rn);
    }
    rn = block_sum<1024>(rn, sh);
    const double beta = rn / rr;
    for (int j = threadIdx.x; j < n; j += 1024) p[j] = fma(beta, p[j], r[j]);
    if (threadIdx.x == 0) {
        sc[0] = rn;
        if (rn <= tol2) sc[1] = 1.0;
    }
}

// skips the products once converged, so a run of enqueued iterations past
// convergence costs only their launches
template <typename TA>
__global__ __launch_bounds__(256)
void k_ne_colsum_live(const Inst* __restrict__ insts, const double* __restrict__ p, double* __restrict__ partial,
                      const double* __restrict__ sc)
{
    if (sc[1] != 0.0) return;
    const Inst& I = insts[0];
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int c = blockIdx.y;
    const int m = I.m, n = I.n;
    if (i >= m) return;
    const TA* __restrict__ A = reinterpret_cast<const TA*>(I.A);
    const int j0 = c * kTdChunk, j1 = min(j0 + kTdChunk, n);
    double s = 0.0;
    for (int j = j0; j < j1; ++j) s = fma((double)A[(long long)j * I.lda + i], p[j], s);
    partial[(long long)c * m + i] = s;
}

__global__ __launch_bounds__(256)
void k_ne_rowsum_live(const Inst* __restrict__ insts, const double* __restrict__ partial, int chunks,
                      double* __restrict__ s, const double* __restrict__ sc)
{
    if (sc[1] != 0.0) return;
    const int m = insts[0].m;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    double v = 0.0;
    for (int c = 0; c < chunks; ++c) v += partial[(long long)c * m + i];
    s[i] = v;
}

template <typename TA>
__global__ __launch_bounds__(256)
void k_ne_dot_t_live(const Inst* __restrict__ insts, const double* __restrict__ w, double* __restrict__ q,
                     const double* __restrict__ sc)
{
    if (sc[1] != 0.0) return;
    const Inst& I = insts[0];
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (j >= I.n) return;
    const TA* __restrict__ col = reinterpret_cast<const TA*>(I.A) + (long long)j * I.lda;
    double d = 0.0;
    for (int i = lane; i < I.m; i += 64) d = fma((double)col[i], w[i], d);
    d = wave_sum(d);
    if (lane == 0) q[j] = d;
}

template <typename TA>
static hipError_t normal_equations_t(const LaunchCtx& c, long m, long n, double* scratch, double* t)
{
    const int chunks = (int)((n + kTdChunk - 1) / kTdChunk);
    double* partial = scratch;
    double* w = partial + (size_t)m * chunks;
    double* q = w + m;
    double* v = q + n;
    double* r = v + n;
    double* p = r + n;
    double* sc = p + n;
    const dim3 g1((unsigned)((m + 255) / 256), (unsigned)chunks);
    const unsigned gm = (unsigned)((m + 255) / 256), gt = (unsigned)((n + 3) / 4);
    const double tol2 = 1e-22 * (double)n;
    k_ne_init<<<1, 1024, 0, c.stream>>>((int)n, v, r, p, sc);
    constexpr int kChunk = 16, kMaxIter = 2000;
    double hs[2] = {0.0, 0.0};
    for (int it = 0; it < kMaxIter; it += kChunk) {
        for (int k = 0; k < kChunk; ++k) {
            k_ne_colsum_live<TA><<<g1, 256, 0, c.stream>>>(c.insts, p, partial, sc);
            k_ne_rowsum_live<<<gm, 256, 0, c.stream>>>(c.insts, partial, chunks, w, sc);
            k_ne_dot_t_live<TA><<<gt, 256, 0, c.stream>>>(c.insts, w, q, sc);
            k_ne_update<<<1, 1024, 0, c.stream>>>((int)n, tol2, v, r, p, q, sc);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        // setup only: the host checks convergence between chunks of iterations
        e = hipMemcpyAsync(hs, sc, sizeof(hs), hipMemcpyDeviceToHost, c.stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
        if (e != hipSuccess) return e;
        if (hs[1] != 0.0) break;
    }
    // t = A v
    k_ne_colsum<TA><<<g1, 256, 0, c.stream>>>(c.insts, v, partial);
    k_tdir_rowsum<<<gm, 256, 0, c.stream>>>(c.insts, partial, chunks, t);
    return hipGetLastError();
}

__global__ void k_fill(double* __restrict__ p, long long n, double v)
{
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x)
        p[k] = v;
}

hipError_t launch_fill(double* p, long n, double v, hipStream_t s)
{
    k_fill<<<(unsigned)std::min<long>((n + 255) / 256, 1024), 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}

size_t tdir_scratch_doubles(long m, long n)
{
    // partial sums, an m-vector and an n-vector; the normal equations add
    // v, r, p and two scalars
    return (size_t)m * ((n + kTdChunk - 1) / kTdChunk) + (size_t)m + 4 * (size_t)n + 8;
}

// scratch: tdir_scratch_doubles(m, n); t: m doubles (the instance's t must
// point there); picked: one int
hipError_t launch_tdir(const LaunchCtx& c, int choice, long m, long n, double* scratch, double* t, int* picked)
{
    if (choice == BXS_T_NORMAL_EQUATIONS) {
        hipError_t e;
        if (c.dtype == BXS_BF16) e = normal_equations_t<__bf16>(c, m, n, scratch, t);
        else if (c.dtype == BXS_F32) e = normal_equations_t<float>(c, m, n, scratch, t);
        else e = normal_equations_t<double>(c, m, n, scratch, t);
        if (e != hipSuccess) return e;
        k_set_int<<<1, 1, 0, c.stream>>>(picked, -1);
        return hipGetLastError();
    }
    const int chunks = (int)((n + kTdChunk - 1) / kTdChunk);
    double* partial = scratch;
    double* s = partial + (size_t)m * chunks;
    double* score = s + m;
    const dim3 g1((unsigned)((m + 255) / 256), (unsigned)chunks);
    if (c.dtype == BXS_BF16) k_tdir_colsum<__bf16><<<g1, 256, 0, c.stream>>>(c.insts, partial);
    else if (c.dtype == BXS_F32) k_tdir_colsum<float><<<g1, 256, 0, c.stream>>>(c.insts, partial);
    else k_tdir_colsum<double><<<g1, 256, 0, c.stream>>>(c.insts, partial);
    k_tdir_rowsum<<<(unsigned)((m + 255) / 256), 256, 0, c.stream>>>(c.insts, partial, chunks, s);
    if (choice != BXS_T_NEG_MEAN_COLUMN) {
        if (c.dtype == BXS_BF16) k_tdir_score<__bf16><<<(unsigned)((n + 3) / 4), 256, 0, c.stream>>>(c.insts, s, score);
        else if (c.dtype == BXS_F32) k_tdir_score<float><<<(unsigned)((n + 3) / 4), 256, 0, c.stream>>>(c.insts, s, score);
        else k_tdir_score<double><<<(unsigned)((n + 3) / 4), 256, 0, c.stream>>>(c.insts, s, score);
    }
    if (c.dtype == BXS_BF16) k_tdir_pick<__bf16><<<1, 1024, 0, c.stream>>>(c.insts, s, score, choice, t, picked);
    else if (c.dtype == BXS_F32) k_tdir_pick<float><<<1, 1024, 0, c.stream>>>(c.insts, s, score, choice, t, picked);
    else k_tdir_pick<double><<<1, 1024, 0, c.stream>>>(c.insts, s, score, choice, t, picked);
    return hipGetLastError();
}

}  // namespace bxs
