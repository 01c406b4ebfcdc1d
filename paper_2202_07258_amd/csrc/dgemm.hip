// FP64 matrix products of the batched solver and of the adjoint, written for
// gfx950's FP64 matrix cores (v_mfma_f64_16x16x4_f64):
//
//     C[M x N] = alpha * op(A)[M x K] * op(B)[K x N] + beta * C
//
// every matrix column-major, op(A)(i, k) = A[i + k lda] (TA = 0) or
// A[k + i lda] (TA = 1), op(B)(k, j) = B[k + j ldb] (TB = 0) or B[j + k ldb]
// (TB = 1).  Used as:
//   R = Y - A X      (TA 0, TB 0)   residuals of every right-hand side
//   G = A^T R        (TA 1, TB 0)   correlations
//   dA = R V^T ...   (TA 0, TB 1)   the adjoint's matrix gradient
// An optional list of column indices maps logical column j of op(B) and C to
// physical column cols[j] (TB = 0), so the products run on the right-hand
// sides still active; an optional device count ends the tiles past it.
//
// Workgroup tile 128 x 128, K step 16, 4 waves of 64 x 64 output (4 x 4
// blocks of 16 x 16).  The operands of a K step go through LDS (K-major, so a
// fragment read is 16 consecutive doubles per quarter-wave); the next K step
// is loaded into registers while the current one is multiplied.  The MFMA is
// issued with the B fragment as its first operand, so its 16 x 16 result
// block is C transposed in the lane layout: for a fixed accumulator register
// the 16 lanes of a quarter-wave hold 16 consecutive rows of one column of C
// (coalesced 128-byte stores).  Summation order: each output element is the
// sum over K steps, in order, of 4-term MFMA partial sums; the result is
// deterministic for a given shape.
//
// Consecutive workgroup ids go round-robin over the 8 XCDs; tiles are
// renumbered so that each XCD takes a contiguous range, row tiles fastest,
// and the panel of op(B) that a run of tiles shares stays in one XCD's L2.
#include "dev_common.h"

#include <algorithm>

namespace bxs {

typedef double d4 __attribute__((ext_vector_type(4)));

struct DgemmArgs {
    const double* A;
    long long lda;
    const double* B;
    long long ldb;
    double* C;
    long long ldc;
    const double* Cin;      // beta term read from here (leading dimension ldcin), or from C when nullptr
    long long ldcin;
    int M, N, K;
    double alpha, beta;
    const int* cols;        // logical -> physical column of op(B) and C, or nullptr (TB = 0 only)
    const int* ncols;       // device count of logical columns in use (<= N), or nullptr
    double* splitk;         // scratch of kDgemmSplitScratch doubles for split-K launches, or nullptr
    int kparts;             // set by the launcher: K split into this many slices (1: no split)
    int kslice;             // K per slice (multiple of the K step)
};

constexpr int kGM = 128, kGN = 128, kGK = 16, kGPad = 2;
// split-K scratch: at most 256 (tile, slice) pairs of 128 x 128 doubles
constexpr size_t kDgemmSplitScratch = (size_t)256 * kGM * kGN;
size_t dgemm_splitk_doubles() { return kDgemmSplitScratch; }

template <int TA, int TB>
__global__ __launch_bounds__(256, 2)
void k_dgemm(DgemmArgs p)
{
    __shared__ double sA[kGK][kGM + kGPad];
    __shared__ double sB[kGK][kGN + kGPad];
    __shared__ int sCol[kGN];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int tilesM = (p.M + kGM - 1) / kGM;
    const int tilesN = (p.N + kGN - 1) / kGN;
    const int total = tilesM * tilesN;
    // split-K: blockIdx.y is the K slice; its partial tile goes to the scratch
    const int ks = blockIdx.y;
    const int kbeg = ks * p.kslice;
    const int kend = min(p.K, kbeg + p.kslice);
    // XCD-aware renumbering: workgroup b runs on XCD b % 8
    const int b = blockIdx.x;
    const int per = (total + 7) / 8;
    const int xcd = b & 7, slot = b >> 3;
    int logical = xcd * per + slot;
    if (per * 8 != total) logical = b;            // ragged tile count: identity order
    if (logical >= total) return;
    const int tm = logical % tilesM, tn = logical / tilesM;
    const int i0 = tm * kGM, j0 = tn * kGN;
    const int nlim = p.ncols ? min(p.N, *p.ncols) : p.N;
    if (j0 >= nlim) return;

    if (tid < kGN) {
        const int j = j0 + tid;
        sCol[tid] = (j < nlim) ? (p.cols ? p.cols[j] : j) : -1;
    }
    __syncthreads();

    // register stage of one K step: 8 doubles of op(A) and 8 of op(B) per thread
    double ra[8], rb[8];
    auto load_k = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = tid + 256 * q;              // 1024 two-element chunks per operand
            if (TA == 0) {                            // i contiguous: chunk = (k, i pair)
                const int k = c >> 6, i = (c & 63) * 2;
                const int gk = k0 + k, gi = i0 + i;
                const double* src = p.A + (long long)gk * p.lda + gi;
                const bool kin = gk < kend;
                ra[2 * q] = (kin && gi < p.M) ? src[0] : 0.0;
                ra[2 * q + 1] = (kin && gi + 1 < p.M) ? src[1] : 0.0;
            } else {                                  // k contiguous: chunk = (i, k pair)
                const int i = c >> 3, k = (c & 7) * 2;
                const int gk = k0 + k, gi = i0 + i;
                const double* src = p.A + (long long)gi * p.lda + gk;
                const bool iin = gi < p.M;
                ra[2 * q] = (iin && gk < kend) ? src[0] : 0.0;
                ra[2 * q + 1] = (iin && gk + 1 < kend) ? src[1] : 0.0;
            }
            if (TB == 0) {                            // k contiguous: chunk = (j, k pair)
                const int j = c >> 3, k = (c & 7) * 2;
                const int gk = k0 + k, pj = sCol[j];
                const double* src = p.B + (long long)(pj < 0 ? 0 : pj) * p.ldb + gk;
                rb[2 * q] = (pj >= 0 && gk < kend) ? src[0] : 0.0;
                rb[2 * q + 1] = (pj >= 0 && gk + 1 < kend) ? src[1] : 0.0;
            } else {                                  // j contiguous: chunk = (k, j pair)
                const int k = c >> 6, j = (c & 63) * 2;
                const int gk = k0 + k, gj = j0 + j;
                const double* src = p.B + (long long)gk * p.ldb + gj;
                const bool kin = gk < kend;
                rb[2 * q] = (kin && gj < nlim) ? src[0] : 0.0;
                rb[2 * q + 1] = (kin && gj + 1 < nlim) ? src[1] : 0.0;
            }
        }
    };
    auto store_k = [&]() {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = tid + 256 * q;
            if (TA == 0) {
                const int k = c >> 6, i = (c & 63) * 2;
                sA[k][i] = ra[2 * q];
                sA[k][i + 1] = ra[2 * q + 1];
            } else {
                const int i = c >> 3, k = (c & 7) * 2;
                sA[k][i] = ra[2 * q];
                sA[k + 1][i] = ra[2 * q + 1];
            }
            if (TB == 0) {
                const int j = c >> 3, k = (c & 7) * 2;
                sB[k][j] = rb[2 * q];
                sB[k + 1][j] = rb[2 * q + 1];
            } else {
                const int k = c >> 6, j = (c & 63) * 2;
                sB[k][j] = rb[2 * q];
                sB[k][j + 1] = rb[2 * q + 1];
            }
        }
    };

    d4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = d4{0.0, 0.0, 0.0, 0.0};

    const int kq = lane >> 4, kr = lane & 15;        // fragment lane -> (k within 4, row/col within 16)
    const int nk = (kend - kbeg + kGK - 1) / kGK;
    load_k(kbeg);
    store_k();
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        if (kt + 1 < nk) load_k(kbeg + (kt + 1) * kGK);
#pragma unroll
        for (int ks = 0; ks < kGK / 4; ++ks) {
            double fa[4], fb[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) fa[a] = sA[ks * 4 + kq][wm * 64 + a * 16 + kr];
#pragma unroll
            for (int c = 0; c < 4; ++c) fb[c] = sB[ks * 4 + kq][wn * 64 + c * 16 + kr];
            // block (a, c): D[jj][ii] = sum_k op(B)(k, jj) op(A)(ii, k) = C(ii, jj)
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    acc[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(fb[c], fa[a], acc[a][c], 0, 0, 0);
        }
        __syncthreads();
        if (kt + 1 < nk) {
            store_k();
            __syncthreads();
        }
    }

    // accumulator register r of lane l holds row 4 r + l / 16 of the MFMA result, i.e.
    // C(ii = l % 16, jj = 4 r + l / 16) of its block (layout checked on gfx950)
    if (p.kparts > 1) {
        // split-K: the slice's partial tile, logical columns, dense M x N per slice
        double* part = p.splitk + (size_t)ks * p.M * p.N;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int gi = i0 + wm * 64 + a * 16 + kr;
            if (gi >= p.M) continue;
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int jl = wn * 64 + c * 16 + 4 * r + kq;
                    if (sCol[jl] < 0) continue;
                    part[(size_t)(j0 + jl) * p.M + gi] = acc[a][c][r];
                }
        }
        return;
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int gi = i0 + wm * 64 + a * 16 + kr;
        if (gi >= p.M) continue;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int jl = wn * 64 + c * 16 + 4 * r + kq;
                const int pj = sCol[jl];
                if (pj < 0) continue;
                double* dst = p.C + (long long)pj * p.ldc + gi;
                const double v = p.alpha * acc[a][c][r];
                if (p.beta != 0.0) {
                    const double cin = p.Cin ? p.Cin[(long long)pj * p.ldcin + gi] : *dst;
                    *dst = fma(p.beta, cin, v);
                } else {
                    *dst = v;
                }
            }
        }
    }
}

// Split-K reduction: C = alpha * (sum of the slices in order) + beta * Cin
__global__ __launch_bounds__(256)
void k_dgemm_splitk_sum(DgemmArgs p)
{
    const int nlim = p.ncols ? min(p.N, *p.ncols) : p.N;
    const long long tot = (long long)p.M * nlim;
    const size_t slice = (size_t)p.M * p.N;
    for (long long k = blockIdx.x * 256LL + threadIdx.x; k < tot; k += (long long)gridDim.x * 256) {
        const int i = (int)(k % p.M);
        const int j = (int)(k / p.M);
        double v = 0.0;
        for (int s = 0; s < p.kparts; ++s) v += p.splitk[s * slice + (size_t)j * p.M + i];
        const int pj = p.cols ? p.cols[j] : j;
        double* dst = p.C + (long long)pj * p.ldc + i;
        const double w = p.alpha * v;
        if (p.beta != 0.0) {
            const double cin = p.Cin ? p.Cin[(long long)pj * p.ldcin + i] : *dst;
            *dst = fma(p.beta, cin, w);
        } else {
            *dst = w;
        }
    }
}

hipError_t launch_dgemm(int ta, int tb, const DgemmArgs& a0, hipStream_t s)
{
    if (a0.M <= 0 || a0.N <= 0) return hipSuccess;
    if (a0.cols && tb != 0) return hipErrorInvalidValue;
    DgemmArgs a = a0;
    const int tiles = ((a.M + kGM - 1) / kGM) * ((a.N + kGN - 1) / kGN);
    // Fewer tiles than the chip's 256 CUs: split K so that about 256
    // workgroups run, each slice at least 4 K steps, the slices summed in a
    // fixed order afterwards (deterministic).  tiles * parts <= 256 keeps the
    // slices within the scratch.
    a.kparts = 1;
    a.kslice = a.K;
    if (a.splitk && tiles < 128) {
        const int maxp = std::max(1, 256 / tiles);
        const int steps = (a.K + kGK - 1) / kGK;
        const int parts = std::min(maxp, std::max(1, steps / 4));
        if (parts > 1) {
            const int per = (steps + parts - 1) / parts;
            a.kslice = per * kGK;
            a.kparts = (steps + per - 1) / per;
        }
    }
    const dim3 grid(tiles, a.kparts), block(256);
    if (ta == 0 && tb == 0) k_dgemm<0, 0><<<grid, block, 0, s>>>(a);
    else if (ta == 1 && tb == 0) k_dgemm<1, 0><<<grid, block, 0, s>>>(a);
    else if (ta == 0 && tb == 1) k_dgemm<0, 1><<<grid, block, 0, s>>>(a);
    else if (ta == 1 && tb == 1) k_dgemm<1, 1><<<grid, block, 0, s>>>(a);
    else return hipErrorInvalidValue;
    if (a.kparts > 1) k_dgemm_splitk_sum<<<1024, 256, 0, s>>>(a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP64 matrix-vector products for the power iteration of the batched
// solver's step size (HBM-bound: one read of A each).
//   k_dgemv_n: partial[c][i] = sum over the c-th chunk of 128 columns of
//              A[i, j] v_j  (threads over rows: coalesced column reads)
//   k_dgemv_sum: w_i = sum_c partial[c][i] in chunk order
//   k_dgemv_t: out_j = a_j^T w (one wave per column, fixed-order butterfly)
// ---------------------------------------------------------------------------
constexpr int kGvChunk = 128;

__global__ __launch_bounds__(256)
void k_dgemv_n(const double* __restrict__ A, long long lda, int m, int n, const double* __restrict__ v,
               double* __restrict__ partial)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= m) return;
    const int j0 = c * kGvChunk, j1 = min(j0 + kGvChunk, n);
    double s = 0.0;
    for (int j = j0; j < j1; ++j) s = fma(A[(long long)j * lda + i], v[j], s);
    partial[(long long)c * m + i] = s;
}

__global__ __launch_bounds__(256)
void k_dgemv_sum(const double* __restrict__ partial, int m, int chunks, double* __restrict__ w)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    double s = 0.0;
    for (int c = 0; c < chunks; ++c) s += partial[(long long)c * m + i];
    w[i] = s;
}

__global__ __launch_bounds__(256)
void k_dgemv_t(const double* __restrict__ A, long long lda, int m, int n, const double* __restrict__ w,
               double* __restrict__ out)
{
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (j >= n) return;
    const double* col = A + (long long)j * lda;
    double s = 0.0;
    for (int i = lane; i < m; i += 64) s = fma(col[i], w[i], s);
    s = wave_sum(s);
    if (lane == 0) out[j] = s;
}

size_t dgemv_partial_doubles(long m, long n) { return (size_t)m * ((n + kGvChunk - 1) / kGvChunk); }

// out = A^T (A v); `w` (m) and `partial` (dgemv_partial_doubles) are scratch
hipError_t launch_dgemv_normal(const double* A, long long lda, int m, int n, const double* v, double* w,
                               double* partial, double* out, hipStream_t s)
{
    const int chunks = (n + kGvChunk - 1) / kGvChunk;
    k_dgemv_n<<<dim3((m + 255) / 256, chunks), 256, 0, s>>>(A, lda, m, n, v, partial);
    k_dgemv_sum<<<(m + 255) / 256, 256, 0, s>>>(partial, m, chunks, w);
    k_dgemv_t<<<(n + 3) / 4, 256, 0, s>>>(A, lda, m, n, w, out);
    return hipGetLastError();
}

}  // namespace bxs
