// Batched non-negative least squares with one shared matrix:
//     for every right-hand side b:  min 1/2 ||A x_b - y_b||^2  s.t. x_b >= 0,
// solved by projected gradient with dynamic Gap-safe screening (Alg. 2) for
// all right-hand sides at once, so that every matrix product is a GEMM.
//
// Two iteration engines share one FP64 certification pass:
//  * FP64: R = Y - A X and G = A^T R as FP64 GEMMs (rocBLAS), the projected
//    step as an elementwise kernel.  Same arithmetic as the FP64 oracle.
//  * BF16x3: hand-written MFMA GEMMs on gfx950 (v_mfma_f32_16x16x16bf16_1k)
//    with every FP32 operand split into bf16 hi + lo parts and the three
//    leading partial products accumulated in FP32 (~2^-16 relative error
//    instead of 2^-8 for plain bf16).  The GEMMs act on increments: each pass
//    starts from the exact FP64 gradient G = A^T (Y - A X) of the previous
//    certification, and every iteration takes the projected step
//    X <- Pi(X + eta G), D = change of X, then G <- G - A^T (A D).  The
//    rounding error of a step is proportional to |D|, so it vanishes as the
//    iteration converges instead of putting a floor under the gap.
//    Converged right-hand sides leave the active list, so later GEMMs shrink.
// Certification every K iterations, per right-hand side, in FP64: the
// residual and correlations from FP64 GEMMs on the stored matrix, dual
// translation along t (Sec. 4.2), the per-coordinate gap with rigorous
// rounding margins, the safe radius and the lower-saturation test of Alg. 2.
// Screened coordinates are fixed at 0 (no fold is needed, Alg. 2).
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "bxs_internal.h"

namespace bxs {

bxs_status set_error(bxs_status s, const char* msg);   // api.hip

typedef __attribute__((ext_vector_type(4))) float f4;
typedef __attribute__((ext_vector_type(4))) short s4;

struct BState {
    int done, status, t_valid, passes;
    int n_active, n_lower, pad0, pad1;
    long long iters, col_iters;
    double gap, radius, eps, primal;
};

// ---------------------------------------------------------------------------
// bf16 helpers (round to nearest even)
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned short bf16_bits(float v) {
    unsigned u = __float_as_uint(v);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_float(unsigned short h) { return __uint_as_float(((unsigned)h) << 16); }

// split v = hi + lo + O(2^-16 |v|) with hi, lo in bf16
__device__ __forceinline__ void split_bf16(float v, short& hi, short& lo) {
    const unsigned short h = bf16_bits(v);
    hi = (short)h;
    lo = (short)bf16_bits(v - bf16_float(h));
}

// ---------------------------------------------------------------------------
// BF16x3 MFMA GEMM on the active right-hand sides.  Output tile 64 x 64 per
// workgroup (4 waves, 32 x 32 each = 2 x 2 MFMA 16x16 blocks), K step 32.
//  EPI 0:  U[:, act[c]]  = (A D[:, act])[:, c]        (M = m, K = n)
//  EPI 1:  G[:, act[c]] -= (A^T U[:, act])[:, c]      (M = n, K = m)
// A is column-major m x n; act lists the active right-hand sides.
// ---------------------------------------------------------------------------
template <int EPI>
__global__ __launch_bounds__(256)
void k_gemm_bf16x3(const float* __restrict__ A, long long lda, int m, int n,
                   const int* __restrict__ act, const int* __restrict__ nact_ptr,
                   const float* __restrict__ Bsrc, long long ldb,
                   float* __restrict__ Out, long long ldo)
{
    const int M = (EPI == 0) ? m : n;
    const int K = (EPI == 0) ? n : m;
    const int nact = *nact_ptr;
    const int row0 = blockIdx.x * 64, col0 = blockIdx.y * 64;
    if (col0 >= nact || row0 >= M) return;
    __shared__ float As[64][33];   // [row][k]
    __shared__ float Bs[32][65];   // [k][col]
    __shared__ int s_act[64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    if (tid < 64) s_act[tid] = (col0 + tid < nact) ? act[col0 + tid] : -1;
    __syncthreads();
    f4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = (f4){0.f, 0.f, 0.f, 0.f};

    for (int k0 = 0; k0 < K; k0 += 32) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int idx = tid + e * 256;
            int r, kk;
            if (EPI == 0) { r = idx & 63; kk = idx >> 6; }     // A[row + k*lda]: contiguous rows
            else { r = idx >> 5; kk = idx & 31; }              // A^T: A[k + row*lda]: contiguous k
            const int gr = row0 + r, gk = k0 + kk;
            float v = 0.f;
            if (gr < M && gk < K) v = (EPI == 0) ? A[gr + (long long)gk * lda] : A[gk + (long long)gr * lda];
            As[r][kk] = v;
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int idx = tid + e * 256;
            const int kk = idx & 31, c = idx >> 5;
            const int gk = k0 + kk, b = s_act[c];
            Bs[kk][c] = (b >= 0 && gk < K) ? Bsrc[gk + (long long)b * ldb] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            const int kb = ks * 16 + 4 * (lane >> 4);
            s4 ahi[2], alo[2], bhi[2], blo[2];
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) {
                const int row = wr * 32 + rb * 16 + (lane & 15);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    short h, l;
                    split_bf16(As[row][kb + v], h, l);
                    ahi[rb][v] = h;
                    alo[rb][v] = l;
                }
            }
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                const int col = wc * 32 + cb * 16 + (lane & 15);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    short h, l;
                    split_bf16(Bs[kb + v][col], h, l);
                    bhi[cb][v] = h;
                    blo[cb][v] = l;
                }
            }
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int cb = 0; cb < 2; ++cb) {
                    acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(alo[rb], bhi[cb], acc[rb][cb], 0, 0, 0);
                    acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi[rb], blo[cb], acc[rb][cb], 0, 0, 0);
                    acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi[rb], bhi[cb], acc[rb][cb], 0, 0, 0);
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = row0 + wr * 32 + rb * 16 + 4 * (lane >> 4) + v;
                const int c = wc * 32 + cb * 16 + (lane & 15);
                const int b = s_act[c];
                if (row >= M || b < 0) continue;
                const float val = acc[rb][cb][v];
                if (EPI == 0) Out[row + (long long)b * ldo] = val;
                else Out[row + (long long)b * ldo] -= val;
            }
}

// ---------------------------------------------------------------------------
// elementwise kernels
// ---------------------------------------------------------------------------
// setup: A64 = (double)A, A32 = (float)A (when stored FP64), X0 clipped at 0,
// FP32 copies of X and Y, sat = 0
template <typename TA>
__global__ void k_b_convert_a(const TA* __restrict__ A, long long lda, int m, int n,
                              double* __restrict__ A64, float* __restrict__ A32)
{
    const long long tot = (long long)m * n;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < tot; k += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(k % m);
        const long long j = k / m;
        const double v = (double)A[i + j * lda];
        A64[k] = v;
        if (A32) A32[k] = (float)v;
    }
}

__global__ void k_b_init(const double* __restrict__ Y, long long ldy, double* __restrict__ X, long long ldx,
                         int m, int n, int B, double* __restrict__ X64, float* __restrict__ X32,
                         double* __restrict__ Y64, float* __restrict__ Y32, signed char* __restrict__ sat,
                         long long ldsat, int* __restrict__ err)
{
    const long long nx = (long long)n * B, ny = (long long)m * B;
    int e = 0;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < nx; k += (long long)gridDim.x * blockDim.x) {
        const int j = (int)(k % n);
        const long long b = k / n;
        double v = X[j + b * ldx];
        if (!isfinite(v)) e = 1;
        v = fmax(v, 0.0);
        X64[k] = v;
        if (X32) X32[k] = (float)v;
        sat[j + b * ldsat] = 0;
    }
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < ny; k += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(k % m);
        const long long b = k / m;
        const double v = Y[i + b * ldy];
        if (!isfinite(v)) e = 1;
        Y64[k] = v;
        if (Y32) Y32[k] = (float)v;
    }
    if (e) atomicOr(err, 1);
}

// column statistics of the FP64 copy: rigorous norm bound, w = A^T t
__global__ __launch_bounds__(256)
void k_b_colstats(const double* __restrict__ A64, int m, int n, const double* __restrict__ t,
                  double* __restrict__ cn, double* __restrict__ w, double* __restrict__ tn, int* __restrict__ err)
{
    const int lane = threadIdx.x & 63;
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    const double gm = gamma_k((double)(m / 64) + 8.0);
    if (j < n) {
        const double* col = A64 + (long long)j * m;
        double s2 = 0.0, sw = 0.0;
        int e = 0;
        for (int i = lane; i < m; i += 64) {
            const double a = col[i];
            if (!isfinite(a)) e = 1;
            s2 = fma(a, a, s2);
            sw = fma(a, t ? t[i] : -1.0, sw);
        }
        for (int off = 32; off >= 1; off >>= 1) {
            s2 += __shfl_xor(s2, off, 64);
            sw += __shfl_xor(sw, off, 64);
        }
        if (e) atomicOr(err, 1);
        if (lane == 0) {
            cn[j] = sqrt(s2 * (1.0 + gm)) * (1.0 + 2.0 * kUnit);
            w[j] = sw;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x < 64) {
        double st = 0.0;
        for (int i = lane; i < m; i += 64) { const double v = t ? t[i] : -1.0; st = fma(v, v, st); }
        for (int off = 32; off >= 1; off >>= 1) st += __shfl_xor(st, off, 64);
        if (lane == 0) *tn = sqrt(st * (1.0 + gm)) * (1.0 + 2.0 * kUnit);
    }
}

// FP64 projected step on every not-stopped right-hand side
__global__ void k_b_update64(double* __restrict__ X64, const double* __restrict__ G64, int n, int B,
                             const signed char* __restrict__ sat, long long ldsat, const BState* __restrict__ st,
                             double eta)
{
    const long long nx = (long long)n * B;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < nx; k += (long long)gridDim.x * blockDim.x) {
        const int j = (int)(k % n);
        const long long b = k / n;
        if (st[b].done) continue;
        X64[k] = (sat[j + b * ldsat] != 0) ? 0.0 : fmax(X64[k] + eta * G64[k], 0.0);
    }
}

// projected step of the BF16x3 engine on the active right-hand sides.  The
// iterate stays in FP64 (an FP32 iterate stalls once eta g drops below half
// an ulp of x); the increment D = x_new - x feeds the GEMMs in FP32.
__global__ void k_b_step_mixed(double* __restrict__ X64, float* __restrict__ D32, const float* __restrict__ G32,
                               int n, const int* __restrict__ act, const int* __restrict__ nact_ptr,
                               const signed char* __restrict__ sat, long long ldsat, double eta)
{
    const long long tot = (long long)n * (*nact_ptr);
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < tot; k += (long long)gridDim.x * blockDim.x) {
        const int j = (int)(k % n);
        const long long b = act[k / n];
        const long long e = j + b * n;
        const double xo = X64[e];
        const double xn = (sat[j + b * ldsat] != 0) ? 0.0 : fmax(0.0, xo + eta * (double)G32[e]);
        X64[e] = xn;
        D32[e] = (float)(xn - xo);
    }
}

__global__ void k_b_g64_to_32(const double* __restrict__ G64, float* __restrict__ G32, int n,
                              const int* __restrict__ act, const int* __restrict__ nact_ptr)
{
    const long long tot = (long long)n * (*nact_ptr);
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < tot; k += (long long)gridDim.x * blockDim.x) {
        const long long e = (k % n) + (long long)act[k / n] * n;
        G32[e] = (float)G64[e];
    }
}

__global__ void k_b_x32_to_64(const float* __restrict__ X32, double* __restrict__ X64, int n, int B,
                              const BState* __restrict__ st)
{
    const long long nx = (long long)n * B;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < nx; k += (long long)gridDim.x * blockDim.x) {
        if (st[k / n].done) continue;
        X64[k] = (double)X32[k];
    }
}

__global__ void k_b_copy(const double* __restrict__ src, double* __restrict__ dst, long long count)
{
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < count; k += (long long)gridDim.x * blockDim.x)
        dst[k] = src[k];
}

__global__ void k_b_output(const double* __restrict__ X64, double* __restrict__ X, long long ldx, int n, int B)
{
    const long long nx = (long long)n * B;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < nx; k += (long long)gridDim.x * blockDim.x) {
        const int j = (int)(k % n);
        const long long b = k / n;
        X[j + b * ldx] = X64[k];
    }
}

// power iteration on A^T A with FP64 GEMVs is done by the host through
// rocBLAS; this normalises v and records the Rayleigh quotient.
__global__ __launch_bounds__(256)
void k_b_normalize(double* __restrict__ v, const double* __restrict__ av, int n, int m, double* __restrict__ lam)
{
    __shared__ double sh[4];
    double s = 0.0, q = 0.0;
    for (int j = threadIdx.x; j < n; j += 256) s = fma(v[j], v[j], s);
    for (int i = threadIdx.x; i < m; i += 256) q = fma(av[i], av[i], q);
    for (int off = 32; off >= 1; off >>= 1) { s += __shfl_xor(s, off, 64); q += __shfl_xor(q, off, 64); }
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    const double ss = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = q;
    __syncthreads();
    const double qq = sh[0] + sh[1] + sh[2] + sh[3];
    // v holds A^T A u for the previous unit vector u, av = A u: ||A u||^2 = u^T A^T A u
    if (threadIdx.x == 0) *lam = qq;
    const double inv = ss > 0.0 ? 1.0 / sqrt(ss) : 0.0;
    for (int j = threadIdx.x; j < n; j += 256) v[j] *= inv;
}

__global__ void k_b_init_vec(double* __restrict__ v, int n)
{
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
        const unsigned h = (unsigned)j * 2654435761u;
        v[j] = (1.0 + ((h >> 31) ? 0.25 : -0.25)) / sqrt((double)n);
    }
}

// ---------------------------------------------------------------------------
// Certification and screening, one workgroup per right-hand side (NNLS:
// l = 0, every u_j = +inf).  R64, G64 hold y - A x and A^T (y - A x) in FP64
// from GEMMs whose summation order is unknown, so every dot product is
// bounded with gamma_m (any order of an m-term sum).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256)
void k_b_screen(int m, int n, int B, const double* __restrict__ R64, const double* __restrict__ G64,
                double* __restrict__ X64, float* __restrict__ X32, const double* __restrict__ Y64,
                const double* __restrict__ cn, const double* __restrict__ w, const double* __restrict__ tn_ptr,
                signed char* __restrict__ sat, long long ldsat, BState* __restrict__ st, int* __restrict__ done_counter,
                double eps_gap, int screening, int final_pass, long long iters, int kk)
{
    constexpr int NT = 256;
    __shared__ double sh[NT / 64];
    const int b = blockIdx.x;
    BState& S = st[b];
    if (S.done) return;
    const int tid = threadIdx.x;
    const double* r = R64 + (long long)b * m;
    const double* g = G64 + (long long)b * n;
    double* x = X64 + (long long)b * n;
    signed char* sb = sat + (long long)b * ldsat;
    const double* y = Y64 + (long long)b * m;
    const double u1 = kUnit;
    const double tnorm = *tn_ptr;
    auto bsum = [&](double v) {
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        if ((tid & 63) == 0) sh[tid >> 6] = v;
        __syncthreads();
        const double t = (sh[0] + sh[1]) + (sh[2] + sh[3]);
        __syncthreads();
        return t;
    };
    auto bmax = [&](double v) {
        for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
        if ((tid & 63) == 0) sh[tid >> 6] = v;
        __syncthreads();
        const double t = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
        __syncthreads();
        return t;
    };
    double rs = 0.0, ys = 0.0;
    for (int i = tid; i < m; i += NT) { rs = fma(r[i], r[i], rs); ys = fma(y[i], y[i], ys); }
    rs = bsum(rs);
    ys = bsum(ys);
    const double gm = gamma_k((double)m + 8.0);
    const double gw = gamma_k((double)(m / 64) + 8.0);
    const double rnorm = sqrt(rs * (1.0 + gamma_k((double)m / NT + 16.0))) * (1.0 + 2.0 * u1);
    const double ynorm = sqrt(ys * (1.0 + gamma_k((double)m / NT + 16.0))) * (1.0 + 2.0 * u1);

    double tv = 1.0, emax = 0.0, mass = 0.0, nact = 0.0;
    for (int j = tid; j < n; j += NT) {
        if (sb[j] != 0) continue;
        nact += 1.0;
        mass = fma(fabs(x[j]), cn[j], mass);
        const double ewj = gw * cn[j] * tnorm;
        if (!(w[j] + ewj < 0.0)) tv = 0.0;
        else emax = fmax(emax, fmax(g[j] + gm * cn[j] * rnorm, 0.0) / (-w[j] - ewj));
    }
    tv = -bmax(-tv);
    emax = bmax(emax);
    mass = bsum(mass);
    nact = bsum(nact);
    const bool fallback = !(tv > 0.5) && nact > 0.5;
    const double eps = fallback ? 0.0 : emax * (1.0 + 4.0 * u1);
    const double delta_r = gamma_k((double)n + 8.0) * (ynorm + mass * (1.0 + gamma_k((double)n + 64.0)));

    double G, zmax = -__builtin_inf();
    if (fallback) {
        const double tt = rnorm + delta_r;
        G = 0.5 * tt * tt * (1.0 + 4.0 * u1);
    } else {
        double acc = 0.0, zz = -__builtin_inf();
        for (int j = tid; j < n; j += NT) {
            if (sb[j] != 0) continue;
            const double cj = fma(eps, w[j], g[j]);
            const double ej = cn[j] * (gm * rnorm + gw * eps * tnorm) + 4.0 * u1 * (fabs(g[j]) + eps * fabs(w[j]));
            acc += x[j] * fmax(ej - cj, 0.0);
            if (cn[j] > 0.0) zz = fmax(zz, -(cj + ej) / cn[j]);
        }
        const double gsum = bsum(acc);
        zmax = bmax(zz);
        const double tt = delta_r + eps * tnorm;
        G = (gsum * (1.0 + 3.0 * u1) + 0.5 * tt * tt * (1.0 + 4.0 * u1)) * (1.0 + gamma_k((double)n + 64.0));
    }
    const double rad = sqrt(2.0 * G) * (1.0 + 2.0 * u1);
    const bool stop = G < eps_gap;
    int nlo = 0;
    if (!(stop || final_pass || !screening || fallback) && zmax >= rad) {
        double cnt = 0.0;
        for (int j = tid; j < n; j += NT) {
            if (sb[j] != 0) continue;
            const double cj = fma(eps, w[j], g[j]);
            const double ej = cn[j] * (gm * rnorm + gw * eps * tnorm) + 4.0 * u1 * (fabs(g[j]) + eps * fabs(w[j]));
            if (cj + ej < -rad * cn[j] * (1.0 + 2.0 * u1)) {
                sb[j] = -1;
                x[j] = 0.0;
                if (X32) X32[(long long)b * n + j] = 0.f;
                cnt += 1.0;
            }
        }
        nlo = (int)bsum(cnt);
    }
    if (tid == 0) {
        S.col_iters += (long long)nact * kk;
        S.gap = G; S.radius = rad; S.eps = eps; S.primal = 0.5 * rs;
        S.t_valid = fallback ? 0 : 1;
        S.passes += 1;
        S.n_lower += nlo;
        S.n_active = (int)nact - nlo;
        if (stop || final_pass) {
            S.done = 1;
            S.status = stop ? BXS_OK : BXS_MAXITER;
            S.iters = iters;
            atomicAdd(done_counter, 1);
        }
    }
}

// compact the active right-hand-side list (one workgroup, order kept)
__global__ __launch_bounds__(1024)
void k_b_compact_rhs(int B, const BState* __restrict__ st, int* __restrict__ act, int* __restrict__ nact)
{
    __shared__ int wsum[16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int out = 0;
    for (int base = 0; base < B; base += 1024) {
        const int b = base + tid;
        const bool keep = b < B && !st[b].done;
        const unsigned long long mk = __ballot(keep);
        if (lane == 0) wsum[wave] = __popcll(mk);
        __syncthreads();
        int off = 0, tot = 0;
        for (int w2 = 0; w2 < 16; ++w2) { if (w2 < wave) off += wsum[w2]; tot += wsum[w2]; }
        const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        if (keep) act[out + off + __popcll(mk & lt)] = b;
        out += tot;
        __syncthreads();
    }
    if (tid == 0) *nact = out;
}

__global__ void k_b_iota(int* __restrict__ act, int B, int* __restrict__ nact)
{
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < B; b += gridDim.x * blockDim.x) act[b] = b;
    if (blockIdx.x == 0 && threadIdx.x == 0) *nact = B;
}

// ---------------------------------------------------------------------------
// host driver
// ---------------------------------------------------------------------------
static thread_local rocblas_handle g_blas = nullptr;

static bxs_status blas_handle(hipStream_t s, rocblas_handle* out)
{
    if (!g_blas) {
        if (rocblas_create_handle(&g_blas) != rocblas_status_success) return set_error(BXS_ERR_DEVICE, "rocblas_create_handle failed");
    }
    if (rocblas_set_stream(g_blas, s) != rocblas_status_success) return set_error(BXS_ERR_DEVICE, "rocblas_set_stream failed");
    *out = g_blas;
    return BXS_OK;
}

#define BXS_HIPB(call)                                                                           \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) return set_error(BXS_ERR_DEVICE, hipGetErrorString(e_));           \
    } while (0)
#define BXS_BLAS(call)                                                                           \
    do {                                                                                         \
        if ((call) != rocblas_status_success) return set_error(BXS_ERR_DEVICE, #call " failed"); \
    } while (0)

static size_t al(size_t v) { return (v + 255) / 256 * 256; }

size_t batched_workspace_bytes(long m, long n, long B, int iter_precision)
{
    size_t b = 0;
    b += al(sizeof(double) * m * n);          // A64
    if (iter_precision == 1) b += al(sizeof(float) * m * n);   // A32 (when A is FP64)
    b += al(sizeof(double) * n * B);          // X64
    b += al(sizeof(double) * m * B);          // R64
    b += al(sizeof(double) * n * B);          // G64
    b += al(sizeof(double) * m * B);          // Y64
    if (iter_precision == 1) {
        b += al(sizeof(float) * n * B);       // D32 (step)
        b += al(sizeof(float) * m * B);       // U32 = A D
        b += al(sizeof(float) * n * B);       // G32
    }
    b += al(sizeof(double) * (4 * (size_t)n + m + 16));   // cn, w, power vectors, scalars
    b += al(sizeof(BState) * B);
    b += al(sizeof(int) * (B + 16));
    return b + 1024;
}

bxs_status batched_nnls_run(long m, long n, long B, int a_dtype, const void* A, long lda, const double* Y, long ldy,
                            double* X, long ldx, signed char* sat, long ldsat, const bxs_opts* o, bxs_info* infos)
{
    hipStream_t s = (hipStream_t)o->stream;
    const int prec = o->iter_precision;
    const size_t need = batched_workspace_bytes(m, n, B, prec);
    void* ws = o->workspace;
    bool owned = false;
    if (ws) {
        if (o->workspace_bytes < need) return set_error(BXS_ERR_NOMEM, "workspace too small for the batched solve");
    } else {
        if (hipMalloc(&ws, need) != hipSuccess) return set_error(BXS_ERR_NOMEM, "hipMalloc failed for the batched workspace");
        owned = true;
    }
    struct Guard { void* p; bool own; hipStream_t s; ~Guard() { if (own) { (void)hipStreamSynchronize(s); (void)hipFree(p); } } } guard{ws, owned, s};
    char* cur = (char*)(((uintptr_t)ws + 255) / 256 * 256);
    auto take = [&](size_t bytes) { char* p = cur; cur += al(bytes); return p; };
    double* A64 = (double*)take(sizeof(double) * m * n);
    float* A32 = nullptr;
    if (prec == 1) A32 = (a_dtype == BXS_F32) ? (float*)A : (float*)take(sizeof(float) * m * n);
    double* X64 = (double*)take(sizeof(double) * n * B);
    double* R64 = (double*)take(sizeof(double) * m * B);
    double* G64 = (double*)take(sizeof(double) * n * B);
    double* Y64 = (double*)take(sizeof(double) * m * B);
    float *X32 = nullptr, *D32 = nullptr, *U32 = nullptr, *G32 = nullptr, *Y32 = nullptr;
    if (prec == 1) {
        D32 = (float*)take(sizeof(float) * n * B);
        U32 = (float*)take(sizeof(float) * m * B);
        G32 = (float*)take(sizeof(float) * n * B);
    }
    double* sc = (double*)take(sizeof(double) * (4 * (size_t)n + m + 16));
    double* cn = sc;
    double* w = sc + n;
    double* pv = sc + 2 * n;         // n
    double* pav = sc + 3 * n;        // m (A v)
    double* scal = sc + 3 * n + m;   // [0] tnorm, [1] lambda
    BState* st = (BState*)take(sizeof(BState) * B);
    int* ints = (int*)take(sizeof(int) * (B + 16));
    int* act = ints;
    int* nact = ints + B;
    int* done_counter = ints + B + 1;
    int* err = ints + B + 2;
    const long long lda32 = (a_dtype == BXS_F32) ? lda : m;   // A32 layout

    rocblas_handle h;
    bxs_status bs = blas_handle(s, &h);
    if (bs != BXS_OK) return bs;

    hipEvent_t e0, e1, e2;
    BXS_HIPB(hipEventCreate(&e0));
    BXS_HIPB(hipEventCreate(&e1));
    BXS_HIPB(hipEventCreate(&e2));
    struct EG { hipEvent_t a, b, c; ~EG() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); (void)hipEventDestroy(c); } } eg{e0, e1, e2};
    BXS_HIPB(hipEventRecord(e0, s));

    BXS_HIPB(hipMemsetAsync(st, 0, sizeof(BState) * B, s));
    BXS_HIPB(hipMemsetAsync(ints, 0, sizeof(int) * (B + 16), s));
    const int grid = 2048;
    if (a_dtype == BXS_F32)
        k_b_convert_a<float><<<grid, 256, 0, s>>>((const float*)A, lda, (int)m, (int)n, A64, nullptr);
    else
        k_b_convert_a<double><<<grid, 256, 0, s>>>((const double*)A, lda, (int)m, (int)n, A64,
                                                    (prec == 1) ? A32 : nullptr);
    k_b_init<<<grid, 256, 0, s>>>(Y, ldy, X, ldx, (int)m, (int)n, (int)B, X64, X32, Y64, Y32, sat, ldsat, err);
    k_b_colstats<<<(int)((n + 3) / 4), 256, 0, s>>>(A64, (int)m, (int)n, o->t, cn, w, scal, err);
    k_b_iota<<<64, 256, 0, s>>>(act, (int)B, nact);
    BXS_HIPB(hipGetLastError());

    // step: power iteration on A^T A with FP64 GEMVs (unless given)
    double eta = o->step;
    double lam_h = 0.0;
    if (!(eta > 0.0)) {
        const double one = 1.0, zero = 0.0;
        k_b_init_vec<<<16, 256, 0, s>>>(pv, (int)n);
        const int np = o->power_iters > 0 ? o->power_iters : 20;
        for (int k = 0; k < np; ++k) {
            BXS_BLAS(rocblas_dgemv(h, rocblas_operation_none, (int)m, (int)n, &one, A64, (int)m, pv, 1, &zero, pav, 1));
            BXS_BLAS(rocblas_dgemv(h, rocblas_operation_transpose, (int)m, (int)n, &one, A64, (int)m, pav, 1, &zero, pv, 1));
            k_b_normalize<<<1, 256, 0, s>>>(pv, pav, (int)n, (int)m, scal + 1);
        }
        BXS_HIPB(hipMemcpyAsync(&lam_h, scal + 1, sizeof(double), hipMemcpyDeviceToHost, s));
    }
    int herr = 0;
    BXS_HIPB(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, s));
    BXS_HIPB(hipStreamSynchronize(s));
    if (herr) return set_error(BXS_ERR_NONFINITE, "non-finite value in A, Y, X0 or t");
    if (!(eta > 0.0)) eta = lam_h > 0.0 ? 1.0 / (1.05 * lam_h) : 1.0;
    BXS_HIPB(hipEventRecord(e1, s));

    const double one = 1.0, mone = -1.0, zero = 0.0;
    auto residual_and_corr = [&]() -> bxs_status {
        k_b_copy<<<grid, 256, 0, s>>>(Y64, R64, (long long)m * B);
        BXS_BLAS(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, (int)m, (int)B, (int)n, &mone, A64,
                               (int)m, X64, (int)n, &one, R64, (int)m));
        BXS_BLAS(rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, (int)n, (int)B, (int)m, &one,
                               A64, (int)m, R64, (int)m, &zero, G64, (int)n));
        return BXS_OK;
    };

    if (prec == 1) {
        bs = residual_and_corr();
        if (bs != BXS_OK) return bs;
        k_b_g64_to_32<<<grid, 256, 0, s>>>(G64, G32, (int)n, act, nact);
    }
    int* hdone = nullptr;
    BXS_HIPB(hipHostMalloc((void**)&hdone, sizeof(int), hipHostMallocDefault));
    struct HG { int* p; ~HG() { (void)hipHostFree(p); } } hg{hdone};
    const int K = o->screen_every;
    long long iters = 0;
    // optional HIP-event timing of the iteration GEMM pairs
    std::vector<hipEvent_t> pev;
    struct PG2 { std::vector<hipEvent_t>* v; ~PG2() { for (auto e : *v) if (e) (void)hipEventDestroy(e); } } pg2{&pev};
    if (o->profile) {
        pev.assign(2 * (size_t)K, nullptr);
        for (auto& e : pev) BXS_HIPB(hipEventCreate(&e));
    }
    double gemm_ms = 0.0;
    long gemm_pairs = 0;
    while (true) {
        const long long kk = std::min<long long>(K, o->max_iter - iters);
        for (long long k = 0; k < kk; ++k) {
            if (prec == 1) {
                k_b_step_mixed<<<grid, 256, 0, s>>>(X64, D32, G32, (int)n, act, nact, sat, ldsat, eta);
                if (o->profile) BXS_HIPB(hipEventRecord(pev[2 * k], s));
                dim3 g0((unsigned)((m + 63) / 64), (unsigned)((B + 63) / 64));
                k_gemm_bf16x3<0><<<g0, 256, 0, s>>>(A32, lda32, (int)m, (int)n, act, nact, D32, n, U32, m);
                dim3 g1((unsigned)((n + 63) / 64), (unsigned)((B + 63) / 64));
                k_gemm_bf16x3<1><<<g1, 256, 0, s>>>(A32, lda32, (int)m, (int)n, act, nact, U32, m, G32, n);
                if (o->profile) BXS_HIPB(hipEventRecord(pev[2 * k + 1], s));
            } else {
                if (o->profile) BXS_HIPB(hipEventRecord(pev[2 * k], s));
                bs = residual_and_corr();
                if (bs != BXS_OK) return bs;
                if (o->profile) BXS_HIPB(hipEventRecord(pev[2 * k + 1], s));
                k_b_update64<<<grid, 256, 0, s>>>(X64, G64, (int)n, (int)B, sat, ldsat, st, eta);
            }
        }
        iters += kk;
        bs = residual_and_corr();
        if (bs != BXS_OK) return bs;
        const int final_pass = iters >= o->max_iter;
        k_b_screen<<<(int)B, 256, 0, s>>>((int)m, (int)n, (int)B, R64, G64, X64, X32, Y64, cn, w, scal, sat, ldsat, st,
                                          done_counter, o->eps_gap, o->screening, final_pass, iters, (int)kk);
        k_b_compact_rhs<<<1, 1024, 0, s>>>((int)B, st, act, nact);
        // the next pass of the BF16x3 engine restarts from the exact gradient
        if (prec == 1) k_b_g64_to_32<<<grid, 256, 0, s>>>(G64, G32, (int)n, act, nact);
        BXS_HIPB(hipGetLastError());
        BXS_HIPB(hipMemcpyAsync(hdone, done_counter, sizeof(int), hipMemcpyDeviceToHost, s));
        BXS_HIPB(hipStreamSynchronize(s));
        if (o->profile) {
            for (long long k = 0; k < kk; ++k) {
                float ms = 0.f;
                BXS_HIPB(hipEventElapsedTime(&ms, pev[2 * k], pev[2 * k + 1]));
                gemm_ms += ms;
                ++gemm_pairs;
            }
        }
        if (*hdone >= B || final_pass) break;
    }
    k_b_output<<<grid, 256, 0, s>>>(X64, X, ldx, (int)n, (int)B);
    BXS_HIPB(hipEventRecord(e2, s));
    std::vector<BState> hs(B);
    BXS_HIPB(hipMemcpyAsync(hs.data(), st, sizeof(BState) * B, hipMemcpyDeviceToHost, s));
    BXS_HIPB(hipStreamSynchronize(s));
    float ms_setup = 0.f, ms_solve = 0.f;
    BXS_HIPB(hipEventElapsedTime(&ms_setup, e0, e1));
    BXS_HIPB(hipEventElapsedTime(&ms_solve, e1, e2));
    bxs_status worst = BXS_OK;
    for (long b = 0; b < B; ++b) {
        const BState& S = hs[b];
        const int status = S.done ? S.status : BXS_MAXITER;
        if (status != BXS_OK) worst = (bxs_status)status;
        if (infos) {
            bxs_info& f = infos[b];
            memset(&f, 0, sizeof(f));
            f.status = status; f.t_valid = S.t_valid;
            f.iters = S.done ? S.iters : iters; f.passes = S.passes;
            f.n_active = S.n_active; f.n_lower = S.n_lower; f.n_upper = 0;
            f.gap = S.gap; f.primal = S.primal; f.radius = S.radius; f.eps = S.eps;
            f.step = eta; f.lipschitz = lam_h; f.ms_setup = ms_setup; f.ms_solve = ms_solve;
            f.col_iters = S.col_iters;
            f.sweep_ms = gemm_ms;
            f.sweep_launches = gemm_pairs;
        }
    }
    return worst;
}

}  // namespace bxs

// ---------------------------------------------------------------------------
// Adjoint of the batched NNLS solution map (implicit differentiation).
// At an optimum with free set F_b = {j : x_jb > 0} the optimality conditions
// (Sec. 3.2, eq. optimality2: a_j^T (y_b - A x_b) = 0 on F_b) give
// x_F = (A_F^T A_F)^{-1} A_F^T y_b, hence for dL/dX:
//     v_b      = (A_F^T A_F)^{-1} (dL/dx_b)_F      (batched masked CG, FP64)
//     dL/dy_b  = A v_b  (v_b = 0 off F_b)
//     dL/dA    = R V^T - (dL/dY) X^T,   R = Y - A X
// ---------------------------------------------------------------------------
namespace bxs {

__global__ void k_adj_init(const double* __restrict__ X, long long ldx, const double* __restrict__ dX, long long ldg,
                           int n, int B, double* __restrict__ V, double* __restrict__ Rc, double* __restrict__ P,
                           signed char* __restrict__ F)
{
    const long long tot = (long long)n * B;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < tot; k += (long long)gridDim.x * blockDim.x) {
        const int j = (int)(k % n);
        const long long b = k / n;
        const bool free_ = X[j + b * ldx] > 0.0;
        const double d = free_ ? dX[j + b * ldg] : 0.0;
        F[k] = free_ ? 1 : 0;
        V[k] = 0.0;
        Rc[k] = d;
        P[k] = d;
    }
}

// per right-hand side dot products of two n x B blocks (one workgroup each)
__global__ __launch_bounds__(256)
void k_adj_dot(const double* __restrict__ U, const double* __restrict__ W, int n, double* __restrict__ out)
{
    __shared__ double sh[4];
    const long long b = blockIdx.x;
    double s = 0.0;
    for (int j = threadIdx.x; j < n; j += 256) s = fma(U[j + b * n], W[j + b * n], s);
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[b] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// S <- mask(S); alpha = rs / (p.S); V += alpha P; Rc -= alpha S.  A column
// whose flag is set (converged, or p^T S <= 0: the masked normal matrix is
// singular along p) is frozen.
__global__ void k_adj_step(double* __restrict__ S, const signed char* __restrict__ F, const double* __restrict__ rs,
                           const double* __restrict__ pq, const int* __restrict__ done, double* __restrict__ V,
                           double* __restrict__ Rc, const double* __restrict__ P, int n, int B)
{
    const long long tot = (long long)n * B;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < tot; k += (long long)gridDim.x * blockDim.x) {
        const long long b = k / n;
        if (done[b] || !(pq[b] > 0.0)) continue;
        const double alpha = rs[b] / pq[b];
        const double sv = F[k] ? S[k] : 0.0;
        V[k] += alpha * P[k];
        Rc[k] -= alpha * sv;
    }
}

__global__ void k_adj_mask(double* __restrict__ S, const signed char* __restrict__ F, long long tot)
{
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < tot; k += (long long)gridDim.x * blockDim.x)
        if (!F[k]) S[k] = 0.0;
}

// P = Rc + (rs_new / rs_old) P for the columns still running
__global__ void k_adj_dir(double* __restrict__ P, const double* __restrict__ Rc, const double* __restrict__ rs_new,
                          const double* __restrict__ rs_old, const int* __restrict__ done, int n, int B)
{
    const long long tot = (long long)n * B;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < tot; k += (long long)gridDim.x * blockDim.x) {
        const long long b = k / n;
        if (done[b]) continue;
        const double beta = (rs_old[b] > 0.0) ? rs_new[b] / rs_old[b] : 0.0;
        P[k] = Rc[k] + beta * P[k];
    }
}

// Per column bookkeeping after a CG step: rs <- rs_new; a column is done when
// its residual fell below tol^2 * rs0 (done = 1) or when p^T A_F^T A_F p <= 0
// or a non-finite value appeared (done = 2, breakdown).
__global__ void k_adj_track(double* __restrict__ rs, const double* __restrict__ rsn, const double* __restrict__ rs0,
                            const double* __restrict__ pq, int* __restrict__ done, int B, double tol2)
{
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < B; b += gridDim.x * blockDim.x) {
        if (done[b]) continue;
        const double r = rsn[b];
        if (!(pq[b] > 0.0) || !isfinite(r)) { done[b] = 2; continue; }
        rs[b] = r;
        if (r <= tol2 * rs0[b]) done[b] = 1;
    }
}

// counters[0] = columns not converged, counters[1] = breakdowns
__global__ void k_adj_count(const int* __restrict__ done, int B, int* __restrict__ counters)
{
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < B; b += gridDim.x * blockDim.x) {
        const int d = done[b];
        if (d != 1) atomicAdd(&counters[0], 1);
        if (d == 2) atomicAdd(&counters[1], 1);
    }
}

__global__ void k_adj_copy2(const double* __restrict__ src, long long lds, double* __restrict__ dst, long long ldd,
                            int rows, int cols)
{
    const long long tot = (long long)rows * cols;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < tot; k += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(k % rows);
        const long long c = k / rows;
        dst[i + c * ldd] = src[i + c * lds];
    }
}

size_t adjoint_workspace_bytes(long m, long n, long B)
{
    size_t b = 0;
    b += al(sizeof(double) * m * n);       // A64
    b += al(sizeof(double) * n * B) * 5;   // X, V, Rc, P, S
    b += al(sizeof(double) * m * B) * 2;   // Q, R
    b += al(sizeof(signed char) * n * B);  // F
    b += al(sizeof(double) * B) * 4;       // rs, rs0, pq, rs_new
    b += al(sizeof(int) * B);              // done
    b += al(sizeof(int) * 16);
    return b + 1024;
}

bxs_status adjoint_run(long m, long n, long B, int a_dtype, const void* A, long lda, const double* Y, long ldy,
                       const double* X, long ldx, const double* dX, long ldg, double* dY, long lddy, double* dA,
                       long ldda, const bxs_opts* o, long* cg_iters)
{
    hipStream_t s = (hipStream_t)o->stream;
    const size_t need = adjoint_workspace_bytes(m, n, B);
    void* ws = o->workspace;
    bool owned = false;
    if (ws) {
        if (o->workspace_bytes < need) return set_error(BXS_ERR_NOMEM, "workspace too small for the adjoint");
    } else {
        if (hipMalloc(&ws, need) != hipSuccess) return set_error(BXS_ERR_NOMEM, "hipMalloc failed for the adjoint workspace");
        owned = true;
    }
    struct Guard { void* p; bool own; hipStream_t s; ~Guard() { if (own) { (void)hipStreamSynchronize(s); (void)hipFree(p); } } } guard{ws, owned, s};
    char* cur = (char*)(((uintptr_t)ws + 255) / 256 * 256);
    auto take = [&](size_t bytes) { char* p = cur; cur += al(bytes); return p; };
    double* A64 = (double*)take(sizeof(double) * m * n);
    double* Xc = (double*)take(sizeof(double) * n * B);
    double* V = (double*)take(sizeof(double) * n * B);
    double* Rc = (double*)take(sizeof(double) * n * B);
    double* P = (double*)take(sizeof(double) * n * B);
    double* S = (double*)take(sizeof(double) * n * B);
    double* Q = (double*)take(sizeof(double) * m * B);
    double* R = (double*)take(sizeof(double) * m * B);
    signed char* F = (signed char*)take(sizeof(signed char) * n * B);
    double* rs = (double*)take(sizeof(double) * B);
    double* rs0 = (double*)take(sizeof(double) * B);
    double* pq = (double*)take(sizeof(double) * B);
    double* rsn = (double*)take(sizeof(double) * B);
    int* done = (int*)take(sizeof(int) * B);
    int* counters = (int*)take(sizeof(int) * 16);

    rocblas_handle h;
    bxs_status bs = blas_handle(s, &h);
    if (bs != BXS_OK) return bs;
    const int grid = 2048;
    if (a_dtype == BXS_F32)
        k_b_convert_a<float><<<grid, 256, 0, s>>>((const float*)A, lda, (int)m, (int)n, A64, nullptr);
    else
        k_b_convert_a<double><<<grid, 256, 0, s>>>((const double*)A, lda, (int)m, (int)n, A64, nullptr);
    k_adj_copy2<<<grid, 256, 0, s>>>(X, ldx, Xc, n, (int)n, (int)B);
    k_adj_init<<<grid, 256, 0, s>>>(X, ldx, dX, ldg, (int)n, (int)B, V, Rc, P, F);
    k_adj_dot<<<(int)B, 256, 0, s>>>(Rc, Rc, (int)n, rs);
    k_b_copy<<<64, 256, 0, s>>>(rs, rs0, B);
    BXS_HIPB(hipMemsetAsync(done, 0, sizeof(int) * B, s));
    BXS_HIPB(hipGetLastError());
    const double one = 1.0, zero = 0.0, mone = -1.0;
    const double tol = o->eps_gap > 0.0 ? o->eps_gap : 1e-12;
    const long maxit = o->max_iter;
    int* hflag = nullptr;
    BXS_HIPB(hipHostMalloc((void**)&hflag, 2 * sizeof(int), hipHostMallocDefault));
    struct HG { int* p; ~HG() { (void)hipHostFree(p); } } hg{hflag};
    hflag[0] = 1;
    hflag[1] = 0;
    long it = 0;
    for (; it < maxit; ++it) {
        // S = mask(A^T (A P))
        BXS_BLAS(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, (int)m, (int)B, (int)n, &one, A64,
                               (int)m, P, (int)n, &zero, Q, (int)m));
        BXS_BLAS(rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, (int)n, (int)B, (int)m, &one,
                               A64, (int)m, Q, (int)m, &zero, S, (int)n));
        k_adj_mask<<<grid, 256, 0, s>>>(S, F, (long long)n * B);
        k_adj_dot<<<(int)B, 256, 0, s>>>(P, S, (int)n, pq);
        k_adj_step<<<grid, 256, 0, s>>>(S, F, rs, pq, done, V, Rc, P, (int)n, (int)B);
        k_adj_dot<<<(int)B, 256, 0, s>>>(Rc, Rc, (int)n, rsn);
        k_adj_dir<<<grid, 256, 0, s>>>(P, Rc, rsn, rs, done, (int)n, (int)B);
        k_adj_track<<<(int)((B + 255) / 256), 256, 0, s>>>(rs, rsn, rs0, pq, done, (int)B, tol * tol);
        if ((it % 8) == 7 || it + 1 == maxit) {
            BXS_HIPB(hipMemsetAsync(counters, 0, 2 * sizeof(int), s));
            k_adj_count<<<16, 256, 0, s>>>(done, (int)B, counters);
            BXS_HIPB(hipMemcpyAsync(hflag, counters, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
            BXS_HIPB(hipStreamSynchronize(s));
            if (hflag[0] == hflag[1]) { ++it; break; }   // every column converged or broke down
        }
    }
    BXS_HIPB(hipGetLastError());
    // dL/dY = A V
    BXS_BLAS(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, (int)m, (int)B, (int)n, &one, A64, (int)m,
                           V, (int)n, &zero, Q, (int)m));
    k_adj_copy2<<<grid, 256, 0, s>>>(Q, m, dY, lddy, (int)m, (int)B);
    if (dA) {
        // R = Y - A X, then dL/dA = R V^T - (dL/dY) X^T
        k_adj_copy2<<<grid, 256, 0, s>>>(Y, ldy, R, m, (int)m, (int)B);
        BXS_BLAS(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, (int)m, (int)B, (int)n, &mone, A64,
                               (int)m, Xc, (int)n, &one, R, (int)m));
        BXS_BLAS(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_transpose, (int)m, (int)n, (int)B, &one, R,
                               (int)m, V, (int)n, &zero, dA, (int)ldda));
        BXS_BLAS(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_transpose, (int)m, (int)n, (int)B, &mone, Q,
                               (int)m, Xc, (int)n, &one, dA, (int)ldda));
    }
    BXS_HIPB(hipStreamSynchronize(s));
    if (cg_iters) *cg_iters = it;
    if (hflag[1] > 0) return BXS_SINGULAR;
    return (hflag[0] == 0) ? BXS_OK : BXS_MAXITER;
}

}  // namespace bxs
