// Batched non-negative least squares with one shared matrix:
//     for every right-hand side b:  min 1/2 ||A x_b - y_b||^2  s.t. x_b >= 0,
// solved by projected gradient with dynamic Gap-safe screening (Alg. 2) for
// all right-hand sides at once, so that every matrix product is a GEMM.
//
// Two iteration engines share one FP64 certification pass:
//  * FP64: R = Y - A X and G = A^T R as FP64 MFMA GEMMs (dgemm.hip) on the
//    right-hand sides still active, the projected step as an elementwise
//    kernel.  Same arithmetic as the FP64 oracle up to summation order.
//  * BF16x3: hand-written MFMA GEMMs on gfx950 (v_mfma_f32_16x16x32_bf16)
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

#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <chrono>
#include <vector>

#include "bxs_internal.h"

namespace bxs {

bxs_status set_error(bxs_status s, const char* msg);   // api.hip
bxs_status event_overhead(hipStream_t s, double* out); // api.hip

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
// BF16x3 MFMA GEMM on the active right-hand sides (gfx950,
// v_mfma_f32_16x16x32_bf16).  Both products of an iteration have the form
//     C[M x ncols] = Aop[M x K] * Bop[K x ncols]
// with Aop row-major (K contiguous, rows and K zero-padded to multiples of
// 128) and every column of Bop K-contiguous; each operand comes as a bf16 hi
// part and a bf16 lo part, and the three leading partial products
// lo*hi + hi*lo + hi*hi are accumulated in FP32.
//  EPI 0:  U = A D            (Aop = A row-major copy, Bop = D, M = m, K = n);
//          U is written as its bf16 hi/lo split for the next product.
//  EPI 1:  G -= A^T U         (Aop = A column-major copy, Bop = U, M = n,
//          K = m), then the projected step on the same tile:
//          x <- max(0, x + eta g) in FP64 (0 where screened), D = x_new - x
//          written as its bf16 hi/lo split.
// Workgroup tile 128 x 128, K step 32, 4 waves of 64 x 64 (4 x 4 MFMA
// blocks); the next K step is loaded into registers while the current one is
// multiplied out of LDS.  Consecutive workgroup ids go round-robin over the
// 8 XCDs, so the tile order is permuted to give each XCD a contiguous block
// of column tiles (each Bop column panel is then read by one XCD's L2).
// ---------------------------------------------------------------------------
typedef unsigned short u16;
typedef __attribute__((ext_vector_type(8))) __bf16 bf8v;

constexpr int kG3K = 32;   // K step (one 16x16x32 MFMA)

struct G3Args {
    const u16* Ahi; const u16* Alo; long long lda;     // Aop, lda = padded K
    int tiles_m, tiles_n, K;                            // K = padded K (multiple of 32)
    const int* act; int nact;                           // active right-hand sides (host bound)
    const int* nact_dev;                                // their device count (<= nact)
    const u16* Bhi; const u16* Blo; long long ldb;     // Bop column b at b * ldb
    u16* Ohi; u16* Olo; long long ldo;                 // EPI 0 output split (U), EPI 1: D
    float* G; double* X; const signed char* sat; long long ldsat;   // EPI 1 (n x B, ld n)
    int n; double eta;
};

__device__ __forceinline__ unsigned pack2(u16 a, u16 b) { return (unsigned)a | ((unsigned)b << 16); }

template <int EPI, int TM, int WR, int WC>
__global__ __launch_bounds__(64 * WR * WC)
void k_gemm3(G3Args p)
{
    constexpr int NT = 64 * WR * WC;           // threads
    constexpr int WTR = TM / WR, WTC = TM / WC;   // wave tile
    constexpr int NBR = WTR / 16, NBC = WTC / 16; // 16 x 16 blocks per wave
    constexpr int NL = 4 * TM / NT;            // 16-byte loads per thread and operand part (1 or 2)
    static_assert(NL == 1 || NL == 2, "one or two load slots per thread");
    // LDS: two buffers of the four operand tiles of one K step (rows of 32
    // bf16 = four 16-byte chunks; chunk c of row r is stored at position
    // (c + r / 4) mod 4, so 16 lanes reading one chunk of 16 consecutive rows,
    // and 16 lanes writing four chunks of four rows, hit distinct banks),
    // reused by the epilogue for CC columns of the FP32 result at a time.
    constexpr int kTile = TM * kG3K;           // bf16 per operand tile
    constexpr int kOpBytes = 2 * 4 * kTile * (int)sizeof(u16);
    constexpr int kCLd = TM + 4;
    constexpr int CC = (kOpBytes / (kCLd * (int)sizeof(float)) >= TM) ? TM : TM / 2;
    static_assert(CC % WTC == 0 && CC * kCLd * (int)sizeof(float) <= kOpBytes, "epilogue staging fits");
    __shared__ __attribute__((aligned(16))) unsigned char smem[kOpBytes];
    u16* const sbase = (u16*)smem;
    float* const sC = (float*)smem;
    __shared__ int s_act[TM];
    const int tiles = p.tiles_m * p.tiles_n;
    const int id = blockIdx.x;
    const int t = (tiles % 8 == 0) ? (id % 8) * (tiles / 8) + id / 8 : id;
    const int row0 = (t % p.tiles_m) * TM, col0 = (t / p.tiles_m) * TM;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // the grid is sized from a host bound that may lag the device count by a
    // pass (the host enqueues one pass ahead); tiles past the count return
    const int nact = min(p.nact, *p.nact_dev);
    if (col0 >= nact) return;
    if (tid < TM) s_act[tid] = (col0 + tid < nact) ? p.act[col0 + tid] : -1;
    __syncthreads();
    auto soff = [](int r, int c) { return r * kG3K + 8 * ((c + (r >> 2)) & 3); };

    // global -> register slots: NL x 16 B of each of Ahi, Alo, Bhi, Blo per
    // thread.  Columns past the active count read column 0 of Bop: each
    // output column depends on its own Bop column only, and those outputs
    // are never stored.
    const int kc = tid & 3, kq = 8 * kc;
    const int r0 = tid >> 2, r1 = r0 + NT / 4;   // second slot only when NL = 2
    const int srow0 = soff(r0, kc), srow1 = soff(r1, kc);
    const u16* const pa0h = p.Ahi + (long long)(row0 + r0) * p.lda + kq;
    const u16* const pa0l = p.Alo + (long long)(row0 + r0) * p.lda + kq;
    const long long bo0 = (long long)max(s_act[r0], 0) * p.ldb + kq;
    const u16* const pb0h = p.Bhi + bo0;
    const u16* const pb0l = p.Blo + bo0;
    const u16* pa1h = pa0h;
    const u16* pa1l = pa0l;
    const u16* pb1h = pb0h;
    const u16* pb1l = pb0l;
    if constexpr (NL > 1) {
        pa1h = p.Ahi + (long long)(row0 + r1) * p.lda + kq;
        pa1l = p.Alo + (long long)(row0 + r1) * p.lda + kq;
        const long long bo1 = (long long)max(s_act[r1], 0) * p.ldb + kq;
        pb1h = p.Bhi + bo1;
        pb1l = p.Blo + bo1;
    }
    uint4 ga0h, ga0l, gb0h, gb0l, ga1h, ga1l, gb1h, gb1l;
    auto gload_step = [&](int k0) {
        ga0h = *(const uint4*)(pa0h + k0); ga0l = *(const uint4*)(pa0l + k0);
        gb0h = *(const uint4*)(pb0h + k0); gb0l = *(const uint4*)(pb0l + k0);
        if constexpr (NL > 1) {
            ga1h = *(const uint4*)(pa1h + k0); ga1l = *(const uint4*)(pa1l + k0);
            gb1h = *(const uint4*)(pb1h + k0); gb1l = *(const uint4*)(pb1l + k0);
        }
    };
    auto lds_store = [&](int buf) {
        u16* const sAh = sbase + (size_t)buf * 4 * kTile;
        u16* const sAl = sAh + kTile;
        u16* const sBh = sAl + kTile;
        u16* const sBl = sBh + kTile;
        *(uint4*)&sAh[srow0] = ga0h;
        *(uint4*)&sAl[srow0] = ga0l;
        *(uint4*)&sBh[srow0] = gb0h;
        *(uint4*)&sBl[srow0] = gb0l;
        if constexpr (NL > 1) {
            *(uint4*)&sAh[srow1] = ga1h;
            *(uint4*)&sAl[srow1] = ga1l;
            *(uint4*)&sBh[srow1] = gb1h;
            *(uint4*)&sBl[srow1] = gb1l;
        }
    };

    const int wr = wave / WC, wc = wave % WC;
    const int lr = lane & 15, lc = lane >> 4;
    f4 acc[NBR][NBC];
#pragma unroll
    for (int a = 0; a < NBR; ++a)
#pragma unroll
        for (int b = 0; b < NBC; ++b) acc[a][b] = (f4){0.f, 0.f, 0.f, 0.f};

    // K steps: step s is multiplied out of buffer s % 2 while step s + 1 is
    // stored into the other buffer and step s + 2 is loaded into registers;
    // one barrier per step.
    gload_step(0);
    lds_store(0);
    __syncthreads();
    if (kG3K < p.K) gload_step(kG3K);
    for (int k0 = 0, buf = 0; k0 < p.K; k0 += kG3K, buf ^= 1) {
        const u16* const sAh = sbase + (size_t)buf * 4 * kTile;
        const u16* const sAl = sAh + kTile;
        const u16* const sBh = sAl + kTile;
        const u16* const sBl = sBh + kTile;
        bf8v ah[NBR], al[NBR], bh[NBC], bl[NBC];
#pragma unroll
        for (int q = 0; q < NBR; ++q) {
            const int ra_ = soff(wr * WTR + q * 16 + lr, lc);
            ah[q] = *(const bf8v*)&sAh[ra_];
            al[q] = *(const bf8v*)&sAl[ra_];
        }
#pragma unroll
        for (int q = 0; q < NBC; ++q) {
            const int rb_ = soff(wc * WTC + q * 16 + lr, lc);
            bh[q] = *(const bf8v*)&sBh[rb_];
            bl[q] = *(const bf8v*)&sBl[rb_];
        }
        if (k0 + kG3K < p.K) {
            lds_store(buf ^ 1);
            if (k0 + 2 * kG3K < p.K) gload_step(k0 + 2 * kG3K);
        }
#pragma unroll
        for (int a = 0; a < NBR; ++a)
#pragma unroll
            for (int b = 0; b < NBC; ++b) {
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
            }
        __syncthreads();
    }

    // Epilogue, CC columns at a time: the waves owning those columns put
    // their accumulators into LDS (column-major; a lane holds rows r..r+3 of
    // one column of each 16 x 16 block), then all threads walk the columns
    // with consecutive lanes on consecutive rows.
#pragma unroll
    for (int h = 0; h < TM / CC; ++h) {
        if (h > 0) __syncthreads();           // previous chunk fully consumed
        if ((wc * WTC) / CC == h) {
#pragma unroll
            for (int cb = 0; cb < NBC; ++cb)
#pragma unroll
                for (int a = 0; a < NBR; ++a)
                    *(f4*)&sC[(wc * WTC - h * CC + cb * 16 + lr) * kCLd + wr * WTR + a * 16 + 4 * lc] = acc[a][cb];
        }
        __syncthreads();
        if (EPI == 0) {
            for (int idx = tid; idx < CC * TM; idx += NT) {
                const int cl = idx / TM, rl = idx % TM;
                const int b = s_act[h * CC + cl];
                if (b < 0) break;             // inactive columns are the last ones of the tile
                const int j = row0 + rl;
                short hh, ll;
                split_bf16(sC[cl * kCLd + rl], hh, ll);
                p.Ohi[(long long)b * p.ldo + j] = (u16)hh;
                p.Olo[(long long)b * p.ldo + j] = (u16)ll;
            }
        } else {
            // EU elements per thread at a time: every load of the batch is
            // issued before the first element is updated
            constexpr int EU = 4;
            for (int base = tid; base < CC * TM; base += NT * EU) {
                long long e[EU];
                bool ok[EU];
                float gv[EU];
                double xv[EU];
                signed char sv[EU];
#pragma unroll
                for (int u = 0; u < EU; ++u) {
                    const int idx = base + NT * u;
                    const int cl = idx / TM, rl = idx % TM;
                    const int b = (idx < CC * TM) ? s_act[h * CC + cl] : -1;
                    const int j = row0 + rl;
                    ok[u] = b >= 0 && j < p.n;
                    const long long bb = ok[u] ? b : 0;
                    const int jj = ok[u] ? j : 0;
                    e[u] = jj + bb * p.n;
                    gv[u] = p.G[e[u]];
                    xv[u] = p.X[e[u]];
                    sv[u] = p.sat[jj + bb * p.ldsat];
                }
#pragma unroll
                for (int u = 0; u < EU; ++u) {
                    if (!ok[u]) continue;
                    const int idx = base + NT * u;
                    const int cl = idx / TM, rl = idx % TM;
                    const int b = s_act[h * CC + cl];
                    const int j = row0 + rl;
                    const float g = gv[u] - sC[cl * kCLd + rl];
                    p.G[e[u]] = g;
                    const double xn = (sv[u] != 0) ? 0.0 : fmax(0.0, xv[u] + p.eta * (double)g);
                    p.X[e[u]] = xn;
                    short hh, ll;
                    split_bf16((float)(xn - xv[u]), hh, ll);
                    p.Ohi[(long long)b * p.ldo + j] = (u16)hh;
                    p.Olo[(long long)b * p.ldo + j] = (u16)ll;
                }
            }
        }
    }
}

// Launch one GEMM of an iteration: 128 x 128 tiles on 8 waves, or 64 x 64
// tiles on 4 waves when the larger ones would leave most of the chip idle
// (fewer tiles than CUs).
template <int EPI>
static void launch_gemm3(G3Args g, long Mpad, int nact, int cus, hipStream_t s)
{
    const int t128 = (int)(Mpad / 128) * ((nact + 127) / 128);
    if (t128 >= cus) {
        g.tiles_m = (int)(Mpad / 128);
        g.tiles_n = (nact + 127) / 128;
        k_gemm3<EPI, 128, 2, 4><<<g.tiles_m * g.tiles_n, 512, 0, s>>>(g);
    } else {
        g.tiles_m = (int)(Mpad / 64);
        g.tiles_n = (nact + 63) / 64;
        k_gemm3<EPI, 64, 2, 2><<<g.tiles_m * g.tiles_n, 256, 0, s>>>(g);
    }
}

// bf16 hi/lo splits of the FP32 matrix in both K-contiguous layouts:
//   AR (row-major, mpad x npad): AR[i * npad + j] = A[i, j]
//   AC (column-major, npad x mpad): AC[j * mpad + i] = A[i, j]
// zero outside m x n.  32 x 32 tiles through LDS for the transposed write.
__global__ __launch_bounds__(256)
void k_b_split_a(const float* __restrict__ A, long long lda, int m, int n, int mpad, int npad,
                 u16* __restrict__ ARh, u16* __restrict__ ARl, u16* __restrict__ ACh, u16* __restrict__ ACl)
{
    __shared__ float tile[32][33];
    const int i0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int jj = ty; jj < 32; jj += 8) {
        const int i = i0 + tx, j = j0 + jj;
        const float v = (i < m && j < n) ? A[i + (long long)j * lda] : 0.f;
        tile[jj][tx] = v;
        short h, l;
        split_bf16(v, h, l);
        ACh[(long long)j * mpad + i] = (u16)h;
        ACl[(long long)j * mpad + i] = (u16)l;
    }
    __syncthreads();
    for (int ii = ty; ii < 32; ii += 8) {
        const int i = i0 + ii, j = j0 + tx;
        short h, l;
        split_bf16(tile[tx][ii], h, l);
        ARh[(long long)i * npad + j] = (u16)h;
        ARl[(long long)i * npad + j] = (u16)l;
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
// an ulp of x); the increment D = x_new - x feeds the GEMMs as its bf16 hi/lo
// split.  This kernel takes the first step of a pass, from the exact
// gradient; the later steps are fused into the epilogue of k_gemm3<1>.
__global__ void k_b_step_split(double* __restrict__ X64, const float* __restrict__ G32, int n,
                               const int* __restrict__ act, const int* __restrict__ nact_ptr,
                               const signed char* __restrict__ sat, long long ldsat, double eta,
                               u16* __restrict__ Dhi, u16* __restrict__ Dlo, long long ldd)
{
    const long long tot = (long long)n * (*nact_ptr);
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < tot; k += (long long)gridDim.x * blockDim.x) {
        const int j = (int)(k % n);
        const long long b = act[k / n];
        const long long e = j + b * n;
        const double xo = X64[e];
        const double xn = (sat[j + b * ldsat] != 0) ? 0.0 : fmax(0.0, xo + eta * (double)G32[e]);
        X64[e] = xn;
        short h, l;
        split_bf16((float)(xn - xo), h, l);
        Dhi[j + b * ldd] = (u16)h;
        Dlo[j + b * ldd] = (u16)l;
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

// one power-iteration step on A^T A (FP64 GEMV pair of dgemm.hip) is
// followed by this kernel: it normalises v and records the Rayleigh quotient.
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

// compact the active right-hand-side list (one workgroup, order kept); with
// host_words set, then publish the active count and the stop counter to
// coherent host memory and, last, with a system-scope release, the number of
// passes run (the host waits on that word instead of a synchronisation)
__global__ __launch_bounds__(1024)
void k_b_compact_rhs(int B, const BState* __restrict__ st, int* __restrict__ act, int* __restrict__ nact,
                     const int* __restrict__ done_counter, int* __restrict__ host_words, int seq)
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
    if (tid == 0) {
        *nact = out;
        if (host_words) {
            host_words[1] = out;
            host_words[2] = *done_counter;
            __threadfence_system();
            __hip_atomic_store(host_words, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

// coordinates with x_jb > 0 per right-hand side (BState::pad0), one workgroup each
__global__ __launch_bounds__(256)
void k_b_count_free(const double* __restrict__ X64, int n, BState* __restrict__ st)
{
    __shared__ int sh[4];
    const long long b = blockIdx.x;
    int c = 0;
    for (int j = threadIdx.x; j < n; j += 256) c += X64[j + b * n] > 0.0 ? 1 : 0;
    for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) st[b].pad0 = sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ void k_b_iota(int* __restrict__ act, int B, int* __restrict__ nact)
{
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < B; b += gridDim.x * blockDim.x) act[b] = b;
    if (blockIdx.x == 0 && threadIdx.x == 0) *nact = B;
}

// ---------------------------------------------------------------------------
// host driver
// ---------------------------------------------------------------------------
struct DgemmArgs {
    const double* A;
    long long lda;
    const double* B;
    long long ldb;
    double* C;
    long long ldc;
    const double* Cin;
    long long ldcin;
    int M, N, K;
    double alpha, beta;
    const int* cols;
    const int* ncols;
    double* splitk;
    int kparts, kslice;
};
hipError_t launch_dgemm(int ta, int tb, const DgemmArgs& a, hipStream_t s);   // dgemm.hip
size_t dgemm_splitk_doubles();
size_t dgemv_partial_doubles(long m, long n);
hipError_t launch_dgemv_normal(const double* A, long long lda, int m, int n, const double* v, double* w,
                               double* partial, double* out, hipStream_t s);

// C[M x N] = alpha op(A) op(B) + beta Cin (Cin = C when nullptr), FP64;
// `splitk` (dgemm_splitk_doubles() doubles) lets small products split K
static DgemmArgs gemm_args(double* splitk, const double* A, long long lda, const double* B, long long ldb, double* C,
                           long long ldc, long M, long N, long K, double alpha, double beta,
                           const double* Cin = nullptr, long long ldcin = 0, const int* cols = nullptr,
                           const int* ncols = nullptr)
{
    DgemmArgs a;
    a.A = A; a.lda = lda; a.B = B; a.ldb = ldb; a.C = C; a.ldc = ldc; a.Cin = Cin; a.ldcin = ldcin;
    a.M = (int)M; a.N = (int)N; a.K = (int)K; a.alpha = alpha; a.beta = beta; a.cols = cols; a.ncols = ncols;
    a.splitk = splitk; a.kparts = 1; a.kslice = (int)K;
    return a;
}

#define BXS_HIPB(call)                                                                           \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) return set_error(BXS_ERR_DEVICE, hipGetErrorString(e_));           \
    } while (0)

static size_t al(size_t v) { return (v + 255) / 256 * 256; }
static size_t pad128(long v) { return (size_t)((v + 127) / 128 * 128); }

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
        const size_t mp = pad128(m), np = pad128(n);
        b += al(sizeof(u16) * mp * np) * 4;   // bf16 hi/lo splits of A, row- and column-major
        b += al(sizeof(u16) * np * B) * 2;    // D hi/lo (step increment)
        b += al(sizeof(u16) * mp * B) * 2;    // U hi/lo = A D
        b += al(sizeof(float) * n * B);       // G32
    }
    b += al(sizeof(double) * (4 * (size_t)n + m + 16));   // cn, w, power vectors, scalars
    b += al(sizeof(double) * dgemv_partial_doubles(m, n));  // power-iteration partial products
    b += al(sizeof(double) * dgemm_splitk_doubles());        // split-K slices of small GEMMs
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
    float *X32 = nullptr, *G32 = nullptr, *Y32 = nullptr;
    const long mp = (long)pad128(m), np = (long)pad128(n);
    u16 *ARh = nullptr, *ARl = nullptr, *ACh = nullptr, *ACl = nullptr;
    u16 *Dh = nullptr, *Dl = nullptr, *Uh = nullptr, *Ul = nullptr;
    if (prec == 1) {
        ARh = (u16*)take(sizeof(u16) * mp * np);
        ARl = (u16*)take(sizeof(u16) * mp * np);
        ACh = (u16*)take(sizeof(u16) * mp * np);
        ACl = (u16*)take(sizeof(u16) * mp * np);
        Dh = (u16*)take(sizeof(u16) * np * B);
        Dl = (u16*)take(sizeof(u16) * np * B);
        Uh = (u16*)take(sizeof(u16) * mp * B);
        Ul = (u16*)take(sizeof(u16) * mp * B);
        G32 = (float*)take(sizeof(float) * n * B);
    }
    double* sc = (double*)take(sizeof(double) * (4 * (size_t)n + m + 16));
    double* cn = sc;
    double* w = sc + n;
    double* pv = sc + 2 * n;         // n
    double* pav = sc + 3 * n;        // m (A v)
    double* scal = sc + 3 * n + m;   // [0] tnorm, [1] lambda
    double* gv_part = (double*)take(sizeof(double) * dgemv_partial_doubles(m, n));
    double* skw = (double*)take(sizeof(double) * dgemm_splitk_doubles());
    BState* st = (BState*)take(sizeof(BState) * B);
    int* ints = (int*)take(sizeof(int) * (B + 16));
    int* act = ints;
    int* nact = ints + B;
    int* done_counter = ints + B + 1;
    int* err = ints + B + 2;
    const long long lda32 = (a_dtype == BXS_F32) ? lda : m;   // A32 layout

    bxs_status bs = BXS_OK;
    hipEvent_t e0, e1, e2;
    BXS_HIPB(hipEventCreate(&e0));
    BXS_HIPB(hipEventCreate(&e1));
    BXS_HIPB(hipEventCreate(&e2));
    struct EG { hipEvent_t a, b, c; ~EG() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); (void)hipEventDestroy(c); } } eg{e0, e1, e2};
    double ev_over = 0.0;
    if (o->profile) {
        bxs_status bs_ev = event_overhead(s, &ev_over);
        if (bs_ev != BXS_OK) return bs_ev;
    }
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
    if (prec == 1) {
        dim3 gs((unsigned)(mp / 32), (unsigned)(np / 32));
        k_b_split_a<<<gs, 256, 0, s>>>(A32, lda32, (int)m, (int)n, (int)mp, (int)np, ARh, ARl, ACh, ACl);
        BXS_HIPB(hipMemsetAsync(Dh, 0, sizeof(u16) * np * B, s));
        BXS_HIPB(hipMemsetAsync(Dl, 0, sizeof(u16) * np * B, s));
    }
    BXS_HIPB(hipGetLastError());

    // step: power iteration on A^T A with FP64 GEMVs (unless given)
    double eta = o->step;
    double lam_h = 0.0;
    if (!(eta > 0.0)) {
        k_b_init_vec<<<16, 256, 0, s>>>(pv, (int)n);
        const int np = o->power_iters > 0 ? o->power_iters : 20;
        for (int k = 0; k < np; ++k) {
            // pav = A v, v <- A^T pav, then normalise
            BXS_HIPB(launch_dgemv_normal(A64, m, (int)m, (int)n, pv, pav, gv_part, pv, s));
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

    // R = Y - A X and G = A^T R on the active right-hand sides (the list
    // `act` and its device count; hnact bounds the count from the host)
    int hnact = (int)B;
    auto residual_and_corr = [&]() -> bxs_status {
        BXS_HIPB(launch_dgemm(0, 0, gemm_args(skw, A64, m, X64, n, R64, m, m, hnact, n, -1.0, 1.0, Y64, m, act, nact), s));
        BXS_HIPB(launch_dgemm(1, 0, gemm_args(skw, A64, m, R64, m, G64, n, n, hnact, m, 1.0, 0.0, nullptr, 0, act, nact),
                              s));
        return BXS_OK;
    };

    if (prec == 1) {
        bs = residual_and_corr();
        if (bs != BXS_OK) return bs;
        k_b_g64_to_32<<<grid, 256, 0, s>>>(G64, G32, (int)n, act, nact);
    }
    int cus = 256;
    {
        int dev = 0;
        BXS_HIPB(hipGetDevice(&dev));
        BXS_HIPB(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    }
    // Coherent host words the compaction kernel publishes after every pass:
    // [0] passes run, [1] active right-hand sides, [2] stopped ones.
    int* hw = nullptr;
    {
        static thread_local struct Words {
            int* p = nullptr;
            ~Words() { if (p) (void)hipHostFree(p); }
        } words;
        if (!words.p) BXS_HIPB(hipHostMalloc((void**)&words.p, 64, hipHostMallocCoherent));
        hw = words.p;
    }
    __atomic_store_n(&hw[0], 0, __ATOMIC_RELEASE);
    int hcnt[2] = {(int)B, 0};          // profile mode: copied back after each pass
    const int K = o->screen_every;
    long long iters = 0;
    // Passes are enqueued one ahead of the host's stop check (its GEMM grids
    // are sized from the active count of the pass before, an upper bound; the
    // kernels bound themselves by the device count).  Profile mode
    // synchronises every pass to read its events.
    const bool ahead = !o->profile;
    // optional HIP-event timing of the iteration GEMM pairs
    std::vector<hipEvent_t> pev;
    struct PG2 { std::vector<hipEvent_t>* v; ~PG2() { for (auto e : *v) if (e) (void)hipEventDestroy(e); } } pg2{&pev};
    if (o->profile) {
        pev.assign(2 * (size_t)K, nullptr);
        for (auto& e : pev) BXS_HIPB(hipEventCreate(&e));
    }
    double gemm_ms = 0.0;
    long gemm_pairs = 0;
    std::vector<long long> pass_kk;      // per enqueued pass: iterations
    std::vector<int> pass_final;
    auto enqueue_pass = [&](int seq) -> bxs_status {
        const long long kk = std::min<long long>(K, o->max_iter - iters);
        if (prec == 1) {
            // step 1 from the exact gradient, then kk-1 x [U = A D; G -= A^T U and step]
            if (kk > 0)
                k_b_step_split<<<grid, 256, 0, s>>>(X64, G32, (int)n, act, nact, sat, ldsat, eta, Dh, Dl, np);
            G3Args g0{};
            g0.Ahi = ARh; g0.Alo = ARl; g0.lda = np; g0.K = (int)np; g0.act = act; g0.nact = hnact;
            g0.nact_dev = nact;
            g0.Bhi = Dh; g0.Blo = Dl; g0.ldb = np; g0.Ohi = Uh; g0.Olo = Ul; g0.ldo = mp;
            G3Args g1{};
            g1.Ahi = ACh; g1.Alo = ACl; g1.lda = mp; g1.K = (int)mp; g1.act = act; g1.nact = hnact;
            g1.nact_dev = nact;
            g1.Bhi = Uh; g1.Blo = Ul; g1.ldb = mp; g1.Ohi = Dh; g1.Olo = Dl; g1.ldo = np;
            g1.G = G32; g1.X = X64; g1.sat = sat; g1.ldsat = ldsat; g1.n = (int)n; g1.eta = eta;
            for (long long k = 1; k < kk && hnact > 0; ++k) {
                if (o->profile) BXS_HIPB(hipEventRecord(pev[2 * k], s));
                launch_gemm3<0>(g0, mp, hnact, cus, s);
                launch_gemm3<1>(g1, np, hnact, cus, s);
                if (o->profile) BXS_HIPB(hipEventRecord(pev[2 * k + 1], s));
            }
        } else {
            for (long long k = 0; k < kk; ++k) {
                if (o->profile) BXS_HIPB(hipEventRecord(pev[2 * k], s));
                bxs_status b2 = residual_and_corr();
                if (b2 != BXS_OK) return b2;
                if (o->profile) BXS_HIPB(hipEventRecord(pev[2 * k + 1], s));
                k_b_update64<<<grid, 256, 0, s>>>(X64, G64, (int)n, (int)B, sat, ldsat, st, eta);
            }
        }
        iters += kk;
        bxs_status b3 = residual_and_corr();
        if (b3 != BXS_OK) return b3;
        const int final_pass = iters >= o->max_iter;
        k_b_screen<<<(int)B, 256, 0, s>>>((int)m, (int)n, (int)B, R64, G64, X64, X32, Y64, cn, w, scal, sat, ldsat, st,
                                          done_counter, o->eps_gap, o->screening, final_pass, iters, (int)kk);
        k_b_compact_rhs<<<1, 1024, 0, s>>>((int)B, st, act, nact, done_counter, ahead ? hw : nullptr, seq);
        // the next pass of the BF16x3 engine restarts from the exact gradient
        if (prec == 1) k_b_g64_to_32<<<grid, 256, 0, s>>>(G64, G32, (int)n, act, nact);
        BXS_HIPB(hipGetLastError());
        if (!ahead) {
            BXS_HIPB(hipMemcpyAsync(hcnt, nact, sizeof(int), hipMemcpyDeviceToHost, s));
            BXS_HIPB(hipMemcpyAsync(hcnt + 1, done_counter, sizeof(int), hipMemcpyDeviceToHost, s));
        }
        pass_kk.push_back(kk);
        pass_final.push_back(final_pass);
        return BXS_OK;
    };

    bs = enqueue_pass(1);
    if (bs != BXS_OK) return bs;
    for (int cur = 1;; ++cur) {
        // the next pass goes out before this one is waited for
        if (ahead && !pass_final[cur - 1]) {
            bs = enqueue_pass(cur + 1);
            if (bs != BXS_OK) return bs;
        }
        int n_active = 0, n_done = 0;
        if (ahead) {
            const auto t0 = std::chrono::steady_clock::now();
            long spins = 0;
            while (__atomic_load_n(&hw[0], __ATOMIC_ACQUIRE) < cur) {
                __builtin_ia32_pause();
                // should the word not advance (it always does), the stream's
                // completion makes every published value final
                if ((++spins & 4095) == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::seconds(2)) {
                    BXS_HIPB(hipStreamSynchronize(s));
                    break;
                }
            }
            n_active = __atomic_load_n(&hw[1], __ATOMIC_ACQUIRE);
            n_done = __atomic_load_n(&hw[2], __ATOMIC_ACQUIRE);
        } else {
            BXS_HIPB(hipStreamSynchronize(s));
            n_active = hcnt[0];
            n_done = hcnt[1];
            for (long long k = (prec == 1) ? 1 : 0; k < pass_kk[cur - 1]; ++k) {
                float ms = 0.f;
                BXS_HIPB(hipEventElapsedTime(&ms, pev[2 * k], pev[2 * k + 1]));
                gemm_ms += ms;
                ++gemm_pairs;
            }
        }
        hnact = n_active;
        if (n_done >= B || pass_final[cur - 1]) break;
        if (!ahead) {
            bs = enqueue_pass(cur + 1);
            if (bs != BXS_OK) return bs;
        }
    }
    k_b_output<<<grid, 256, 0, s>>>(X64, X, ldx, (int)n, (int)B);
    k_b_count_free<<<(int)B, 256, 0, s>>>(X64, (int)n, st);
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
            f.event_overhead_ms = ev_over;
            f.t_column = -1;
            f.dual = S.primal - S.gap;
            f.n_free = S.pad0;       // coordinates strictly inside the box (x_jb > 0)
        }
    }
    return worst;
}

}  // namespace bxs

// ---------------------------------------------------------------------------
// Adjoint of the batched box-constrained solution map (implicit
// differentiation), with bounds l, u shared by the right-hand sides (NNLS:
// l = 0, u = +inf).  At an optimum with free set F_b = {j : l_j < x_jb < u_j}
// the optimality conditions (Sec. 3.2, eq. optimality2: a_j^T (y_b - A x_b)
// = 0 on F_b) give x_F = (A_F^T A_F)^{-1} A_F^T (y_b - A_S x_S), hence for dL/dX:
//     v_b      = (A_F^T A_F)^{-1} (dL/dx_b)_F      (batched masked CG, FP64)
//     dL/dy_b  = A v_b  (v_b = 0 off F_b)
//     dL/dA    = R V^T - (dL/dY) X^T,   R = Y - A X
//     dL/dl_jb = (dL/dx_b - A^T dL/dy_b)_j at a lower bound, dL/du likewise at an upper one
// ---------------------------------------------------------------------------
namespace bxs {

__global__ void k_adj_init(const double* __restrict__ X, long long ldx, const double* __restrict__ dX, long long ldg,
                           const double* __restrict__ l, const double* __restrict__ u,
                           int n, int B, double* __restrict__ V, double* __restrict__ Rc, double* __restrict__ P,
                           signed char* __restrict__ F)
{
    const long long tot = (long long)n * B;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < tot; k += (long long)gridDim.x * blockDim.x) {
        const int j = (int)(k % n);
        const long long b = k / n;
        const double xj = X[j + b * ldx];
        const bool free_ = xj > (l ? l[j] : 0.0) && xj < (u ? u[j] : __builtin_inf());
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

// p^T S and p^T p per right-hand side
__global__ __launch_bounds__(256)
void k_adj_dot2(const double* __restrict__ P, const double* __restrict__ S, int n, double* __restrict__ pq,
                double* __restrict__ pp)
{
    __shared__ double sh[2][4];
    const long long b = blockIdx.x;
    double s = 0.0, q = 0.0;
    for (int j = threadIdx.x; j < n; j += 256) {
        const double v = P[j + b * n];
        s = fma(v, S[j + b * n], s);
        q = fma(v, v, q);
    }
    for (int off = 32; off >= 1; off >>= 1) {
        s += __shfl_xor(s, off, 64);
        q += __shfl_xor(q, off, 64);
    }
    if ((threadIdx.x & 63) == 0) { sh[0][threadIdx.x >> 6] = s; sh[1][threadIdx.x >> 6] = q; }
    __syncthreads();
    if (threadIdx.x == 0) {
        pq[b] = (sh[0][0] + sh[0][1]) + (sh[0][2] + sh[0][3]);
        pp[b] = (sh[1][0] + sh[1][1]) + (sh[1][2] + sh[1][3]);
    }
}

// sum of squares of the m x n matrix (an upper bound of the largest
// eigenvalue of every masked normal matrix A_F^T A_F); one workgroup
__global__ __launch_bounds__(1024)
void k_adj_frob(const double* __restrict__ A, long long count, double* __restrict__ out)
{
    __shared__ double sh[16];
    double s = 0.0;
    for (long long k = threadIdx.x; k < count; k += 1024) s = fma(A[k], A[k], s);
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < 16; ++w) t += sh[w];
        *out = t;
    }
}

// S <- mask(S); alpha = rs / (p.S); V += alpha P; Rc -= alpha S.  A column
// whose flag is set (converged or broken down) is frozen, and so is one whose
// p^T S is at the rounding level (it is flagged by k_adj_track next).
__global__ void k_adj_step(double* __restrict__ S, const signed char* __restrict__ F, const double* __restrict__ rs,
                           const double* __restrict__ pq, const double* __restrict__ pp, const double* __restrict__ frob,
                           int m, const int* __restrict__ done, double* __restrict__ V,
                           double* __restrict__ Rc, const double* __restrict__ P, int n, int B)
{
    const double floor_ = 2.0 * gamma_k((double)m + 2.0) * (*frob);
    const long long tot = (long long)n * B;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < tot; k += (long long)gridDim.x * blockDim.x) {
        const long long b = k / n;
        if (done[b] || !(pq[b] > floor_ * pp[b])) continue;
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
// its residual fell below tol^2 * rs0 (done = 1), or broke down (done = 2):
// p^T A_F^T A_F p at or below the rounding level of its FP64 evaluation,
// taken as 2 gamma_m |p|^2 ||A||_F^2 (A_F rank deficient along p), or a
// non-finite value.
__global__ void k_adj_track(double* __restrict__ rs, const double* __restrict__ rsn, const double* __restrict__ rs0,
                            const double* __restrict__ pq, const double* __restrict__ pp, const double* __restrict__ frob,
                            int m, int* __restrict__ done, int B, double tol2)
{
    const double floor_ = 2.0 * gamma_k((double)m + 2.0) * (*frob);
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < B; b += gridDim.x * blockDim.x) {
        if (done[b]) continue;
        const double r = rsn[b];
        if (!(pq[b] > floor_ * pp[b]) || !isfinite(r)) { done[b] = 2; continue; }
        rs[b] = r;
        if (r <= tol2 * rs0[b]) done[b] = 1;
    }
}

// the gradient of a broken-down column is set to 0 (no valid solve)
__global__ void k_adj_zero_broken(double* __restrict__ V, const int* __restrict__ done, int n, int B)
{
    const long long tot = (long long)n * B;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < tot; k += (long long)gridDim.x * blockDim.x)
        if (done[k / n] == 2) V[k] = 0.0;
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
    b += al(sizeof(double) * B) * 5;       // rs, rs0, pq, rs_new, pp
    b += al(sizeof(double) * 4);           // ||A||_F^2
    b += al(sizeof(int) * B);              // done
    b += al(sizeof(int) * 16);
    b += al(sizeof(double) * dgemm_splitk_doubles());   // split-K slices of small GEMMs
    return b + 1024;
}

// dL/dl = dL/dx - A^T dL/dy on the coordinates at their lower bound, dL/du
// the same at the upper bound, 0 elsewhere (either output may be NULL)
__global__ void k_adj_bound_grad(const double* __restrict__ dX, long long ldg, const double* __restrict__ AtdY,
                                 const signed char* __restrict__ F, const double* __restrict__ X, long long ldx,
                                 const double* __restrict__ l, const double* __restrict__ u, int n, int B,
                                 double* __restrict__ dl, long long lddl, double* __restrict__ du, long long lddu)
{
    const long long tot = (long long)n * B;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < tot; k += (long long)gridDim.x * blockDim.x) {
        const int j = (int)(k % n);
        const long long b = k / n;
        const double c = F[k] ? 0.0 : dX[j + b * ldg] - AtdY[k];
        const double xj = X[j + b * ldx];
        if (dl) dl[j + b * lddl] = (xj <= (l ? l[j] : 0.0)) ? c : 0.0;
        if (du) du[j + b * lddu] = (xj >= (u ? u[j] : __builtin_inf())) ? c : 0.0;
    }
}

bxs_status adjoint_run(long m, long n, long B, int a_dtype, const void* A, long lda, const double* Y, long ldy,
                       const double* X, long ldx, const double* l, const double* u, const double* dX, long ldg,
                       double* dY, long lddy, double* dA, long ldda, double* dl, long lddl, double* du, long lddu,
                       const bxs_opts* o, long* cg_iters)
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
    double* pp = (double*)take(sizeof(double) * B);
    double* frob = (double*)take(sizeof(double) * 4);
    int* done = (int*)take(sizeof(int) * B);
    int* counters = (int*)take(sizeof(int) * 16);
    double* skw = (double*)take(sizeof(double) * dgemm_splitk_doubles());

    const int grid = 2048;
    if (a_dtype == BXS_F32)
        k_b_convert_a<float><<<grid, 256, 0, s>>>((const float*)A, lda, (int)m, (int)n, A64, nullptr);
    else
        k_b_convert_a<double><<<grid, 256, 0, s>>>((const double*)A, lda, (int)m, (int)n, A64, nullptr);
    k_adj_copy2<<<grid, 256, 0, s>>>(X, ldx, Xc, n, (int)n, (int)B);
    k_adj_init<<<grid, 256, 0, s>>>(X, ldx, dX, ldg, l, u, (int)n, (int)B, V, Rc, P, F);
    k_adj_dot<<<(int)B, 256, 0, s>>>(Rc, Rc, (int)n, rs);
    k_b_copy<<<64, 256, 0, s>>>(rs, rs0, B);
    k_adj_frob<<<1, 1024, 0, s>>>(A64, (long long)m * n, frob);
    BXS_HIPB(hipMemsetAsync(done, 0, sizeof(int) * B, s));
    BXS_HIPB(hipGetLastError());
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
        BXS_HIPB(launch_dgemm(0, 0, gemm_args(skw, A64, m, P, n, Q, m, m, B, n, 1.0, 0.0), s));
        BXS_HIPB(launch_dgemm(1, 0, gemm_args(skw, A64, m, Q, m, S, n, n, B, m, 1.0, 0.0), s));
        k_adj_mask<<<grid, 256, 0, s>>>(S, F, (long long)n * B);
        k_adj_dot2<<<(int)B, 256, 0, s>>>(P, S, (int)n, pq, pp);
        k_adj_step<<<grid, 256, 0, s>>>(S, F, rs, pq, pp, frob, (int)m, done, V, Rc, P, (int)n, (int)B);
        k_adj_dot<<<(int)B, 256, 0, s>>>(Rc, Rc, (int)n, rsn);
        k_adj_dir<<<grid, 256, 0, s>>>(P, Rc, rsn, rs, done, (int)n, (int)B);
        k_adj_track<<<(int)((B + 255) / 256), 256, 0, s>>>(rs, rsn, rs0, pq, pp, frob, (int)m, done, (int)B,
                                                           tol * tol);
        if ((it % 8) == 7 || it + 1 == maxit) {
            BXS_HIPB(hipMemsetAsync(counters, 0, 2 * sizeof(int), s));
            k_adj_count<<<16, 256, 0, s>>>(done, (int)B, counters);
            BXS_HIPB(hipMemcpyAsync(hflag, counters, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
            BXS_HIPB(hipStreamSynchronize(s));
            if (hflag[0] == hflag[1]) { ++it; break; }   // every column converged or broke down
        }
    }
    k_adj_zero_broken<<<grid, 256, 0, s>>>(V, done, (int)n, (int)B);
    BXS_HIPB(hipGetLastError());
    // dL/dY = A V
    BXS_HIPB(launch_dgemm(0, 0, gemm_args(skw, A64, m, V, n, dY, lddy, m, B, n, 1.0, 0.0), s));
    if (dA) {
        // R = Y - A X, then dL/dA = R V^T - (dL/dY) X^T
        BXS_HIPB(launch_dgemm(0, 0, gemm_args(skw, A64, m, Xc, n, R, m, m, B, n, -1.0, 1.0, Y, ldy), s));
        BXS_HIPB(launch_dgemm(0, 1, gemm_args(skw, R, m, V, n, dA, ldda, m, n, B, 1.0, 0.0), s));
        BXS_HIPB(launch_dgemm(0, 1, gemm_args(skw, dY, lddy, Xc, n, dA, ldda, m, n, B, -1.0, 1.0), s));
    }
    if (dl || du) {
        // S = A^T dL/dY (S is free once the CG is done)
        BXS_HIPB(launch_dgemm(1, 0, gemm_args(skw, A64, m, dY, lddy, S, n, n, B, m, 1.0, 0.0), s));
        k_adj_bound_grad<<<grid, 256, 0, s>>>(dX, ldg, S, F, Xc, n, l, u, (int)n, (int)B, dl, lddl, du, lddu);
        BXS_HIPB(hipGetLastError());
    }
    BXS_HIPB(hipStreamSynchronize(s));
    if (cg_iters) *cg_iters = it;
    if (hflag[1] > 0) return BXS_SINGULAR;
    return (hflag[0] == 0) ? BXS_OK : BXS_MAXITER;
}

}  // namespace bxs
