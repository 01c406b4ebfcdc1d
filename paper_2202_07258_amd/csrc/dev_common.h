// Device helpers shared by the gfx950 kernels of the boxscreen library:
// bound accessors, wave and block reductions with a fixed summation order,
// branch-free global loads and stores, and the wave-level reduce-scatter
// used by the column sweeps.
#pragma once

#include "bxs_internal.h"

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
// Low-latency wave sum through DPP lane moves (a few cycles each, against a
// round trip through the LDS crossbar for a shuffle): pairs within quads,
// then half rows and rows (mirrors), then the four rows through the row
// broadcasts, which leave the total in lane 63; v_readlane hands it to every
// lane.  The order is fixed, so the result repeats bit for bit.  Used where a
// reduction sits on a sequential critical path (coordinate descent).
template <int CTRL, int ROWM>
__device__ __forceinline__ double dpp_move(double v) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, ROWM, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, ROWM, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ double wave_sum_dpp(double v) {
    v += dpp_move<0xB1, 0xF>(v);     // quad_perm [1,0,3,2]
    v += dpp_move<0x4E, 0xF>(v);     // quad_perm [2,3,0,1]
    v += dpp_move<0x141, 0xF>(v);    // row_half_mirror: quads 0-1 / 2-3 of each row
    v += dpp_move<0x140, 0xF>(v);    // row_mirror: the two halves of each row
    v += dpp_move<0x142, 0xA>(v);    // row_bcast:15 into rows 1 and 3
    v += dpp_move<0x143, 0xC>(v);    // row_bcast:31 into rows 2 and 3
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, 63);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), 63);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
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

// Stores through a global address-space pointer: a store through a generic
// pointer is a flat store, which the compiler's wait-count tracking handles
// conservatively (it would wait for every outstanding load, including the
// next round's prefetch).
template <typename T>
__device__ __forceinline__ void gstore(T* p, T v) { *(__attribute__((address_space(1))) T*)p = v; }
template <typename T>
__device__ __forceinline__ T gload(const T* p) { return *(const __attribute__((address_space(1))) T*)p; }

// Branch-free form for the column sweeps: one vector load through a global
// address-space pointer, from row `row` if row < m and from row 0 otherwise,
// so the loads of the next round stay in flight while the current round is
// reduced (a load under a divergent branch is waited for inside the branch).
// Elements at rows >= m hold whatever the column's padding holds; the caller
// masks them before they can reach a stored result.
template <typename TA, int V>
__device__ __forceinline__ void load_pack_nb(const TA* __restrict__ col, int row, int m, TA (&o)[V]) {
    const int rr = (row < m) ? row : 0;
    if constexpr (V == 1) {
        o[0] = *(const __attribute__((address_space(1))) TA*)(col + rr);
    } else {
        typedef TA VecT __attribute__((ext_vector_type(V)));
        const VecT v = *(const __attribute__((address_space(1))) VecT*)(col + rr);
#pragma unroll
        for (int e = 0; e < V; ++e) o[e] = v[e];
    }
}

// ---------------------------------------------------------------------------
// Wave-level reduce-scatter of CBI per-lane partial sums: after log2(CBI)
// halving exchanges and the remaining butterfly steps, lane L holds the full
// 64-lane sum of column col_of_lane(L).  10 shuffles for CBI = 8 instead of 48
// for eight separate butterflies; the summation order is fixed.
// ---------------------------------------------------------------------------
template <int CBI>
struct Log2C { static constexpr int v = (CBI >= 8) ? 3 : (CBI >= 4) ? 2 : (CBI >= 2) ? 1 : 0; };

// One halving step S of the reduce-scatter, then recurse on the next step;
// the recursion makes every array index a compile-time constant.
template <int CBI, int S, bool END = (S >= Log2C<CBI>::v)>
struct ReduceScatterStep {
    static __device__ __forceinline__ void run(double (&v)[CBI], int lane) {
        constexpr int off = 32 >> S;
        constexpr int half = CBI >> (S + 1);
        const bool upper = (lane & off) != 0;
#pragma unroll
        for (int i = 0; i < half; ++i) {
            const double send = upper ? v[i] : v[i + half];
            const double keep = upper ? v[i + half] : v[i];
            v[i] = keep + __shfl_xor(send, off, 64);
        }
        ReduceScatterStep<CBI, S + 1>::run(v, lane);
    }
};
template <int CBI, int S>
struct ReduceScatterStep<CBI, S, true> {
    static __device__ __forceinline__ void run(double (&)[CBI], int) {}
};

template <int CBI>
__device__ __forceinline__ double wave_reduce_scatter(double (&v)[CBI], int lane) {
    constexpr int LOGC = Log2C<CBI>::v;
    ReduceScatterStep<CBI, 0>::run(v, lane);
    double s0 = v[0];
#pragma unroll
    for (int off = 32 >> LOGC; off >= 1; off >>= 1) s0 += __shfl_xor(s0, off, 64);
    return s0;
}

// An empty register constraint: the compiler must treat the value as new, so
// a column element is converted to FP64 once for the dot product and again
// for the update instead of keeping all converted values live in between.
__device__ __forceinline__ float opaque(float v) { asm volatile("" : "+v"(v)); return v; }
__device__ __forceinline__ double opaque(double v) { return v; }
__device__ __forceinline__ __bf16 opaque(__bf16 v) { return v; }

template <int CBI>
__device__ __forceinline__ int col_of_lane(int lane) { return (lane >> (6 - Log2C<CBI>::v)) & (CBI - 1); }
template <int CBI>
__device__ __forceinline__ int lane_of_col(int c) { return c << (6 - Log2C<CBI>::v); }

}  // namespace bxs
