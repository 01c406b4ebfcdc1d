// Internal device-side data structures of the boxscreen library (gfx950).
//
// A solve handles `count` independent problems ("instances") with one set of
// launches.  Per-instance constants live in `Inst`, per-instance mutable
// scalars (preserved-set size, gap, step, flags) in `State`; both are in
// device memory so that a pass never needs the host except to learn whether
// every instance has stopped.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "boxscreen.h"

namespace bxs {

// Columns of one instance are split into work items of `cb` consecutive
// positions of the preserved-set list; one workgroup handles one item and
// writes one partial m-vector.  cb is re-chosen after every compaction.
constexpr int kCbMin = 4;
constexpr int kCbMax = 256;

struct Inst {
    const void* A;          // column-major, element type given by the launch
    long long lda;
    int m, n;
    const double* y;        // [m]
    const double* l;        // [n] or nullptr (0)
    const double* u;        // [n] or nullptr (+inf)
    const double* t;        // [m] or nullptr (-1)
    double* x;              // [n] caller iterate (original index space)
    signed char* sat;       // [n]
    double* yp;             // [m] data with the screened part folded in (Remark 3)
    double* r;              // [m] residual yp - A_P x_P (or power-iteration vector)
    double* g;              // [n] correlations a_j^T r
    double* w;              // [n] a_j^T t
    double* cn;             // [n] rigorous upper bound of ||a_j||_2
    double* cn2;            // [n] FP64 sum of squares of column j (CD curvature)
    int* idx;               // [n] preserved set, ascending original index
    int* fidx;              // [n] columns screened by the last pass
    double* fval;           // [n] bound value of those columns
    double* fdx;            // [n] bound value minus the iterate before fixing
    double* part;           // [items_cap * m] partial A-products per work item
    double* part2;          // [items_cap * m] second partial (fold pass only)
    double* iscal;          // [items_cap] per-item scalar (power iteration)
    bxs_pass_record* rec;   // [rec_cap] per-pass records
    int rec_cap;
    int items_cap;          // ceil(n / kCbMin): grid extent reserved for this instance
    int g_target;           // workgroups the instance should spread over
    int item_base;          // first work item of this instance in its bucket list
};

struct State {
    int n_active;           // |P|
    int n_fold;             // columns screened by the last pass
    int cb;                 // columns per work item for the preserved set
    int cb_fold;            // columns per work item for the fold list
    int done;               // 1 once stopped (gap reached or budget spent)
    int status;             // bxs_status
    int t_valid;            // 0: theta = 0 fallback in use
    int err;                // input-validation flags (kErr*)
    int passes;
    int n_lower, n_upper;
    int pad_;
    long long iters;        // iterations done when the instance stopped
    long long col_iters;    // sum over primal iterations of n_active
    double step;            // PG step
    double lipschitz;       // power-iteration estimate of ||A||_2^2
    double gap, radius, eps, primal;
    double tnorm;           // upper bound of ||t||_2
    double ynorm;           // upper bound of ||y||_2
    double mass_screened;   // sum over screened j of |x_j| * cn_j
};

constexpr int kErrNonfinite = 1;
constexpr int kErrBounds = 2;

struct Item {               // one workgroup of a column sweep
    int inst;
    int t;                  // item index within the instance
};

struct RItem {              // one workgroup of a partial reduction
    int inst;
    int rb;                 // block of 64 rows
};

enum SweepMode : int {
    kModePG = 0,            // g = A^T r, x <- Pi(x + eta g), partial += A x
    kModeCorr = 1,          // g = A^T r stored
    kModeAx = 2,            // partial += A x
    kModeFold = 3,          // partial += A_S b_S, partial2 += A_S (b_S - x_S)
    kModePow = 4            // g = A^T r, partial += A g, iscal += ||g||^2
};

enum ReduceMode : int {
    kRedResidual = 0,       // r = yp - sum
    kRedFold = 1,           // yp -= sum, r -= sum2
    kRedPow = 2             // r = sum
};

// gamma_k = k u / (1 - k u), u = 2^-53: the standard bound on the relative
// error of a k-term floating-point sum or dot product (Higham, Accuracy and
// Stability of Numerical Algorithms, 2nd ed., Sec. 3.1).
__host__ __device__ inline double gamma_k(double k) {
    const double u = 1.1102230246251565e-16;
    return (k * u) / (1.0 - k * u);
}
constexpr double kUnit = 1.1102230246251565e-16;

// Depth of the summation tree of one column dot product in a sweep: R <= 16
// sequential FMAs per thread, a 6-level wave butterfly, and at most 16
// cross-wave additions.  The rounding error of every correlation a_j^T r is
// therefore at most gamma(kDotDepth) * sum_i |a_ij r_i|.
constexpr double kDotDepth = 64.0;

// Kernel instantiation buckets, chosen by the number of rows m:
// TPC threads share one column, NG column groups per workgroup,
// R rows per thread; capacity TPC * R rows.
struct BucketSpec { int tpc, ng, rows; };
constexpr int kNumBuckets = 9;
constexpr BucketSpec kBuckets[kNumBuckets] = {
    {64, 4, 1}, {64, 4, 2}, {64, 4, 4}, {64, 4, 8},
    {256, 1, 4}, {256, 1, 8}, {256, 1, 16},
    {512, 1, 16}, {1024, 1, 16},
};

inline int bucket_for_rows(long m) {
    for (int b = 0; b < kNumBuckets; ++b)
        if (m <= (long)kBuckets[b].tpc * kBuckets[b].rows) return b;
    return -1;
}

// Host-side launch helpers (defined in kernels.hip).
struct LaunchCtx {
    hipStream_t stream;
    int dtype;              // bxs_dtype
    int vec;                // 1: 16-byte loads of A are valid for every instance
    const Inst* insts;
    State* st;
    int* done_counter;
};

hipError_t launch_init(const LaunchCtx& c, int count, const double* x0_is_given);
hipError_t launch_colstats(const LaunchCtx& c, int bucket, const Item* items, int n_items);
hipError_t launch_sweep(const LaunchCtx& c, int bucket, int mode, const Item* items, int n_items);
hipError_t launch_reduce(const LaunchCtx& c, int mode, const RItem* ritems, int n_ritems);
hipError_t launch_pow_init(const LaunchCtx& c, int count);
hipError_t launch_set_step(const LaunchCtx& c, int count, double step);
hipError_t launch_pow_normalize(const LaunchCtx& c, int count, int last, double user_step);
hipError_t launch_screen(const LaunchCtx& c, int count, double eps_gap, int screening,
                         int final_pass, long long iters, int kk);
hipError_t launch_cd(const LaunchCtx& c, int bucket, const int* inst_list, int n_list, int sweeps);

}  // namespace bxs
