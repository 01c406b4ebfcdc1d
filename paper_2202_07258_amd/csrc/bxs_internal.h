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

// Lanczos steps of the ||A||_2^2 estimate when the caller gives no step.
constexpr int kLanczosDefault = 8;
constexpr int kLanczosMax = 64;

struct Inst {
    const void* A;          // column-major, element type given by the launch
    long long lda;
    int m, n;
    const double* y;        // [m]
    const double* l;        // [n] or nullptr (0)
    const double* u;        // [n] or nullptr (+inf)
    const double* t;        // [m] or nullptr (-1)
    const double* ts;       // [m] known dual optimum used in place of the dual update, or nullptr
    double* x;              // [n] caller iterate (original index space)
    signed char* sat;       // [n]
    double* yp;             // [m] data with the screened part folded in (Remark 3)
    double* r;              // [m] residual yp - A_P x_P (or the Lanczos vector)
    double* r2;             // [m] residual after the step taken ahead of a screening test
    double* xs;             // [n] iterate at the screening point (before that step)
    double* g;              // [n] correlations a_j^T r
    double* w;              // [n] a_j^T t
    double* gs;             // [n] a_j^T ts (when ts is given)
    double* cn;             // [n] rigorous upper bound of ||a_j||_2
    double* cn2;            // [n] FP64 sum of squares of column j (CD curvature)
    int* idx;               // [n] preserved set, ascending original index
    int* fidx;              // [n] columns screened by the last pass
    double* fval;           // [n] bound value of those columns
    double* fdx;            // [n] bound value minus the iterate before fixing
    double* part;           // [items_cap * m] partial A-products per work item
    double* part2;          // [items_cap * m] second partial (fold pass only)
    double* iscal;          // [items_cap * kItemScalars] per-item scalars of the screening pass
    bxs_pass_record* rec;   // [rec_cap] per-pass records
    int rec_cap;
    int items_cap;          // ceil(n / kCbMin): grid extent reserved for this instance
    int g_target;           // workgroups the instance should spread over
    int item_base;          // first work item of this instance in its bucket list
    int lz_steps;           // Lanczos steps of the ||A||_2^2 estimate (0: step given)
    double* lz;             // [2 lz_steps + 2 m] alpha, beta, q_k, q_{k-1}
    double hub;             // Huber threshold delta of the fidelity; +inf for least squares
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
    int ahead;              // 1: the step after the last screening pass is already taken
    long long iters;        // iterations done when the instance stopped
    long long col_iters;    // sum over primal iterations of n_active
    double step;            // PG step
    double lipschitz;       // Lanczos estimate of ||A||_2^2
    double gap, radius, eps, primal;
    double tnorm;           // upper bound of ||t||_2
    double tsnorm;          // upper bound of ||ts||_2
    double ynorm;           // upper bound of ||y||_2
    double mass_screened;   // sum over screened j of |x_j| * cn_j
    int t_column;           // column picked for t by the library (bxs_translation), or -1
    int n_free;             // coordinates strictly inside the box at exit
    double margin;          // last pass: rounding margin of a correlation per unit column norm
    int cdb_n;              // block CD: preserved-list length + 1 its Gram blocks were formed for
};

// Per-item scalars written by the correlation sweep for the screening pass:
// sum |x_j| ||a_j||, interior flag of t, largest translation ratio, presence
// of u_j = +inf columns, gap terms at eps = 0, largest screening score at
// eps = 0.
constexpr int kItemScalars = 8;
enum ItemScalar : int { kIsMass = 0, kIsTv = 1, kIsEmax = 2, kIsHasInf = 3, kIsGap0 = 4, kIsZmax0 = 5 };

constexpr int kErrNonfinite = 1;
constexpr int kErrBounds = 2;

struct Item {               // one workgroup of a column sweep
    int inst;
    int t;                  // item index within the instance
};

constexpr int kRedRows = 16;   // rows per workgroup of the partial reduction
constexpr int kRedRowsN = 256; // rows per workgroup of the narrow reduction (one thread per row)
constexpr int kRedNarrowMax = 64;   // instances with at most this many work items use it

struct RItem {              // one workgroup of a partial reduction
    int inst;
    int rb;                 // block of kRedRows rows
};

enum SweepMode : int {
    kModePG = 0,            // g = A^T r, x <- Pi(x + eta g), partial += A x
    kModeCorr = 1,          // g = A^T r stored
    kModeAx = 2,            // partial += A x
    kModeFold = 3,          // partial += A_S b_S, partial2 += A_S (b_S - x_S)
    kModePow = 4,           // g = A^T r, partial += A g (one product with A A^T)
    kModePGS = 5,           // kModeCorr at x and the kModePG step from x in one pass;
                            // x is kept in xs, g stored
    // Two-pass forms for the shapes whose fused form does not fit the register
    // file (TPC * rows >= 16384: the residual is staged in LDS instead): a dot
    // pass, then a product pass over the same columns.
    kModeStep = 6,          // kModePG without the product: x <- Pi(x + eta g)
    kModeStepS = 7,         // kModePGS without the product
    kModePowG = 8,          // g = A^T r stored
    kModeAg = 9,            // partial += A g
    kModePG1 = 10,          // kModePG for the first iteration of a pass: returns at once
                            // when the previous screening pass took this step (a kernel
                            // of its own, so profiles separate it from the full sweeps)
    // Chambolle-Pock iteration (the dual iterate v lives in r2): x+ = Pi(x - tau A^T v),
    // partial += A (2 x+ - x); the two-pass form keeps 2 x+ - x in xs for the product pass
    kModeCP = 11,
    kModeStepCP = 12,       // kModeCP without the product
    kModeAxS = 13           // partial += A xs
};

// Shapes that run the PG step, the screening sweep and the products with
// A A^T as two passes (dot pass + product pass).
constexpr bool two_pass_shape(int tpc, int rows) { return tpc * rows >= 16384; }

enum ReduceMode : int {
    kRedResidual = 0,       // r = yp - sum
    kRedFold = 1,           // yp -= sum, r -= sum2
    kRedPow = 2,            // r = sum (= A A^T r)
    kRedAhead = 3,          // r2 = yp - sum
    kRedCP = 4              // Chambolle-Pock dual step: r2 = (r2 + s (sum - yp)) / (1 + s), s = step
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
// therefore at most gamma(kDotDepth) * sum_i |a_ij r_i|.  Every sweep shape
// (fused and two-pass forms alike) is checked against it below.
constexpr double kDotDepth = 64.0;
constexpr int dot_depth(int tpc, int rows) { return rows + 6 + tpc / 64; }

// Column-sweep kernel variants: TPC threads share one column, NG column
// groups per workgroup, R rows per thread (capacity TPC * R rows), CBI
// columns per round, PD rounds of prefetch.  X(id, TPC, NG, R, CBI, PD).
// Variants 0..8 are the row classes (smallest capacity first); all others
// are alternatives the tuner may select for a class they can hold.
#define BXS_SWEEP_VARIANTS(X)   \
    X(0, 64, 4, 1, 8, 1)        \
    X(1, 64, 4, 2, 8, 1)        \
    X(2, 64, 4, 4, 8, 1)        \
    X(3, 128, 2, 4, 8, 1)       \
    X(4, 256, 1, 4, 8, 1)       \
    X(5, 512, 1, 4, 8, 1)       \
    X(6, 1024, 1, 4, 8, 1)      \
    X(7, 1024, 1, 8, 4, 1)      \
    X(8, 1024, 1, 16, 2, 1)     \
    X(9, 1024, 1, 4, 4, 1)      \
    X(10, 512, 1, 8, 4, 1)      \
    X(11, 256, 1, 16, 2, 1)     \
    X(12, 512, 1, 4, 4, 1)      \
    X(13, 256, 1, 8, 4, 1)      \
    X(14, 256, 1, 4, 4, 1)      \
    X(15, 64, 4, 8, 4, 1)       \
    X(16, 128, 2, 8, 4, 1)      \
    X(17, 256, 1, 16, 1, 1)     \
    X(18, 512, 1, 8, 2, 1)      \
    X(19, 1024, 1, 4, 2, 1)     \
    X(20, 256, 1, 8, 2, 1)      \
    X(21, 512, 1, 4, 2, 1)      \
    X(22, 512, 1, 8, 2, 2)      \
    X(23, 1024, 1, 4, 2, 2)     \
    X(24, 256, 1, 16, 1, 2)     \
    X(25, 512, 1, 8, 1, 2)      \
    X(26, 256, 1, 8, 2, 2)      \
    X(27, 512, 1, 4, 2, 2)      \
    X(28, 1024, 1, 8, 1, 2)     \
    X(29, 1024, 1, 16, 1, 2)     \
    X(30, 512, 1, 16, 1, 1)      \
    X(31, 512, 1, 16, 2, 1)      \
    X(32, 512, 1, 16, 1, 2)

struct VariantSpec { int tpc, ng, rows, cbi, pd; };
constexpr int kNumVariants = 33;
constexpr int kNumDefaultVariants = 9;
constexpr VariantSpec kVariants[kNumVariants] = {
#define BXS_VS(ID, TPC, NG, R, CBI, PD) {TPC, NG, R, CBI, PD},
    BXS_SWEEP_VARIANTS(BXS_VS)
#undef BXS_VS
};

// The rounding margin of the screening test assumes every correlation sum is
// at most kDotDepth deep: a new sweep shape must stay within it.
constexpr bool variants_within_dot_depth()
{
    for (int v = 0; v < kNumVariants; ++v)
        if (dot_depth(kVariants[v].tpc, kVariants[v].rows) > (int)kDotDepth) return false;
    return true;
}
static_assert(variants_within_dot_depth(), "a sweep variant's dot products are deeper than kDotDepth");

// Translation units the 16-byte-load sweep variants are split over.
constexpr int kSweepParts = 3;

inline long variant_capacity(int v) { return (long)kVariants[v].tpc * kVariants[v].rows; }
inline bool variant_two_pass(int v) { return two_pass_shape(kVariants[v].tpc, kVariants[v].rows); }

inline int default_variant_for_rows(long m) {
    for (int b = 0; b < kNumDefaultVariants; ++b)
        if (m <= variant_capacity(b)) return b;
    return -1;
}

// Resident threads per CU the sweep is sized for (VGPR-limited occupancy).
constexpr int kThreadsPerCU = 1024;

// Coordinate-descent kernel buckets (one workgroup of TPC threads per
// instance, R rows per thread).
struct CdSpec { int tpc, rows; };
constexpr int kNumCdBuckets = 9;
constexpr CdSpec kCdBuckets[kNumCdBuckets] = {
    {64, 1}, {64, 2}, {64, 4}, {64, 8}, {256, 4}, {256, 8}, {256, 16}, {512, 16}, {1024, 16},
};
inline int cd_bucket_for_rows(long m) {
    for (int b = 0; b < kNumCdBuckets; ++b)
        if (m <= (long)kCdBuckets[b].tpc * kCdBuckets[b].rows) return b;
    return -1;
}

// Host-side launch helpers (defined in kernels.hip).
struct LaunchCtx {
    hipStream_t stream;
    int dtype;              // bxs_dtype
    int vec;                // 1: 16-byte loads of A are valid for every instance
    int single;             // 1: one instance (work item k is {0, k}, row block k is {0, k})
    const Inst* insts;
    State* st;
    int* done_counter;
};

hipError_t launch_init(const LaunchCtx& c, int count, const double* x0_is_given);
hipError_t launch_colstats(const LaunchCtx& c, int variant, const Item* items, int n_items);
// first = 1 marks the first primal iteration of a pass: its sweep and
// reduction return at once for instances whose step was already taken by
// the kModePGS sweep of the previous pass.
hipError_t launch_sweep(const LaunchCtx& c, int variant, int mode, const Item* items, int n_items,
                        int first = 0);
// ritems: row blocks of kRedRows rows (instances with many work items);
// nritems: row blocks of kRedRowsN rows (instances with at most kRedNarrowMax)
hipError_t launch_reduce(const LaunchCtx& c, int mode, const RItem* ritems, int n_ritems, int first = 0,
                         const RItem* nritems = nullptr, int n_nritems = 0);
hipError_t launch_validate(const LaunchCtx& c, int count);
hipError_t launch_publish(const LaunchCtx& c, int* host_dst);
hipError_t launch_pow_init(const LaunchCtx& c, int count);
hipError_t launch_set_step(const LaunchCtx& c, int count, double step);
// cp = 1: the step is the Chambolle-Pock tau = sigma = 1 / (1.05 sqrt(L_est))
hipError_t launch_lanczos(const LaunchCtx& c, int count, int k, int last, int cp = 0);
// Chambolle-Pock start: v = sigma (A x0 - y') / (1 + sigma) = -sigma r / (1 + sigma) into r2
hipError_t launch_cp_init(const LaunchCtx& c, int count);
hipError_t launch_count_free(const LaunchCtx& c, int count);
// host_done: pinned host word that receives the stop counter at the end of
// the pass (nullptr: the caller copies it itself); host_gap: pinned host
// double that receives the gap of instance 0 (single-instance calls), or
// nullptr; host_seq: pinned (coherent) host word that receives the number of
// screening passes run, written last with a system-scope release, or nullptr;
// kind: kScreenLS; kScreenOracleDual (the instances carry a given dual
// optimum, Inst::ts); kScreenHuber (the Huber fidelity, Inst::hub);
// host_nact: pinned host word that receives the preserved-list length of
// instance 0 after the pass (single-instance calls), or nullptr.
enum ScreenKind : int { kScreenLS = 0, kScreenOracleDual = 1, kScreenHuber = 2 };
hipError_t launch_screen(const LaunchCtx& c, int count, double eps_gap, int screening,
                         int final_pass, int K, int kk, int ahead, int* host_done, double* host_gap,
                         int* host_seq, int kind, int* host_nact = nullptr);
hipError_t launch_cd(const LaunchCtx& c, int bucket, const int* inst_list, int n_list, int sweeps);
// translation direction computed from A (tdir.hip, one instance)
size_t tdir_scratch_doubles(long m, long n);
hipError_t launch_tdir(const LaunchCtx& c, int choice, long m, long n, double* scratch, double* t, int* picked);

// Block-sequential CD of one instance (cdblock.hip): blocks of kCdbB
// preserved positions, kCdbRows rows per workgroup of the block products.
constexpr int kCdbB = 128;
constexpr int kCdbRows = 64;
size_t cdb_gram_doubles(long n);        // Gram and cross-Gram blocks of up to n preserved columns
size_t cdb_pg_doubles(long m);          // chunk partials of two blocks' correlations
hipError_t launch_cdb_gram(const LaunchCtx& c, long n, double* gram);
// one sweep over at most nb blocks (an upper bound of the device's count)
hipError_t launch_cdb_sweep(const LaunchCtx& c, long m, long n, long n_bound, double* pg, const double* gram,
                            double* delta);
hipError_t launch_fill(double* p, long n, double v, hipStream_t s);

}  // namespace bxs
