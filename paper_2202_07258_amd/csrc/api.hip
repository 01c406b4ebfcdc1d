// Host driver and C ABI of the boxscreen library.
//
// The driver validates arguments, lays out one workspace for all instances of
// a call, and runs the screening loop of Alg. 1:
//   setup : x0 clipped, y' = y, column norms, w = A^T t, step from power
//           iteration on A A^T (unless given), r = y' - A x0;
//   pass  : K primal iterations (PG: fused g = A_P^T r / update / A_P x sweep
//           + partial reduction; CD: one sequential sweep per instance), a
//           correlation sweep g = A_P^T r, the screening kernel (dual point,
//           gap, radius, safe rule, compaction) and the fold of the newly
//           screened columns into y' and r;
//   stop  : after each pass the host reads one counter of stopped instances.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <chrono>
#include <mutex>
#include <vector>

#include "bxs_internal.h"

namespace bxs {

static thread_local std::string g_last_error;

static bxs_status fail(bxs_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

bxs_status set_error(bxs_status s, const char* msg) { return fail(s, "%s", msg); }

size_t batched_workspace_bytes(long m, long n, long B, int iter_precision);
size_t adjoint_workspace_bytes(long m, long n, long B);
bxs_status adjoint_run(long m, long n, long B, int a_dtype, const void* A, long lda, const double* Y, long ldy,
                       const double* X, long ldx, const double* l, const double* u, const double* dX, long ldg,
                       double* dY, long lddy, double* dA, long ldda, double* dl, long lddl, double* du, long lddu,
                       const bxs_opts* o, long* cg_iters);
bxs_status batched_nnls_run(long m, long n, long B, int a_dtype, const void* A, long lda, const double* Y, long ldy,
                            double* X, long ldx, signed char* sat, long ldsat, const bxs_opts* o, bxs_info* infos);

#define BXS_HIP(call)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(BXS_ERR_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_));   \
    } while (0)

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Dispatch overhead seen by a pair of HIP events around one launch: the
// average elapsed time around an empty kernel on the caller's stream, taken
// once per process and device (profile mode only).
__global__ void k_noop() {}

static double g_event_overhead_ms[64];
static bool g_event_overhead_done[64];

bxs_status event_overhead(hipStream_t s, double* out)
{
    int dev = 0;
    BXS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) { *out = 0.0; return BXS_OK; }
    if (!g_event_overhead_done[dev]) {
        constexpr int kReps = 32;
        hipEvent_t e[2 * kReps];
        for (auto& x : e) BXS_HIP(hipEventCreate(&x));
        struct G { hipEvent_t* e; ~G() { for (int i = 0; i < 2 * kReps; ++i) (void)hipEventDestroy(e[i]); } } g{e};
        k_noop<<<1, 64, 0, s>>>();                       // warm-up
        for (int i = 0; i < kReps; ++i) {
            BXS_HIP(hipEventRecord(e[2 * i], s));
            k_noop<<<1, 64, 0, s>>>();
            BXS_HIP(hipEventRecord(e[2 * i + 1], s));
        }
        BXS_HIP(hipGetLastError());
        BXS_HIP(hipEventSynchronize(e[2 * kReps - 1]));
        double tot = 0.0;
        for (int i = 0; i < kReps; ++i) {
            float ms = 0.f;
            BXS_HIP(hipEventElapsedTime(&ms, e[2 * i], e[2 * i + 1]));
            tot += ms;
        }
        g_event_overhead_ms[dev] = tot / kReps;
        g_event_overhead_done[dev] = true;
    }
    *out = g_event_overhead_ms[dev];
    return BXS_OK;
}

struct InstSpec {
    long m, n, lda;
    const void* A;
    const double *y, *l, *u;
    double* x;
    signed char* sat;
};

struct PlanSizes {
    int items_cap;
    int g_target;
    size_t bytes;
};

// Per-instance device bytes.
static PlanSizes instance_sizes(long m, long n, int g_target, long rec_cap, int lz_steps, int tdir, int cdb)
{
    PlanSizes p;
    p.g_target = g_target;
    long cap = std::max<long>((long)g_target + 1, (n + kCbMax - 1) / kCbMax);
    cap = std::min<long>(cap, (n + kCbMin - 1) / kCbMin);
    p.items_cap = (int)std::max<long>(cap, 1);
    size_t b = 0;
    b += align_up(sizeof(double) * 3 * m, 256);                   // yp, r, r2
    b += align_up(sizeof(double) * 8 * n, 256);                   // g, w, cn, cn2, fval, fdx, xs, gs
    b += align_up(sizeof(int) * 2 * n, 256);                      // idx, fidx
    b += align_up(sizeof(double) * 2 * (size_t)p.items_cap * m, 256);  // part, part2
    b += align_up(sizeof(double) * kItemScalars * p.items_cap, 256);  // iscal
    b += align_up(sizeof(bxs_pass_record) * std::max<long>(rec_cap, 0), 256);
    if (lz_steps > 0) b += align_up(sizeof(double) * (2 * (size_t)lz_steps + 2 * m), 256);  // Lanczos
    if (tdir) b += align_up(sizeof(double) * ((size_t)m + tdir_scratch_doubles(m, n)), 256);  // t and its scratch
    if (cdb) b += align_up(sizeof(double) * (cdb_gram_doubles(n) + cdb_pg_doubles(m) + 2 * kCdbB), 256);  // block CD
    p.bytes = b;
    return p;
}

static int device_cus()
{
    static thread_local int cached = 0;
    if (cached) return cached;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
            cus = prop.multiProcessorCount;
    }
    cached = cus;
    return cus;
}

// Sweep-variant preference per row-count class (the smallest default
// variant whose capacity holds m); set by bxs_set_sweep_variant.  Defaults:
// for m up to 512 the narrow shapes that pack several columns per workgroup
// (best for batches of small instances); above, the autotuner's choices on
// one MI355X for a single instance with the class's largest row count and
// four times as many columns (up to 256 MB).
static int g_variant_pref[kNumDefaultVariants] = {0, 1, 2, 3, 12, 12, 18, 31, 29};

// bfloat16 storage moves half the bytes per column, so the classes that are
// latency-limited at 8 rows per thread keep twice the columns in flight
// (measured on MI355X at 4000 x 16000: 38.9 us per sweep with 4 columns per
// round against 46.3 us with 2).  Not changed by bxs_set_sweep_variant.
static const int g_variant_pref_bf16[kNumDefaultVariants] = {0, 1, 2, 3, 12, 10, 10, 31, 29};

static int choose_variant(long m, int dtype = BXS_F32)
{
    const int cls = default_variant_for_rows(m);
    if (cls < 0) return -1;
    const int v = (dtype == BXS_BF16) ? g_variant_pref_bf16[cls] : g_variant_pref[cls];
    return (v >= 0 && v < kNumVariants && variant_capacity(v) >= m) ? v : cls;
}

// Work-group targets: spread the columns of each instance over a share of
// the chip's resident workgroups (CUs x kThreadsPerCU / workgroup size)
// proportional to its size m*n, at least one.
// Fraction of the chip's resident workgroups an instance's work items are
// spread over, per row class (fewer, longer items write fewer partial
// products; set by bxs_set_group_scale).  Defaults from the autotuner on one
// MI355X, as for the shapes; for 4000 x 16000 the spread 0.5 gives one
// workgroup of 64 columns per CU (43 us per sweep against 49 us at 1), and
// for 1000 x 3000 (FP64) 13.0 us per iteration against 14.3 us at 1; for
// 8000 x 8000 with the 512 x 16 shape 54 us against 62 us for 1024 x 8 at 1.
static double g_group_scale[kNumDefaultVariants] = {1, 1, 1, 1, 0.5, 0.5, 0.5, 0.5, 1};

static std::vector<int> group_targets(const std::vector<InstSpec>& specs, const std::vector<int>& variant, int cus)
{
    double total = 0.0;
    for (auto& s : specs) total += (double)s.m * (double)s.n;
    std::vector<int> g(specs.size());
    for (size_t i = 0; i < specs.size(); ++i) {
        const double share = total > 0 ? (double)specs[i].m * (double)specs[i].n / total : 1.0;
        const int wg = kVariants[variant[i]].tpc * kVariants[variant[i]].ng;
        const int cls = default_variant_for_rows(specs[i].m);
        const double scale = (cls >= 0) ? g_group_scale[cls] : 1.0;
        const double resident = (double)cus * std::max(1, kThreadsPerCU / wg) * scale;
        g[i] = std::max(1, (int)ceil(resident * share));
    }
    return g;
}

static size_t common_bytes(long count, long total_items, long total_ritems)
{
    size_t b = 0;
    b += align_up(sizeof(Inst) * count, 256);
    b += align_up(sizeof(State) * count, 256);
    b += align_up(sizeof(Item) * total_items, 256);
    b += align_up(sizeof(RItem) * total_ritems, 256);
    b += align_up(sizeof(int) * (count + 16), 256);               // instance lists + counter
    return b;
}

static bxs_status check_opts(const bxs_opts* o)
{
    if (!o) return fail(BXS_ERR_ARG, "opts is NULL");
    if (o->solver != BXS_PG && o->solver != BXS_CD && o->solver != BXS_CP)
        return fail(BXS_ERR_ARG, "unknown solver %d", o->solver);
    if (o->screening != 0 && o->screening != 1) return fail(BXS_ERR_ARG, "screening must be 0 or 1");
    if (o->screen_every < 1) return fail(BXS_ERR_ARG, "screen_every must be >= 1");
    if (o->max_iter < 1) return fail(BXS_ERR_ARG, "max_iter must be >= 1");
    if (!(o->eps_gap >= 0.0) || isinf(o->eps_gap)) return fail(BXS_ERR_ARG, "eps_gap must be finite and >= 0");
    if (isnan(o->step) || isinf(o->step)) return fail(BXS_ERR_ARG, "step must be finite");
    if (o->workspace && o->workspace_bytes == 0) return fail(BXS_ERR_ARG, "workspace given with 0 bytes");
    if (o->history && o->history_cap < 0) return fail(BXS_ERR_ARG, "history_cap < 0");
    if (o->iter_precision != BXS_ITER_F64 && o->iter_precision != BXS_ITER_BF16X3)
        return fail(BXS_ERR_ARG, "unknown iter_precision %d", o->iter_precision);
    if (o->power_iters > kLanczosMax) return fail(BXS_ERR_ARG, "power_iters must be <= %d", kLanczosMax);
    if (o->t_choice < BXS_T_GIVEN || o->t_choice > BXS_T_NORMAL_EQUATIONS)
        return fail(BXS_ERR_ARG, "unknown t_choice %d", o->t_choice);
    if (o->t_choice != BXS_T_GIVEN && o->t) return fail(BXS_ERR_ARG, "t_choice computes t: opts->t must be NULL");
    if (o->fidelity != BXS_FID_LS && o->fidelity != BXS_FID_HUBER)
        return fail(BXS_ERR_ARG, "unknown fidelity %d", o->fidelity);
    if (o->fidelity == BXS_FID_HUBER) {
        if (!(o->huber_delta > 0.0) || isinf(o->huber_delta))
            return fail(BXS_ERR_ARG, "huber_delta must be finite and > 0");
        if (o->solver == BXS_CD) return fail(BXS_ERR_ARG, "the Huber fidelity runs with the PG and CP solvers");
        if (o->theta_star) return fail(BXS_ERR_ARG, "the Huber fidelity takes no theta_star");
    }
    if (o->deterministic != 0 && o->deterministic != 1) return fail(BXS_ERR_ARG, "deterministic must be 0 or 1");
    return BXS_OK;
}

// Lanczos steps of the ||A||_2^2 estimate of the sweep solvers (0 when the
// caller gives the step).
static int lanczos_steps(const bxs_opts* o)
{
    if (o->step > 0.0) return 0;
    return o->power_iters > 0 ? o->power_iters : kLanczosDefault;
}

static bxs_status check_spec(const InstSpec& s, long i)
{
    if (s.m < 1 || s.n < 1) return fail(BXS_ERR_SHAPE, "problem %ld: m=%ld n=%ld must be >= 1", i, s.m, s.n);
    if (s.lda < s.m) return fail(BXS_ERR_SHAPE, "problem %ld: lda=%ld < m=%ld", i, s.lda, s.m);
    if (s.m > BXS_MAX_ROWS) return fail(BXS_ERR_SHAPE, "problem %ld: m=%ld exceeds %d rows", i, s.m, BXS_MAX_ROWS);
    if (s.n > 0x7fffffffL / 2) return fail(BXS_ERR_SHAPE, "problem %ld: n=%ld too large", i, s.n);
    if (!s.A || !s.y || !s.x || !s.sat) return fail(BXS_ERR_ARG, "problem %ld: NULL array argument", i);
    return BXS_OK;
}

struct Plan {
    std::vector<InstSpec> specs;
    std::vector<PlanSizes> sizes;
    std::vector<Inst> insts;                 // host copy of the device descriptors
    std::vector<Item> items[kNumVariants];
    std::vector<RItem> ritems;      // wide reduction (kRedRows rows per block)
    std::vector<RItem> nritems;     // narrow reduction (kRedRowsN rows per block)
    std::vector<int> cd_list[kNumCdBuckets];
    std::vector<int> variant;                // sweep variant per instance
    long rec_cap = 0;
    int lz_steps = 0;
    int tdir = 0;                            // bxs_translation computed by the library (one instance)
    double* tbuf = nullptr;                  // its t (device) and scratch
    double* tscratch = nullptr;
    int cdb = 0;                             // block-sequential CD (one instance)
    double* cdb_gram = nullptr;              // its Gram blocks, chunk partials and block update
    double* cdb_pg = nullptr;
    double* cdb_delta = nullptr;
    int vec = 1;
    size_t bytes = 0;
};

// Block-sequential CD for single-instance CD solves (on unless switched off
// by bxs_set_cd_block; batches keep one workgroup per instance).
static int g_cd_block = 1;
static int cd_block_on(const bxs_opts* o, long count)
{
    return (g_cd_block && count == 1 && o->solver == BXS_CD) ? 1 : 0;
}

static bxs_status build_plan(Plan& P, int dtype, long rec_cap, int lz_steps, int tdir = 0, int cdb = 0)
{
    const long count = (long)P.specs.size();
    const int cus = device_cus();
    P.variant.resize(count);
    for (long i = 0; i < count; ++i) P.variant[i] = choose_variant(P.specs[i].m, dtype);
    std::vector<int> g = group_targets(P.specs, P.variant, cus);
    P.rec_cap = rec_cap;
    P.lz_steps = lz_steps;
    P.tdir = (count == 1) ? tdir : 0;
    P.cdb = (count == 1) ? cdb : 0;
    P.sizes.resize(count);
    long total_items = 0;
    size_t inst_bytes = 0;
    const size_t esz = dtype == BXS_BF16 ? 2 : (dtype == BXS_F32 ? 4 : 8);
    const int vecw = (int)(16 / esz);                   // elements per 16-byte load
    P.vec = 1;
    for (long i = 0; i < count; ++i) {
        const InstSpec& s = P.specs[i];
        P.sizes[i] = instance_sizes(s.m, s.n, g[i], (i == 0 && count == 1) ? rec_cap : 0, lz_steps, P.tdir, P.cdb);
        total_items += P.sizes[i].items_cap;
        inst_bytes += P.sizes[i].bytes;
        if ((s.lda % vecw) != 0 || ((uintptr_t)s.A % 16) != 0) P.vec = 0;
        (void)esz;
    }
    long total_ritems = 0;
    for (auto& s : P.specs) total_ritems += (s.m + kRedRows - 1) / kRedRows;
    P.bytes = common_bytes(count, total_items, total_ritems) + inst_bytes + 256;
    return BXS_OK;
}

// Lay out the workspace and fill the host-side descriptor / item tables.
static void layout(Plan& P, char* base)
{
    const long count = (long)P.specs.size();
    long total_items = 0, total_ritems = 0;
    for (long i = 0; i < count; ++i) {
        total_items += P.sizes[i].items_cap;
        total_ritems += (P.specs[i].m + kRedRows - 1) / kRedRows;
    }
    char* cur = (char*)align_up((uintptr_t)base, 256);
    auto take = [&](size_t bytes) { char* p = cur; cur += align_up(bytes, 256); return p; };
    take(sizeof(Inst) * count);
    take(sizeof(State) * count);
    take(sizeof(Item) * total_items);
    take(sizeof(RItem) * total_ritems);
    take(sizeof(int) * (count + 16));
    P.insts.resize(count);
    for (int b = 0; b < kNumVariants; ++b) P.items[b].clear();
    for (int b = 0; b < kNumCdBuckets; ++b) P.cd_list[b].clear();
    P.ritems.clear();
    P.nritems.clear();
    for (long i = 0; i < count; ++i) {
        const InstSpec& s = P.specs[i];
        const PlanSizes& z = P.sizes[i];
        Inst I;
        memset(&I, 0, sizeof(I));
        I.A = s.A; I.lda = s.lda; I.m = (int)s.m; I.n = (int)s.n;
        I.y = s.y; I.l = s.l; I.u = s.u; I.t = nullptr; I.x = s.x; I.sat = s.sat;
        I.yp = (double*)take(sizeof(double) * 3 * s.m);
        I.r = I.yp + s.m;
        I.r2 = I.yp + 2 * s.m;
        double* nv = (double*)take(sizeof(double) * 8 * s.n);
        I.g = nv; I.w = nv + s.n; I.cn = nv + 2 * s.n; I.cn2 = nv + 3 * s.n;
        I.fval = nv + 4 * s.n; I.fdx = nv + 5 * s.n; I.xs = nv + 6 * s.n; I.gs = nv + 7 * s.n;
        int* iv = (int*)take(sizeof(int) * 2 * s.n);
        I.idx = iv; I.fidx = iv + s.n;
        I.part = (double*)take(sizeof(double) * 2 * (size_t)z.items_cap * s.m);
        I.part2 = I.part + (size_t)z.items_cap * s.m;
        I.iscal = (double*)take(sizeof(double) * kItemScalars * z.items_cap);
        const long rc = (i == 0 && count == 1) ? P.rec_cap : 0;
        I.rec = rc > 0 ? (bxs_pass_record*)take(sizeof(bxs_pass_record) * rc) : nullptr;
        I.rec_cap = (int)rc;
        I.items_cap = z.items_cap;
        I.g_target = z.g_target;
        I.lz_steps = P.lz_steps;
        I.lz = P.lz_steps > 0 ? (double*)take(sizeof(double) * (2 * (size_t)P.lz_steps + 2 * s.m)) : nullptr;
        if (P.tdir) {
            P.tbuf = (double*)take(sizeof(double) * ((size_t)s.m + tdir_scratch_doubles(s.m, s.n)));
            P.tscratch = P.tbuf + s.m;
        }
        if (P.cdb) {
            P.cdb_gram = (double*)take(sizeof(double) * (cdb_gram_doubles(s.n) + cdb_pg_doubles(s.m) + 2 * kCdbB));
            P.cdb_pg = P.cdb_gram + cdb_gram_doubles(s.n);
            P.cdb_delta = P.cdb_pg + cdb_pg_doubles(s.m);
        }
        const int b = P.variant[i];
        I.item_base = (int)P.items[b].size();
        for (int t = 0; t < z.items_cap; ++t) P.items[b].push_back(Item{(int)i, t});
        P.cd_list[cd_bucket_for_rows(s.m)].push_back((int)i);
        // an instance never has more work items in use than items_cap
        if (z.items_cap <= kRedNarrowMax)
            for (int rb = 0; rb < (int)((s.m + kRedRowsN - 1) / kRedRowsN); ++rb) P.nritems.push_back(RItem{(int)i, rb});
        else
            for (int rb = 0; rb < (int)((s.m + kRedRows - 1) / kRedRows); ++rb) P.ritems.push_back(RItem{(int)i, rb});
        P.insts[i] = I;
    }
}

struct DevTables {
    Inst* insts;
    State* st;
    Item* items[kNumVariants];
    int n_items[kNumVariants];
    RItem* ritems;
    int n_ritems;
    RItem* nritems;     // after the wide ones in the same table
    int n_nritems;
    int* lists[kNumCdBuckets];
    int n_list[kNumCdBuckets];
    int* done_counter;
};

struct PinnedBuf {
    void* p = nullptr;
    size_t bytes = 0;
    ~PinnedBuf() { if (p) (void)hipHostFree(p); }
};

// Pinned host staging area for the device tables of a solve (one copy
// uploads them all) and for the State download at its end.  A solve
// synchronises its stream before it returns, so the next call of the same
// thread finds the area free.
static bxs_status staging(size_t bytes, void** out)
{
    static thread_local PinnedBuf buf;
    if (buf.bytes < bytes) {
        if (buf.p) (void)hipHostFree(buf.p);
        buf.p = nullptr;
        buf.bytes = 0;
        BXS_HIP(hipHostMalloc(&buf.p, bytes, hipHostMallocDefault));
        buf.bytes = bytes;
    }
    *out = buf.p;
    return BXS_OK;
}

// Coherent (fine-grained) pinned words the screening kernel writes for the
// host: the stop counter, the gap and the pass sequence number.
static bxs_status pinned(size_t bytes, void** out)
{
    static thread_local PinnedBuf buf;
    if (buf.bytes < bytes) {
        if (buf.p) (void)hipHostFree(buf.p);
        buf.p = nullptr;
        buf.bytes = 0;
        BXS_HIP(hipHostMalloc(&buf.p, bytes, hipHostMallocCoherent));
        buf.bytes = bytes;
    }
    *out = buf.p;
    return BXS_OK;
}

// A library-owned stream per device (non-blocking, default priority) for
// callers that pass the null stream: a graph cannot be captured on it.
static hipStream_t g_side_stream[64];

static bxs_status side_stream(hipStream_t* out)
{
    int dev = 0;
    BXS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(BXS_ERR_DEVICE, "device index %d out of range", dev);
    if (!g_side_stream[dev]) BXS_HIP(hipStreamCreateWithFlags(&g_side_stream[dev], hipStreamNonBlocking));
    *out = g_side_stream[dev];
    return BXS_OK;
}

// Allocation-free mode (solve_bvls_noalloc): the workspace is the library's
// fixed device scratch array, the device tables go up from a fixed host area,
// and the host learns the stop counter by a copy and a stream
// synchronisation after every pass: no device or pinned-host allocation, no
// event, no graph.
struct FixedArea {
    void* dev;              // device scratch (address from hipGetSymbolAddress)
    size_t dev_bytes;
    char* host;             // pageable host staging area
    size_t host_bytes;
};

static bxs_status run(Plan& P, int dtype, const bxs_opts* o, const double* t, bxs_info* infos,
                      bxs_pass_record* history, long history_cap, const FixedArea* fixed = nullptr)
{
    const long count = (long)P.specs.size();
    hipStream_t stream = (hipStream_t)o->stream;
    const bool noalloc = fixed != nullptr;
    const auto host_t0 = std::chrono::steady_clock::now();
    const bool want_graph = !noalloc && o->graph && !o->profile && o->max_iter >= 3LL * o->screen_every;
    // With the null stream and graph replay, the solve runs on the side
    // stream, ordered after the caller's earlier work; every path below ends
    // with that stream synchronised, so the caller needs no further wait.
    struct SideGuard {
        hipStream_t s = nullptr;
        ~SideGuard() { if (s) (void)hipStreamSynchronize(s); }
    } side_guard;
    if (want_graph && stream == nullptr) {
        hipStream_t side = nullptr;
        const bxs_status ss = side_stream(&side);
        if (ss != BXS_OK) return ss;
        hipEvent_t ev;
        BXS_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        const hipError_t e1 = hipEventRecord(ev, stream);
        const hipError_t e2 = (e1 == hipSuccess) ? hipStreamWaitEvent(side, ev, 0) : e1;
        (void)hipEventDestroy(ev);
        BXS_HIP(e2);
        stream = side;
        side_guard.s = side;
    }
    void* ws = o->workspace;
    bool owned = false;
    if (noalloc) {
        if (P.bytes > fixed->dev_bytes)
            return fail(BXS_ERR_NOMEM, "problem needs %zu bytes of workspace; the fixed scratch array holds %zu",
                        P.bytes, fixed->dev_bytes);
        ws = fixed->dev;
    } else if (ws) {
        if (o->workspace_bytes < P.bytes)
            return fail(BXS_ERR_NOMEM, "workspace of %zu bytes, %zu needed", o->workspace_bytes, P.bytes);
    } else {
        if (hipMalloc(&ws, P.bytes) != hipSuccess) return fail(BXS_ERR_NOMEM, "hipMalloc(%zu) failed", P.bytes);
        owned = true;
    }
    struct Guard {
        void* p; bool own; hipStream_t s;
        ~Guard() { if (own && p) { (void)hipStreamSynchronize(s); (void)hipFree(p); } }
    } guard{ws, owned, stream};

    layout(P, (char*)ws);
    for (long i = 0; i < count; ++i) {
        P.insts[i].t = P.tdir ? P.tbuf : t;
        P.insts[i].ts = o->theta_star;
        P.insts[i].hub = (o->fidelity == BXS_FID_HUBER) ? o->huber_delta : HUGE_VAL;
    }

    // device tables
    DevTables D;
    char* cur = (char*)align_up((uintptr_t)ws, 256);
    long total_items = 0;
    for (long i = 0; i < count; ++i) total_items += P.sizes[i].items_cap;
    D.insts = (Inst*)cur; cur += align_up(sizeof(Inst) * count, 256);
    D.st = (State*)cur; cur += align_up(sizeof(State) * count, 256);
    Item* items_base = (Item*)cur; cur += align_up(sizeof(Item) * total_items, 256);
    D.ritems = (RItem*)cur; cur += align_up(sizeof(RItem) * (P.ritems.size() + P.nritems.size()), 256);
    int* ints = (int*)cur;
    D.done_counter = ints + count;
    D.n_ritems = (int)P.ritems.size();
    D.nritems = D.ritems + P.ritems.size();
    D.n_nritems = (int)P.nritems.size();
    // Host image of the tables (descriptors, zeroed states, work items,
    // reduction items, CD lists, zeroed stop counter and ticket), uploaded
    // with one copy from pinned memory.
    const size_t tbytes = (size_t)((char*)(D.done_counter + 3) - (char*)D.insts);   // + ticket, pass count
    const size_t sbytes = sizeof(State) * count;
    void* stage_p = nullptr;
    if (noalloc) {
        if (std::max(tbytes, sbytes) > fixed->host_bytes - 64)   // the last 64 bytes hold the host words
            return fail(BXS_ERR_NOMEM, "device tables of %zu bytes exceed the fixed host staging area of %zu",
                        std::max(tbytes, sbytes), fixed->host_bytes);
        stage_p = fixed->host;
    } else {
        bxs_status ss = staging(std::max(tbytes, sbytes), &stage_p);
        if (ss != BXS_OK) return ss;
    }
    char* img = (char*)stage_p;
    memset(img, 0, tbytes);
    auto at = [&](const void* dev) { return img + ((const char*)dev - (const char*)D.insts); };
    memcpy(at(D.insts), P.insts.data(), sizeof(Inst) * count);
    long off = 0, loff = 0;
    for (int b = 0; b < kNumVariants; ++b) {
        D.items[b] = items_base + off;
        D.n_items[b] = (int)P.items[b].size();
        if (D.n_items[b] > 0) memcpy(at(D.items[b]), P.items[b].data(), sizeof(Item) * P.items[b].size());
        off += D.n_items[b];
    }
    if (!P.ritems.empty()) memcpy(at(D.ritems), P.ritems.data(), sizeof(RItem) * P.ritems.size());
    if (!P.nritems.empty()) memcpy(at(D.nritems), P.nritems.data(), sizeof(RItem) * P.nritems.size());
    for (int b = 0; b < kNumCdBuckets; ++b) {
        D.lists[b] = ints + loff;
        D.n_list[b] = (int)P.cd_list[b].size();
        if (D.n_list[b] > 0) memcpy(at(D.lists[b]), P.cd_list[b].data(), sizeof(int) * P.cd_list[b].size());
        loff += D.n_list[b];
    }
    BXS_HIP(hipMemcpyAsync(D.insts, img, tbytes, hipMemcpyHostToDevice, stream));
    struct StageGuard {
        hipStream_t s;
        bool done = false;
        ~StageGuard() { if (!done) (void)hipStreamSynchronize(s); }   // the area is reused by the next call
    } stage_guard{stream};

    LaunchCtx c;
    c.stream = stream; c.dtype = dtype; c.vec = P.vec; c.single = (count == 1) ? 1 : 0;
    c.insts = D.insts; c.st = D.st; c.done_counter = D.done_counter;

    // Sweeps that read A and also accumulate a product with A: one fused pass,
    // or a dot pass and a product pass for the shapes too large for the fused
    // kernel's registers.
    auto sweep_pg = [&](int b, int first) -> hipError_t {
        if (!variant_two_pass(b)) return launch_sweep(c, b, first ? kModePG1 : kModePG, D.items[b], D.n_items[b]);
        const hipError_t e = launch_sweep(c, b, kModeStep, D.items[b], D.n_items[b], first);
        return e != hipSuccess ? e : launch_sweep(c, b, kModeAx, D.items[b], D.n_items[b], first);
    };
    auto sweep_pgs = [&](int b) -> hipError_t {
        if (!variant_two_pass(b)) return launch_sweep(c, b, kModePGS, D.items[b], D.n_items[b]);
        const hipError_t e = launch_sweep(c, b, kModeStepS, D.items[b], D.n_items[b]);
        return e != hipSuccess ? e : launch_sweep(c, b, kModeAx, D.items[b], D.n_items[b]);
    };
    auto sweep_cp = [&](int b) -> hipError_t {
        if (!variant_two_pass(b)) return launch_sweep(c, b, kModeCP, D.items[b], D.n_items[b]);
        const hipError_t e = launch_sweep(c, b, kModeStepCP, D.items[b], D.n_items[b]);
        return e != hipSuccess ? e : launch_sweep(c, b, kModeAxS, D.items[b], D.n_items[b]);
    };
    auto sweep_pow = [&](int b) -> hipError_t {
        if (!variant_two_pass(b)) return launch_sweep(c, b, kModePow, D.items[b], D.n_items[b]);
        const hipError_t e = launch_sweep(c, b, kModePowG, D.items[b], D.n_items[b]);
        return e != hipSuccess ? e : launch_sweep(c, b, kModeAg, D.items[b], D.n_items[b]);
    };

    hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr;
    if (!noalloc) {
        BXS_HIP(hipEventCreate(&ev0));
        BXS_HIP(hipEventCreate(&ev1));
        BXS_HIP(hipEventCreate(&ev2));
    }
    struct EvGuard {
        hipEvent_t a, b, c;
        ~EvGuard() {
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
            if (c) (void)hipEventDestroy(c);
        }
    } eg{ev0, ev1, ev2};
    double ev_over = 0.0;
    if (o->profile) {
        bxs_status es = event_overhead(stream, &ev_over);
        if (es != BXS_OK) return es;
    }
    if (!noalloc) BXS_HIP(hipEventRecord(ev0, stream));

    // ---- setup ----
    if (P.tdir) BXS_HIP(launch_fill(P.tbuf, P.specs[0].m, -1.0, stream));   // finite until computed
    BXS_HIP(launch_init(c, (int)count, nullptr));
    for (int b = 0; b < kNumVariants; ++b) BXS_HIP(launch_colstats(c, b, D.items[b], D.n_items[b]));
    if (P.tdir) {
        // t from the column norms, then the column statistics again for w = A^T t
        BXS_HIP(launch_tdir(c, P.tdir, P.specs[0].m, P.specs[0].n, P.tscratch, P.tbuf, &D.st[0].t_column));
        for (int b = 0; b < kNumVariants; ++b) BXS_HIP(launch_colstats(c, b, D.items[b], D.n_items[b]));
    }
    BXS_HIP(launch_validate(c, (int)count));
    const bool do_pow = !(o->step > 0.0);
    if (do_pow) {
        // Lanczos on A A^T from a fixed unit vector: one sweep per step
        BXS_HIP(launch_pow_init(c, (int)count));
        const int np = P.lz_steps;
        for (int k = 0; k < np; ++k) {
            for (int b = 0; b < kNumVariants; ++b) BXS_HIP(sweep_pow(b));
            BXS_HIP(launch_reduce(c, kRedPow, D.ritems, D.n_ritems, 0, D.nritems, D.n_nritems));
            BXS_HIP(launch_lanczos(c, (int)count, k, k == np - 1, o->solver == BXS_CP));
        }
    } else {
        BXS_HIP(launch_set_step(c, (int)count, o->step));
    }
    for (int b = 0; b < kNumVariants; ++b) BXS_HIP(launch_sweep(c, b, kModeAx, D.items[b], D.n_items[b]));
    BXS_HIP(launch_reduce(c, kRedResidual, D.ritems, D.n_ritems, 0, D.nritems, D.n_nritems));
    if (o->solver == BXS_CP) BXS_HIP(launch_cp_init(c, (int)count));
    if (!noalloc) BXS_HIP(hipEventRecord(ev1, stream));

    // instances that failed validation are stopped on the device (k_validate)
    // and reported after the loop
    std::vector<State> hst(count);

    // ---- screening loop ----
    int* hdone = nullptr;
    if (noalloc) {
        // plain host words in the staging area, after the table image
        hdone = (int*)(fixed->host + fixed->host_bytes - 64);
    } else {
        void* pp = nullptr;
        bxs_status s = pinned(64, &pp);
        if (s != BXS_OK) return s;
        hdone = (int*)pp;                                   // stop counter per slot: bytes 0..7
    }
    double* hgap = (double*)((char*)hdone + 16);            // gap per slot: bytes 16..31
    hgap[0] = hgap[1] = -1.0;
    int* hseq = (int*)((char*)hdone + 32);                  // passes published: bytes 32..35
    __atomic_store_n(hseq, 0, __ATOMIC_RELEASE);
    int* hnact = (int*)((char*)hdone + 40);                 // preserved-list length per slot: bytes 40..47
    hnact[0] = hnact[1] = (int)P.specs[0].n;
    // block-sequential CD: an upper bound of the preserved-list length, taken
    // from the last pass the host has seen (the list only shrinks), so that a
    // sweep launches only the blocks that can still exist
    const int K = o->screen_every;
    long long iters = 0;
    // Passes are enqueued one ahead of the stop check: while the host waits
    // for pass p's stop counter, pass p+1 is already queued (its kernels return
    // at once for stopped instances), so the GPU never idles on the host.
    // Optional per-launch timing of the primal-iteration sweeps.
    std::vector<hipEvent_t> pev, dev_done(2);
    struct PevGuard {
        std::vector<hipEvent_t>* v;
        std::vector<hipEvent_t>* w;
        ~PevGuard() {
            for (auto e : *v) if (e) (void)hipEventDestroy(e);
            for (auto e : *w) if (e) (void)hipEventDestroy(e);
        }
    } pguard{&pev, &dev_done};
    for (auto& e : dev_done) {
        e = nullptr;
        if (!noalloc) BXS_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    if (o->profile) {
        pev.assign(4 * (size_t)K, nullptr);
        for (auto& e : pev) BXS_HIP(hipEventCreate(&e));
    }
    double sweep_ms = 0.0;
    long sweep_launches = 0;
    long long slot_kk[2] = {0, 0};
    int slot_final[2] = {0, 0};
    int slot_gap[2] = {0, 0};

    // The kernels of one pass: kk primal iterations, the correlation sweep,
    // the screening kernel and the fold.  `slot` selects the profile events.
    // PG: the correlation sweep also takes the next step from the screening
    // point (kModePGS); when the screening kernel keeps that step, the first
    // iteration of the next pass returns at once, so a pass reads A kk times
    // instead of kk + 1.  Every iterate is the one of the plain order (test,
    // fold, step): the step is only kept when the test fixed nothing.
    const bool pg = o->solver == BXS_PG;
    const bool cp = o->solver == BXS_CP;
    // Direct launches without profiling: the host waits for a pass by reading
    // the pass count the screening kernel publishes (no completion event
    // between passes on the stream); graph replay and profiling use events.
    const bool poll = !o->profile && !want_graph && !noalloc;
    int enq_passes = 0;
    int slot_seq[2] = {0, 0};
    // host_done: where the screening kernel publishes the stop counter
    // (nullptr inside a captured graph: a copy kernel follows the replay).
    long cdb_bound = P.cdb ? P.specs[0].n : 0;
    auto enqueue_kernels = [&](int slot, long long kk, int final_pass, int* host_done) -> bxs_status {
        for (long long k = 0; k < kk; ++k) {
            const int first = (k == 0) ? 1 : 0;
            if (o->profile) BXS_HIP(hipEventRecord(pev[(size_t)slot * 2 * K + 2 * k], stream));
            if (pg) {
                for (int b = 0; b < kNumVariants; ++b) BXS_HIP(sweep_pg(b, first));
            } else if (cp) {
                for (int b = 0; b < kNumVariants; ++b) BXS_HIP(sweep_cp(b));
            } else if (P.cdb) {
                // Gram blocks of the preserved list, which changes only at a screening
                // pass (the kernel returns at once when the list is unchanged); the
                // host's n bounds the device's block count
                if (k == 0) BXS_HIP(launch_cdb_gram(c, P.specs[0].n, P.cdb_gram));
                BXS_HIP(launch_cdb_sweep(c, P.specs[0].m, P.specs[0].n, cdb_bound, P.cdb_pg, P.cdb_gram,
                                         P.cdb_delta));
            } else {
                for (int b = 0; b < kNumCdBuckets; ++b) BXS_HIP(launch_cd(c, b, D.lists[b], D.n_list[b], 1));
            }
            if (o->profile) BXS_HIP(hipEventRecord(pev[(size_t)slot * 2 * K + 2 * k + 1], stream));
            if (pg) {
                BXS_HIP(launch_reduce(c, kRedResidual, D.ritems, D.n_ritems, first, D.nritems, D.n_nritems));
            } else if (cp) {
                BXS_HIP(launch_reduce(c, kRedCP, D.ritems, D.n_ritems, 0, D.nritems, D.n_nritems));
            } else if (!P.cdb || k == kk - 1) {
                // fresh residual from the updated iterate.  The block sweep keeps r
                // current itself (r -= A_J delta_J per block), so it needs this only
                // before a screening pass, whose rounding bounds take r = y' - A x
                // formed afresh.
                for (int b = 0; b < kNumVariants; ++b) BXS_HIP(launch_sweep(c, b, kModeAx, D.items[b], D.n_items[b]));
                BXS_HIP(launch_reduce(c, kRedResidual, D.ritems, D.n_ritems, 0, D.nritems, D.n_nritems));
            }
        }
        if (pg) {
            for (int b = 0; b < kNumVariants; ++b) BXS_HIP(sweep_pgs(b));
            BXS_HIP(launch_reduce(c, kRedAhead, D.ritems, D.n_ritems, 0, D.nritems, D.n_nritems));
        } else {
            if (cp) {
                // the screening test needs the residual at x (the iteration carries A x-bar)
                for (int b = 0; b < kNumVariants; ++b) BXS_HIP(launch_sweep(c, b, kModeAx, D.items[b], D.n_items[b]));
                BXS_HIP(launch_reduce(c, kRedResidual, D.ritems, D.n_ritems, 0, D.nritems, D.n_nritems));
            }
            for (int b = 0; b < kNumVariants; ++b) BXS_HIP(launch_sweep(c, b, kModeCorr, D.items[b], D.n_items[b]));
        }
        BXS_HIP(launch_screen(c, (int)count, o->eps_gap, o->screening, final_pass, K, (int)kk, pg ? 1 : 0,
                              host_done, (host_done && count == 1) ? hgap + slot : nullptr,
                              (host_done && poll) ? hseq : nullptr,
                              o->theta_star ? kScreenOracleDual
                                            : (o->fidelity == BXS_FID_HUBER ? kScreenHuber : kScreenLS),
                              (host_done && count == 1 && P.cdb) ? hnact + slot : nullptr));
        if (o->screening) {
            for (int b = 0; b < kNumVariants; ++b) BXS_HIP(launch_sweep(c, b, kModeFold, D.items[b], D.n_items[b]));
            BXS_HIP(launch_reduce(c, kRedFold, D.ritems, D.n_ritems, 0, D.nritems, D.n_nritems));
        }
        return BXS_OK;
    };

    // A regular pass (K iterations, not the last) has the same launches and
    // arguments every time: capture it once as a graph and replay it.
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    struct GraphGuard {
        hipGraph_t* g;
        hipGraphExec_t* e;
        ~GraphGuard() {
            if (*e) (void)hipGraphExecDestroy(*e);
            if (*g) (void)hipGraphDestroy(*g);
        }
    } gguard{&graph, &gexec};
    if (want_graph) {
        BXS_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
        const bxs_status cs = enqueue_kernels(0, K, 0, nullptr);
        const hipError_t ce = hipStreamEndCapture(stream, &graph);
        if (cs != BXS_OK) return cs;
        BXS_HIP(ce);
        BXS_HIP(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
    }

    auto enqueue_pass = [&](int slot) -> bxs_status {
        const long long kk = std::min<long long>(K, o->max_iter - iters);
        iters += kk;
        const int final_pass = iters >= o->max_iter;
        if (gexec && kk == K && !final_pass) {
            BXS_HIP(hipGraphLaunch(gexec, stream));
            BXS_HIP(launch_publish(c, hdone + slot));
        } else {
            const bxs_status es = enqueue_kernels(slot, kk, final_pass, noalloc ? nullptr : hdone + slot);
            if (es != BXS_OK) return es;
        }
        if (noalloc) BXS_HIP(hipMemcpyAsync(hdone + slot, D.done_counter, sizeof(int), hipMemcpyDeviceToHost, stream));
        else if (poll) slot_seq[slot] = ++enq_passes;
        else BXS_HIP(hipEventRecord(dev_done[slot], stream));
        slot_kk[slot] = kk;
        slot_final[slot] = final_pass;
        slot_gap[slot] = (!noalloc && count == 1 && !(gexec && kk == K && !final_pass)) ? 1 : 0;
        return BXS_OK;
    };

    // Single instance: the gaps of the last two passes predict the next one
    // (linear convergence); when it is predicted below eps_gap, the pass after
    // it is not enqueued ahead (it would only return at once), at the cost of
    // one host reaction when the prediction fails.
    double g_old = -1.0, g_new = -1.0;
    auto predict_stop = [&]() -> bool {
        if (!(g_old > 0.0) || !(g_new >= 0.0) || !(g_new < g_old)) return false;
        return g_new * (g_new / g_old) < o->eps_gap;
    };

    // Batches: each time the unfinished instances fall to half of those still
    // running at the last rebuild, the work-item, reduction and CD tables are
    // rebuilt over the unfinished ones (the stream is drained first, since
    // the pass in flight reads the tables), so the launches of the tail carry
    // no workgroups of finished instances.  Not under graph replay (the
    // captured pass holds the tables' sizes) nor without allocation.
    const bool compact_ok = !want_graph && !noalloc && count > 1;
    long live_prev = count;
    auto rebuild_tables = [&]() -> bxs_status {
        BXS_HIP(hipStreamSynchronize(stream));
        std::vector<State> hs(count);
        BXS_HIP(hipMemcpy(hs.data(), D.st, sbytes, hipMemcpyDeviceToHost));
        auto live = [&](int inst) { return hs[inst].done == 0; };
        long nlive = 0;
        for (long i = 0; i < count; ++i) nlive += live((int)i) ? 1 : 0;
        for (int b = 0; b < kNumVariants; ++b) {
            std::vector<Item>& v = P.items[b];
            v.erase(std::remove_if(v.begin(), v.end(), [&](const Item& it) { return !live(it.inst); }), v.end());
            if (!v.empty()) BXS_HIP(hipMemcpy(D.items[b], v.data(), sizeof(Item) * v.size(), hipMemcpyHostToDevice));
            D.n_items[b] = (int)v.size();
        }
        auto filt = [&](std::vector<RItem>& v) {
            v.erase(std::remove_if(v.begin(), v.end(), [&](const RItem& r) { return !live(r.inst); }), v.end());
        };
        filt(P.ritems);
        filt(P.nritems);
        // the narrow list keeps its place after the wide one's original end
        if (!P.ritems.empty())
            BXS_HIP(hipMemcpy(D.ritems, P.ritems.data(), sizeof(RItem) * P.ritems.size(), hipMemcpyHostToDevice));
        if (!P.nritems.empty())
            BXS_HIP(hipMemcpy(D.nritems, P.nritems.data(), sizeof(RItem) * P.nritems.size(), hipMemcpyHostToDevice));
        D.n_ritems = (int)P.ritems.size();
        D.n_nritems = (int)P.nritems.size();
        for (int b = 0; b < kNumCdBuckets; ++b) {
            std::vector<int>& v = P.cd_list[b];
            v.erase(std::remove_if(v.begin(), v.end(), [&](int i) { return !live(i); }), v.end());
            if (!v.empty()) BXS_HIP(hipMemcpy(D.lists[b], v.data(), sizeof(int) * v.size(), hipMemcpyHostToDevice));
            D.n_list[b] = (int)v.size();
        }
        live_prev = nlive;
        return BXS_OK;
    };

    int slot = 0;
    {
        bxs_status s = enqueue_pass(slot);
        if (s != BXS_OK) return s;
    }
    while (true) {
        const int nxt = slot ^ 1;
        bool queued_next = false;
        // allocation-free mode waits for each pass before enqueueing the next
        if (!noalloc && !slot_final[slot] && !predict_stop()) {
            bxs_status s = enqueue_pass(nxt);
            if (s != BXS_OK) return s;
            queued_next = true;
        }
        if (poll) {
            // spin on the coherent word; should it not advance (it always
            // does), the stream's completion makes every published value final
            const auto t0 = std::chrono::steady_clock::now();
            long spins = 0;
            while (__atomic_load_n(hseq, __ATOMIC_ACQUIRE) < slot_seq[slot]) {
                __builtin_ia32_pause();
                if ((++spins & 4095) == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::seconds(2)) {
                    BXS_HIP(hipStreamSynchronize(stream));
                    break;
                }
            }
        } else if (noalloc) {
            BXS_HIP(hipStreamSynchronize(stream));
        } else {
            BXS_HIP(hipEventSynchronize(dev_done[slot]));
        }
        if (slot_gap[slot]) {
            g_old = g_new;
            g_new = hgap[slot];
        }
        // the pass that just completed published its preserved-list length
        // (graph replay keeps the captured launches)
        if (P.cdb && slot_gap[slot] && hnact[slot] >= 0 && hnact[slot] < cdb_bound) cdb_bound = hnact[slot];
        if (o->profile) {
            for (long long k = 0; k < slot_kk[slot]; ++k) {
                // PG: the first sweep of a pass returns at once when the step
                // was taken ahead, so it is left out of the timing
                if (pg && k == 0 && K > 1) continue;
                float ms = 0.f;
                BXS_HIP(hipEventElapsedTime(&ms, pev[(size_t)slot * 2 * K + 2 * k], pev[(size_t)slot * 2 * K + 2 * k + 1]));
                sweep_ms += ms;
                ++sweep_launches;
            }
        }
        if (hdone[slot] >= count || slot_final[slot]) break;
        if (compact_ok) {
            const long live_now = count - hdone[slot];
            if (2 * live_now <= live_prev && live_prev - live_now >= 16) {
                const bxs_status rs = rebuild_tables();
                if (rs != BXS_OK) return rs;
            }
        }
        if (!queued_next) {
            bxs_status s = enqueue_pass(nxt);
            if (s != BXS_OK) return s;
        }
        slot = nxt;
    }
    if (!noalloc) BXS_HIP(hipEventRecord(ev2, stream));
    BXS_HIP(launch_count_free(c, (int)count));
    BXS_HIP(hipMemcpyAsync(img, D.st, sbytes, hipMemcpyDeviceToHost, stream));
    std::vector<bxs_pass_record> hrec;
    long nrec = 0;
    if (history && count == 1 && P.rec_cap > 0 && !noalloc) {
        hrec.resize(P.rec_cap);
        BXS_HIP(hipMemcpyAsync(hrec.data(), P.insts[0].rec, sizeof(bxs_pass_record) * P.rec_cap,
                               hipMemcpyDeviceToHost, stream));
    }
    BXS_HIP(hipStreamSynchronize(stream));
    stage_guard.done = true;
    memcpy(hst.data(), img, sbytes);
    for (long i = 0; i < count; ++i) {
        if (hst[i].err & kErrNonfinite) return fail(BXS_ERR_NONFINITE, "problem %ld: non-finite value in A, y, x0, t or bounds", i);
        if (hst[i].err & kErrBounds) return fail(BXS_ERR_BOUNDS, "problem %ld: l_j = -inf, u_j = -inf or l_j > u_j", i);
    }
    float ms_setup = 0.f, ms_solve = 0.f;
    if (noalloc) {
        // no events: the host's wall time of the whole call
        ms_solve = (float)std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - host_t0).count();
    } else {
        BXS_HIP(hipEventElapsedTime(&ms_setup, ev0, ev1));
        BXS_HIP(hipEventElapsedTime(&ms_solve, ev1, ev2));
    }

    bxs_status worst = BXS_OK;
    for (long i = 0; i < count; ++i) {
        const State& S = hst[i];
        const int status = S.done ? S.status : BXS_MAXITER;
        if (status != BXS_OK) worst = (bxs_status)status;
        if (infos) {
            bxs_info& f = infos[i];
            memset(&f, 0, sizeof(f));
            f.status = status;
            f.t_valid = S.t_valid;
            f.iters = S.done ? S.iters : iters;
            f.passes = S.passes;
            f.n_active = S.n_active;
            f.n_lower = S.n_lower;
            f.n_upper = S.n_upper;
            f.gap = S.gap;
            f.primal = S.primal;
            f.radius = S.radius;
            f.eps = S.eps;
            f.step = S.step;
            f.lipschitz = S.lipschitz;
            f.ms_setup = ms_setup;
            f.ms_solve = ms_solve;
            f.col_iters = S.col_iters;
            f.sweep_ms = sweep_ms;
            f.sweep_launches = sweep_launches;
            f.event_overhead_ms = ev_over;
            f.t_column = P.tdir ? S.t_column : -1;
            f.dual = S.primal - S.gap;
            f.max_margin = S.margin;
            f.n_free = S.n_free;
        }
    }
    if (history && count == 1) {
        nrec = std::min<long>(hst[0].passes, std::min<long>(history_cap, P.rec_cap));
        if (noalloc) {
            // straight into the caller's array, the records of the passes run only
            if (nrec > 0) {
                BXS_HIP(hipMemcpyAsync(history, P.insts[0].rec, sizeof(bxs_pass_record) * nrec,
                                       hipMemcpyDeviceToHost, stream));
                BXS_HIP(hipStreamSynchronize(stream));
            }
        } else {
            for (long k = 0; k < nrec; ++k) history[k] = hrec[k];
        }
    }
    return worst;
}

// Fixed device scratch of the allocation-free entry point: one copy per GPU,
// held from the library's load until the process ends.  In host code the
// name `scratch` is only a host-side stand-in; the device address of each
// GPU's copy comes from hipGetSymbolAddress and is the only form passed on.
static __device__ __align__(256) unsigned char scratch[BXS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static void* g_scratch_ptr[kMaxDevices];
// Serialises the allocation-free calls of the process: they share each GPU's
// scratch array and the host staging area below.
static std::mutex g_noalloc_mu;
constexpr size_t kNoallocHostBytes = (size_t)4 << 20;
alignas(256) static char g_noalloc_host[kNoallocHostBytes];

static bxs_status scratch_for_current_device(void** out)
{
    int dev = 0;
    BXS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(BXS_ERR_DEVICE, "device index %d out of range", dev);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(BXS_ERR_DEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return BXS_OK;
}

}  // namespace bxs

using namespace bxs;

extern "C" {

void bxs_default_opts(bxs_opts* o)
{
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->solver = BXS_PG;
    o->screening = 1;
    o->screen_every = 10;
    o->max_iter = 100000;
    o->eps_gap = 1e-6;
    o->step = 0.0;
    o->power_iters = 0;
    o->graph = 0;
}

const char* bxs_last_error(void) { return g_last_error.c_str(); }

int bxs_num_sweep_variants(void) { return kNumVariants; }

bxs_status bxs_sweep_variant_info(int v, int* tpc, int* ng, int* rows, int* cbi, int* pd, long* capacity)
{
    if (v < 0 || v >= kNumVariants) return fail(BXS_ERR_ARG, "variant %d out of range", v);
    if (pd) *pd = kVariants[v].pd;
    if (tpc) *tpc = kVariants[v].tpc;
    if (ng) *ng = kVariants[v].ng;
    if (rows) *rows = kVariants[v].rows;
    if (cbi) *cbi = kVariants[v].cbi;
    if (capacity) *capacity = variant_capacity(v);
    return BXS_OK;
}

int bxs_row_class(long m) { return default_variant_for_rows(m); }

int bxs_sweep_variant_for_rows(long m) { return choose_variant(m); }

bxs_status bxs_set_sweep_variant(int row_class, int v)
{
    if (row_class < 0 || row_class >= kNumDefaultVariants) return fail(BXS_ERR_ARG, "row class %d out of range", row_class);
    if (v < 0) v = row_class;
    if (v >= kNumVariants) return fail(BXS_ERR_ARG, "variant %d out of range", v);
    if (variant_capacity(v) < variant_capacity(row_class))
        return fail(BXS_ERR_ARG, "variant %d holds %ld rows, class %d needs %ld", v, variant_capacity(v), row_class,
                    variant_capacity(row_class));
    g_variant_pref[row_class] = v;
    return BXS_OK;
}

bxs_status bxs_set_group_scale(int row_class, double scale)
{
    if (row_class < 0 || row_class >= kNumDefaultVariants) return fail(BXS_ERR_ARG, "row class %d out of range", row_class);
    if (!(scale >= 1.0 / 64.0 && scale <= 4.0)) return fail(BXS_ERR_ARG, "group scale %g outside [1/64, 4]", scale);
    g_group_scale[row_class] = scale;
    return BXS_OK;
}

bxs_status bxs_set_cd_block(int enable)
{
    if (enable != 0 && enable != 1) return fail(BXS_ERR_ARG, "enable must be 0 or 1");
    g_cd_block = enable;
    return BXS_OK;
}

double bxs_group_scale(int row_class)
{
    return (row_class >= 0 && row_class < kNumDefaultVariants) ? g_group_scale[row_class] : 0.0;
}

const char* bxs_version(void) { return "boxscreen 0.1.0 (gfx950)"; }

bxs_status bxs_workspace_size_batch(long count, const long* m, const long* n, const bxs_opts* opts, size_t* bytes)
{
    if (count < 1 || !m || !n || !bytes) return fail(BXS_ERR_ARG, "bad arguments to bxs_workspace_size_batch");
    bxs_status s = check_opts(opts);
    if (s != BXS_OK) return s;
    Plan P;
    P.specs.resize(count);
    for (long i = 0; i < count; ++i) {
        InstSpec& sp = P.specs[i];
        memset(&sp, 0, sizeof(sp));
        sp.m = m[i]; sp.n = n[i]; sp.lda = m[i];
        if (sp.m < 1 || sp.n < 1 || sp.m > BXS_MAX_ROWS) return fail(BXS_ERR_SHAPE, "problem %ld: bad shape", i);
    }
    build_plan(P, BXS_F64, (count == 1 && opts->history) ? opts->history_cap : 0, lanczos_steps(opts),
               opts->t_choice, cd_block_on(opts, count));
    *bytes = P.bytes;
    return BXS_OK;
}

bxs_status bxs_workspace_size(long m, long n, const bxs_opts* opts, size_t* bytes)
{
    return bxs_workspace_size_batch(1, &m, &n, opts, bytes);
}

static bxs_status solve_common(std::vector<InstSpec>& specs, int a_dtype, const bxs_opts* opts, bxs_info* infos,
                               const FixedArea* fixed = nullptr)
{
    g_last_error.clear();
    bxs_status s = check_opts(opts);
    if (s != BXS_OK) return s;
    if (a_dtype != BXS_F64 && a_dtype != BXS_F32 && a_dtype != BXS_BF16)
        return fail(BXS_ERR_ARG, "unknown a_dtype %d", a_dtype);
    for (size_t i = 0; i < specs.size(); ++i) {
        s = check_spec(specs[i], (long)i);
        if (s != BXS_OK) return s;
    }
    if (opts->t_choice != BXS_T_GIVEN && specs.size() != 1)
        return fail(BXS_ERR_ARG, "t_choice is available for single problems only");
    if (opts->t_choice == BXS_T_NORMAL_EQUATIONS && specs[0].n > specs[0].m)
        return fail(BXS_ERR_ARG, "the normal-equations direction (Prop. 2, case 1) needs n <= m, got n=%ld m=%ld",
                    specs[0].n, specs[0].m);
    Plan P;
    P.specs = specs;
    const long rc = (specs.size() == 1 && opts->history) ? opts->history_cap : 0;
    // the allocation-free entry keeps its fixed scratch bound: one workgroup per instance
    const int cdb = fixed ? 0 : cd_block_on(opts, (long)specs.size());
    s = build_plan(P, a_dtype, rc, lanczos_steps(opts), opts->t_choice, cdb);
    if (s != BXS_OK) return s;
    return run(P, a_dtype, opts, opts->t, infos, opts->history, opts->history_cap, fixed);
}

bxs_status solve_bvls(long m, long n, int a_dtype, const void* A, long lda, const double* y, const double* l,
                      const double* u, double* x, signed char* sat, const bxs_opts* opts, bxs_info* info)
{
    if (!l || !u) return fail(BXS_ERR_ARG, "solve_bvls needs both bound arrays (use solve_nnls for l=0, u=+inf)");
    std::vector<InstSpec> specs(1);
    specs[0] = InstSpec{m, n, lda, A, y, l, u, x, sat};
    return solve_common(specs, a_dtype, opts, info);
}

bxs_status solve_bvls_noalloc(long m, long n, int a_dtype, const void* A, long lda, const double* y,
                              const double* l, const double* u, double* x, signed char* sat, const bxs_opts* opts,
                              bxs_info* info)
{
    g_last_error.clear();
    if (!l || !u) return fail(BXS_ERR_ARG, "solve_bvls_noalloc needs both bound arrays");
    if (!opts) return fail(BXS_ERR_ARG, "opts is NULL");
    if (opts->workspace) return fail(BXS_ERR_ARG, "solve_bvls_noalloc uses its fixed scratch: opts->workspace must be NULL");
    if (opts->graph) return fail(BXS_ERR_ARG, "solve_bvls_noalloc does not capture graphs: opts->graph must be 0");
    if (opts->profile) return fail(BXS_ERR_ARG, "solve_bvls_noalloc creates no events: opts->profile must be 0");
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    void* dev_scratch = nullptr;
    bxs_status s = scratch_for_current_device(&dev_scratch);
    if (s != BXS_OK) return s;
    const FixedArea fixed{dev_scratch, (size_t)BXS_NOALLOC_SCRATCH_BYTES, g_noalloc_host, kNoallocHostBytes};
    std::vector<InstSpec> specs(1);
    specs[0] = InstSpec{m, n, lda, A, y, l, u, x, sat};
    return solve_common(specs, a_dtype, opts, info, &fixed);
}

bxs_status solve_nnls(long m, long n, int a_dtype, const void* A, long lda, const double* y, double* x,
                      signed char* sat, const bxs_opts* opts, bxs_info* info)
{
    std::vector<InstSpec> specs(1);
    specs[0] = InstSpec{m, n, lda, A, y, nullptr, nullptr, x, sat};
    return solve_common(specs, a_dtype, opts, info);
}

static bxs_status check_batched(long m, long n, long B, int a_dtype, const void* A, long lda, const double* Y,
                                long ldy, const double* X, long ldx, const signed char* sat, long ldsat,
                                const bxs_opts* opts)
{
    bxs_status s = check_opts(opts);
    if (s != BXS_OK) return s;
    if (opts->solver != BXS_PG) return fail(BXS_ERR_ARG, "the batched shared-matrix solver runs projected gradient");
    if (opts->fidelity != BXS_FID_LS) return fail(BXS_ERR_ARG, "the batched shared-matrix solver is least squares only");
    if (a_dtype != BXS_F64 && a_dtype != BXS_F32) return fail(BXS_ERR_ARG, "unknown a_dtype %d", a_dtype);
    if (m < 1 || n < 1 || B < 1) return fail(BXS_ERR_SHAPE, "m=%ld n=%ld B=%ld must be >= 1", m, n, B);
    if (lda < m || ldy < m || ldx < n || ldsat < n) return fail(BXS_ERR_SHAPE, "a leading dimension is too small");
    if ((double)m * (double)B > 2e9 || (double)n * (double)B > 2e9 || (double)m * (double)n > 2e9)
        return fail(BXS_ERR_SHAPE, "batched problem too large for 32-bit GEMM sizes");
    if (!A || !Y || !X || !sat) return fail(BXS_ERR_ARG, "NULL array argument");
    return BXS_OK;
}

bxs_status bxs_workspace_size_batched(long m, long n, long B, const bxs_opts* opts, size_t* bytes)
{
    if (!opts || !bytes) return fail(BXS_ERR_ARG, "NULL argument");
    if (m < 1 || n < 1 || B < 1) return fail(BXS_ERR_SHAPE, "m=%ld n=%ld B=%ld must be >= 1", m, n, B);
    *bytes = batched_workspace_bytes(m, n, B, opts->iter_precision);
    return BXS_OK;
}

bxs_status solve_nnls_batched_shared(long m, long n, long B, int a_dtype, const void* A, long lda, const double* Y,
                                     long ldy, double* X, long ldx, signed char* sat, long ldsat, const bxs_opts* opts,
                                     bxs_info* infos)
{
    g_last_error.clear();
    bxs_status s = check_batched(m, n, B, a_dtype, A, lda, Y, ldy, X, ldx, sat, ldsat, opts);
    if (s != BXS_OK) return s;
    return batched_nnls_run(m, n, B, a_dtype, A, lda, Y, ldy, X, ldx, sat, ldsat, opts, infos);
}

bxs_status bxs_workspace_size_adjoint(long m, long n, long B, size_t* bytes)
{
    if (!bytes) return fail(BXS_ERR_ARG, "NULL argument");
    if (m < 1 || n < 1 || B < 1) return fail(BXS_ERR_SHAPE, "m=%ld n=%ld B=%ld must be >= 1", m, n, B);
    *bytes = adjoint_workspace_bytes(m, n, B);
    return BXS_OK;
}

static bxs_status adjoint_common(long m, long n, long B, int a_dtype, const void* A, long lda, const double* Y,
                                 long ldy, const double* X, long ldx, const double* l, const double* u,
                                 const double* dX, long ldg, double* dY, long lddy, double* dA, long ldda, double* dl,
                                 long lddl, double* du, long lddu, const bxs_opts* opts, long* cg_iters)
{
    g_last_error.clear();
    if (!opts) return fail(BXS_ERR_ARG, "opts is NULL");
    if (opts->max_iter < 1) return fail(BXS_ERR_ARG, "max_iter must be >= 1");
    if (!(opts->eps_gap >= 0.0) || isinf(opts->eps_gap)) return fail(BXS_ERR_ARG, "eps_gap must be finite and >= 0");
    if (opts->fidelity != BXS_FID_LS) return fail(BXS_ERR_ARG, "the adjoint is for the least-squares fidelity");
    if (a_dtype != BXS_F64 && a_dtype != BXS_F32) return fail(BXS_ERR_ARG, "unknown a_dtype %d", a_dtype);
    if (m < 1 || n < 1 || B < 1) return fail(BXS_ERR_SHAPE, "m=%ld n=%ld B=%ld must be >= 1", m, n, B);
    if (lda < m || ldy < m || ldx < n || ldg < n || lddy < m || (dA && ldda < m) || (dl && lddl < n) ||
        (du && lddu < n))
        return fail(BXS_ERR_SHAPE, "a leading dimension is too small");
    if ((double)m * (double)B > 2e9 || (double)n * (double)B > 2e9 || (double)m * (double)n > 2e9)
        return fail(BXS_ERR_SHAPE, "adjoint problem too large for 32-bit GEMM sizes");
    if (!A || !Y || !X || !dX || !dY) return fail(BXS_ERR_ARG, "NULL array argument");
    return adjoint_run(m, n, B, a_dtype, A, lda, Y, ldy, X, ldx, l, u, dX, ldg, dY, lddy, dA, ldda, dl, lddl, du,
                       lddu, opts, cg_iters);
}

bxs_status nnls_adjoint(long m, long n, long B, int a_dtype, const void* A, long lda, const double* Y, long ldy,
                        const double* X, long ldx, const double* dX, long ldg, double* dY, long lddy, double* dA,
                        long ldda, double* dl, long lddl, const bxs_opts* opts, long* cg_iters)
{
    return adjoint_common(m, n, B, a_dtype, A, lda, Y, ldy, X, ldx, nullptr, nullptr, dX, ldg, dY, lddy, dA, ldda,
                          dl, lddl, nullptr, 0, opts, cg_iters);
}

bxs_status bvls_adjoint(long m, long n, long B, int a_dtype, const void* A, long lda, const double* Y, long ldy,
                        const double* X, long ldx, const double* l, const double* u, const double* dX, long ldg,
                        double* dY, long lddy, double* dA, long ldda, double* dl, long lddl, double* du, long lddu,
                        const bxs_opts* opts, long* cg_iters)
{
    return adjoint_common(m, n, B, a_dtype, A, lda, Y, ldy, X, ldx, l, u, dX, ldg, dY, lddy, dA, ldda, dl, lddl,
                          du, lddu, opts, cg_iters);
}

bxs_status solve_bvls_varbatch(long count, int a_dtype, const bxs_problem* probs, const bxs_opts* opts,
                               bxs_info* infos)
{
    if (count < 1 || !probs) return fail(BXS_ERR_ARG, "count < 1 or probs is NULL");
    if (!opts) return fail(BXS_ERR_ARG, "opts is NULL");
    std::vector<InstSpec> specs(count);
    for (long i = 0; i < count; ++i) {
        const bxs_problem& p = probs[i];
        specs[i] = InstSpec{p.m, p.n, p.lda, p.A, p.y, p.l, p.u, p.x, p.sat};
    }
    bxs_opts o2 = *opts;
    o2.history = nullptr;
    o2.history_cap = 0;
    return solve_common(specs, a_dtype, &o2, infos);
}

}  // extern "C"
