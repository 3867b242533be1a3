// plan.hip -- host side of the fused uneven batch: validation, work units,
// cost-ordered per-XCD queues, graph capture, and the per-shape grouped
// execution that serves as its comparison.
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "../../include/mi355blas.h"
#include "fused_tuned.h"
#include "mb_internal.h"

namespace {

using mb::FusedTask;

// Per problem with work: the task template (i0 = j0 = 0) and its tiling.
struct ProblemWork {
    FusedTask t;
    int tile_rows, tile_cols;  // rows / columns of C per task
    int64_t tiles_m, tiles_n;
};

int tcode(char t)
{
    switch (t) {
    case 'N': case 'n': return 0;
    case 'T': case 't': case 'C': case 'c': return 1;
    default: return -1;
    }
}

int laset_code(char u)  // 0 upper, 1 lower, 2 all, -1 illegal
{
    switch (u) {
    case 'U': case 'u': return 0;
    case 'L': case 'l': return 1;
    case 'A': case 'a': return 2;
    default: return -1;
    }
}

// Elements spanned by a column-major rows x cols operand with leading dimension ld.
int64_t span(int64_t rows, int64_t cols, int64_t ld)
{
    return (rows == 0 || cols == 0) ? 0 : ld * (cols - 1) + rows;
}

constexpr int64_t kMaxSpan = ((int64_t)1 << 32) / 8 - 1;  // 32-bit byte offsets

// Validate one problem: MB_OK, MB_ERR_INVALID_PROBLEM or MB_ERR_UNSUPPORTED.
// *work is false for a dgemm quick return.
int check_problem(const mb_problem &p, bool *work)
{
    *work = false;
    if (p.op == MB_OP_DGEMM) {
        const int ta = tcode(p.transa), tb = tcode(p.transb);
        if (ta < 0 || tb < 0 || p.m < 0 || p.n < 0 || p.k < 0)
            return MB_ERR_INVALID_PROBLEM;
        const int arows = ta ? p.k : p.m, acols = ta ? p.m : p.k;
        const int brows = tb ? p.n : p.k, bcols = tb ? p.k : p.n;
        if (p.lda < std::max(1, arows) || p.ldb < std::max(1, brows) || p.ldc < std::max(1, p.m))
            return MB_ERR_INVALID_PROBLEM;
        if (p.m == 0 || p.n == 0 || ((p.alpha == 0.0 || p.k == 0) && p.beta == 1.0))
            return MB_OK;
        const bool reads_ab = p.alpha != 0.0 && p.k > 0;
        if ((reads_ab && (!p.A || !p.B)) || !p.C)
            return MB_ERR_INVALID_PROBLEM;
        if (span(arows, acols, p.lda) > kMaxSpan || span(brows, bcols, p.ldb) > kMaxSpan ||
            span(p.m, p.n, p.ldc) > kMaxSpan)
            return MB_ERR_UNSUPPORTED;
        *work = true;
        return MB_OK;
    }
    if (p.op == MB_OP_DPOTRF_ADJOINT) {
        if (p.n < 0 || p.lda < std::max(1, p.n) || p.ldb < std::max(1, p.n) ||
            p.ldc < std::max(1, p.n))
            return MB_ERR_INVALID_PROBLEM;
        if (p.n > mb::POTRF_MAX_N)
            return MB_ERR_UNSUPPORTED;
        if (p.n == 0)
            return MB_OK;
        if (!p.A || !p.B || !p.C)
            return MB_ERR_INVALID_PROBLEM;
        if (span(p.n, p.n, p.lda) > kMaxSpan || span(p.n, p.n, p.ldb) > kMaxSpan ||
            span(p.n, p.n, p.ldc) > kMaxSpan)
            return MB_ERR_UNSUPPORTED;
        *work = true;
        return MB_OK;
    }
    if (p.op == MB_OP_DLASET) {
        if (laset_code(p.uplo) < 0 || p.m < 0 || p.n < 0 || p.ldc < std::max(1, p.m))
            return MB_ERR_INVALID_PROBLEM;
        if (p.m == 0 || p.n == 0)
            return MB_OK;
        if (!p.C)
            return MB_ERR_INVALID_PROBLEM;
        if (span(p.m, p.n, p.ldc) > kMaxSpan)
            return MB_ERR_UNSUPPORTED;
        *work = true;
        return MB_OK;
    }
    if (p.op == MB_OP_DPOTRF) {
        if (p.uplo == 'U' || p.uplo == 'u')
            return MB_ERR_UNSUPPORTED;
        if ((p.uplo != 'L' && p.uplo != 'l') || p.n < 0 || p.ldc < std::max(1, p.n))
            return MB_ERR_INVALID_PROBLEM;
        if (p.n > mb::POTRF_MAX_N)
            return MB_ERR_UNSUPPORTED;
        if ((p.n > 0 && !p.C) || !p.info)
            return MB_ERR_INVALID_PROBLEM;
        if (span(p.n, p.n, p.ldc) > kMaxSpan)
            return MB_ERR_UNSUPPORTED;
        *work = true;  // n == 0 still writes info = 0
        return MB_OK;
    }
    return MB_ERR_INVALID_PROBLEM;
}

double gemm_unit_ns(int tm, int tn, int k)
{
    const int chunks = (k + 15) / 16;
    return mb::kFusedGemmFixedNs + mb::kFusedGemmTileNs * tm * tn +
           chunks * (mb::kFusedGemmMfmaNs * tm * tn + mb::kFusedGemmLoadNs * (tm + tn));
}

double potrf_unit_ns(int n)
{
    const double t = (n + 15) / 16;
    const double *c = mb::kFusedPotrfNs;
    return c[0] + t * (c[1] + t * (c[2] + t * c[3]));
}

double adjoint_unit_ns(int n)
{
    const double t = (n + 15) / 16;
    const double *c = mb::kFusedAdjointNs;
    return c[0] + t * (c[1] + t * (c[2] + t * c[3]));
}

// Sub-allocation of the plan's single device block.
struct Arena {
    size_t size = 0;
    size_t take(size_t bytes)
    {
        const size_t at = size;
        size += (bytes + 255) & ~(size_t)255;
        return at;
    }
};

}  // namespace

// One pointer-array batched call of the grouped execution.
struct PlanGroup {
    int op, ta, tb, m, n, k, lda, ldb, ldc;
    double alpha, beta;
    int64_t off, count;  // slice of the group pointer arrays
    int64_t info_off;    // dpotrf: slice of the info staging array
};

struct mb_plan {
    int device = 0;
    int64_t problems = 0, units = 0, idle = 0;
    int grid = 0, waves_per_cu = 0;
    double cost_ns = 0.0;
    char *dmem = nullptr;
    mb::FusedArgs args{};
    hipStream_t cap = nullptr;
    hipGraphExec_t fused_exec = nullptr;
    // grouped execution
    std::vector<PlanGroup> groups;
    int64_t gemm_groups = 0, other_groups = 0;
    const double **gA = nullptr, **gB = nullptr;
    double **gC = nullptr;
    int *ginfo = nullptr;
    int **ginfo_dst = nullptr;
    int64_t ninfo = 0;
    hipGraphExec_t grouped_exec = nullptr;
};

namespace {

int to_status(hipError_t e) { return e == hipSuccess ? MB_OK : MB_ERR_HIP; }

void release(mb_plan *p)
{
    if (p->fused_exec)
        (void)hipGraphExecDestroy(p->fused_exec);
    if (p->grouped_exec)
        (void)hipGraphExecDestroy(p->grouped_exec);
    if (p->cap)
        (void)hipStreamDestroy(p->cap);
    if (p->dmem)
        (void)hipFree(p->dmem);
    delete p;
}

int run_fused(mb_plan *p, hipStream_t s)
{
    if (p->units == 0)
        return MB_OK;
    return to_status(mb::launch_fused(p->args, p->grid, s));
}

int run_grouped(mb_plan *p, hipStream_t s)
{
    for (const PlanGroup &g : p->groups) {
        int st;
        if (g.op == MB_OP_DGEMM) {
            mb::GemmArgs a{};
            a.m = g.m; a.n = g.n; a.k = g.k; a.alpha = g.alpha; a.beta = g.beta;
            a.Aarr = p->gA + g.off; a.lda = g.lda;
            a.Barr = p->gB + g.off; a.ldb = g.ldb;
            a.Carr = p->gC + g.off; a.ldc = g.ldc;
            a.batch = (int)g.count;
            st = mb::run_gemm(g.ta, g.tb, a, MB_VARIANT_AUTO, -1, s);
        } else if (g.op == MB_OP_DPOTRF) {
            mb::PotrfArgs a{};
            a.n = g.n; a.Aarr = p->gC + g.off; a.lda = g.ldc;
            a.info = p->ginfo + g.info_off; a.batch = (int)g.count;
            st = mb::run_potrf(a, s);
        } else if (g.op == MB_OP_DPOTRF_ADJOINT) {
            mb::PotrfAdjArgs a{};
            a.n = g.n;
            a.Larr = p->gA + g.off; a.ldl = g.lda;
            a.Lbararr = p->gB + g.off; a.ldlb = g.ldb;
            a.Abararr = p->gC + g.off; a.ldab = g.ldc;
            a.batch = (int)g.count;
            st = to_status(mb::launch_potrf_adj(a, s));
        } else {
            mb::LasetArgs a{};
            a.uplo = g.ta; a.m = g.m; a.n = g.n; a.alpha = g.alpha; a.beta = g.beta;
            a.Aarr = p->gC + g.off; a.lda = g.ldc; a.batch = (int)g.count;
            st = to_status(mb::launch_laset(a, s));
        }
        if (st != MB_OK)
            return st;
    }
    return to_status(mb::launch_scatter_info(p->ginfo, p->ginfo_dst, (int)p->ninfo, s));
}

// Capture fn(plan, cap) on the plan's own stream into an executable graph.
template <class Fn>
int capture(mb_plan *p, Fn fn, hipGraphExec_t *out)
{
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess)
        return MB_ERR_HIP;
    const int st = fn(p, p->cap);
    e = hipStreamEndCapture(p->cap, &g);
    if (st != MB_OK || e != hipSuccess) {
        if (g)
            (void)hipGraphDestroy(g);
        return st != MB_OK ? st : MB_ERR_HIP;
    }
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    return to_status(e);
}

// Restores the caller's current device on scope exit.
struct DeviceGuard {
    int saved = -1;
    bool ok = false;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&saved) != hipSuccess)
            return;
        ok = saved == dev || hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (saved >= 0 && hipGetDevice(&cur) == hipSuccess && cur != saved)
            (void)hipSetDevice(saved);
    }
};

}  // namespace

extern "C" {

int mb_plan_create(const mb_problem *problems, int64_t count, mb_plan **plan,
                   int64_t *bad_index)
{
    if (count > 0 && !problems) return -1;
    if (count < 0) return -2;
    if (!plan) return -3;
    return mb_plan_create_ex(problems, count, nullptr, plan, bad_index);
}

int mb_plan_create_ex(const mb_problem *problems, int64_t count, const mb_plan_options *options,
                      mb_plan **plan, int64_t *bad_index)
{
    if (count > 0 && !problems) return -1;
    if (count < 0) return -2;
    if (!plan) return -4;
    if (options && options->potrf_waves > mb::kFusedWaves) return -3;
    const int two_min =
        (options && options->tile_two_min >= 0) ? options->tile_two_min : mb::kFusedTwoMin;
    *plan = nullptr;
    if (count > (int64_t)UINT32_MAX) return MB_ERR_UNSUPPORTED;

    // ---- validate, choose tiles, estimate costs ---------------------------
    std::vector<ProblemWork> desc;
    std::vector<double> unit_ns;   // per problem with work
    std::vector<uint32_t> nunits;  // per problem with work
    std::vector<int64_t> src;      // problem index of each descriptor
    int64_t idle = 0, total_units = 0;
    double total_ns = 0.0;
    for (int64_t i = 0; i < count; ++i) {
        const mb_problem &q = problems[i];
        bool work = false;
        const int st = check_problem(q, &work);
        if (st != MB_OK) {
            if (bad_index) *bad_index = i;
            return st;
        }
        if (!work) {
            ++idle;
            continue;
        }
        ProblemWork w{};
        FusedTask &d = w.t;
        double ns;
        int64_t nu;
        if (q.op == MB_OP_DGEMM) {
            const int ta = tcode(q.transa), tb = tcode(q.transb);
            const bool scale_only = q.alpha == 0.0 || q.k == 0;
            const int tm = q.m > two_min ? 2 : 1;
            const int tn = q.n > two_min ? 2 : 1;
            d.A = scale_only ? nullptr : q.A;
            d.B = scale_only ? nullptr : q.B;
            d.C = q.C;
            d.alpha = scale_only ? 0.0 : q.alpha;
            d.beta = q.beta;
            d.m = q.m; d.n = q.n; d.k = scale_only ? 0 : q.k;
            d.lda = q.lda; d.ldb = q.ldb; d.ldc = q.ldc;
            d.kind = (2 * ta + tb) | ((tm - 1) << 2) | ((tn - 1) << 3);
            w.tile_rows = 16 * tm;
            w.tile_cols = 16 * tn;
            w.tiles_m = (q.m + w.tile_rows - 1) / w.tile_rows;
            w.tiles_n = (q.n + w.tile_cols - 1) / w.tile_cols;
            nu = w.tiles_m * w.tiles_n;
            ns = gemm_unit_ns(tm, tn, d.k);
        } else if (q.op == MB_OP_DPOTRF) {
            d.C = q.C; d.info = q.info;
            d.n = q.n; d.ldc = q.ldc;
            d.kind = mb::FUSED_POTRF;
            w.tiles_m = w.tiles_n = 1;
            nu = 1;
            ns = potrf_unit_ns(q.n);
        } else if (q.op == MB_OP_DPOTRF_ADJOINT) {
            d.A = q.A; d.B = q.B; d.C = q.C;
            d.n = q.n; d.lda = q.lda; d.ldb = q.ldb; d.ldc = q.ldc;
            d.kind = mb::FUSED_POTRF_ADJ;
            w.tiles_m = w.tiles_n = 1;
            nu = 1;
            ns = adjoint_unit_ns(q.n);
        } else {  // MB_OP_DLASET: one task per block of columns
            d.C = q.C;
            d.m = q.m; d.n = q.n; d.ldc = q.ldc; d.k = laset_code(q.uplo);
            d.alpha = q.alpha; d.beta = q.beta;
            d.kind = mb::FUSED_LASET;
            w.tile_rows = q.m;
            w.tile_cols = mb::FUSED_LASET_COLS;
            w.tiles_m = 1;
            w.tiles_n = (q.n + w.tile_cols - 1) / w.tile_cols;
            nu = w.tiles_n;
            ns = mb::kFusedLasetNs;
        }
        if (total_units + nu > (int64_t)INT32_MAX) {
            if (bad_index) *bad_index = i;
            return MB_ERR_UNSUPPORTED;
        }
        desc.push_back(w);
        unit_ns.push_back(ns);
        nunits.push_back((uint32_t)nu);
        src.push_back(i);
        total_units += nu;
        total_ns += ns * nu;
    }

    // ---- longest-processing-time order, greedy balance over the queues ----
    const int64_t nd = (int64_t)desc.size();
    std::vector<uint32_t> order(nd);
    for (int64_t i = 0; i < nd; ++i) order[i] = (uint32_t)i;
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t a, uint32_t b) { return unit_ns[a] > unit_ns[b]; });
    // dpotrf problems: longest first, each to the least-loaded XCD (greedy
    // LPT); dgemm problems: in address order, cut into one contiguous run per
    // XCD of equal estimated cost, so that concurrent tiles touch nearby
    // memory (problem order is arena order for the usual tight layouts).
    std::vector<std::vector<uint32_t>> qprob(mb::FUSED_QUEUES);
    double load[mb::FUSED_XCDS] = {};
    double gemm_ns = 0.0;
    auto long_kind = [&](int64_t i) {
        return desc[i].t.kind == mb::FUSED_POTRF || desc[i].t.kind == mb::FUSED_POTRF_ADJ;
    };
    for (uint32_t pi : order) {
        if (!long_kind(pi))
            continue;
        int best = 0;
        for (int x = 1; x < mb::FUSED_XCDS; ++x)
            if (load[x] < load[best]) best = x;
        load[best] += unit_ns[pi] * nunits[pi];
        qprob[mb::FUSED_CLASSES * best + 0].push_back(pi);
    }
    for (int64_t i = 0; i < nd; ++i)
        if (!long_kind(i)) gemm_ns += unit_ns[i] * nunits[i];
    // waves of a workgroup that start on the dpotrf class: in proportion to
    // its share of the estimated work (scaled by the measured best split), at
    // least one while both classes exist
    int potrf_waves = 0;
    if (options && options->potrf_waves >= 0) {
        potrf_waves = options->potrf_waves;
    } else {
        const double potrf_ns = total_ns - gemm_ns;
        if (potrf_ns > 0.0 && gemm_ns <= 0.0) {
            potrf_waves = mb::kFusedWaves;
        } else if (potrf_ns > 0.0) {
            const double share = std::min(1.0, potrf_ns / total_ns * mb::kFusedPotrfShareScale);
            potrf_waves = (int)(mb::kFusedWaves * share + 0.5);
            potrf_waves = std::min(std::max(potrf_waves, 1), mb::kFusedWaves - 1);
        }
    }
    double done = 0.0;
    for (int64_t i = 0; i < nd; ++i) {
        if (long_kind(i))
            continue;
        int x = gemm_ns > 0.0 ? (int)(done / gemm_ns * mb::FUSED_XCDS) : 0;
        if (x >= mb::FUSED_XCDS) x = mb::FUSED_XCDS - 1;
        qprob[mb::FUSED_CLASSES * x + 1].push_back((uint32_t)i);
        done += unit_ns[i] * nunits[i];
    }
    // a queue lists its problems in that order, the tiles of one problem
    // adjacent (column-major over the tile grid) so they share the L2
    std::vector<FusedTask> units;
    units.reserve((size_t)total_units);
    std::vector<int> qoff(mb::FUSED_QUEUES + 1, 0);
    for (int q = 0; q < mb::FUSED_QUEUES; ++q) {
        qoff[q] = (int)units.size();
        for (uint32_t pi : qprob[q]) {
            const ProblemWork &w = desc[pi];
            for (int64_t tn = 0; tn < w.tiles_n; ++tn)
                for (int64_t tm = 0; tm < w.tiles_m; ++tm) {
                    FusedTask t = w.t;
                    t.i0 = (int)(tm * w.tile_rows);
                    t.j0 = (int)(tn * w.tile_cols);
                    units.push_back(t);
                }
        }
    }
    qoff[mb::FUSED_QUEUES] = (int)units.size();

    // ---- grouped execution: one batched call per distinct shape -----------
    typedef std::tuple<int, int, int, int, int, int, int, int, int, uint64_t, uint64_t> Key;
    std::map<Key, std::vector<int64_t>> gmap;  // key -> problem indices
    for (int64_t di = 0; di < nd; ++di) {
        const mb_problem &q = problems[src[di]];
        uint64_t ab = 0, bb = 0;
        Key key;
        if (q.op == MB_OP_DGEMM) {
            memcpy(&ab, &q.alpha, 8);
            memcpy(&bb, &q.beta, 8);
            key = Key(0, tcode(q.transa), tcode(q.transb), q.m, q.n, q.k, q.lda, q.ldb, q.ldc,
                      ab, bb);
        } else if (q.op == MB_OP_DPOTRF) {
            key = Key(1, 0, 0, 0, q.n, 0, 0, 0, q.ldc, 0, 0);
        } else if (q.op == MB_OP_DPOTRF_ADJOINT) {
            key = Key(2, 0, 0, 0, q.n, 0, q.lda, q.ldb, q.ldc, 0, 0);
        } else {
            memcpy(&ab, &q.alpha, 8);
            memcpy(&bb, &q.beta, 8);
            key = Key(3, laset_code(q.uplo), 0, q.m, q.n, 0, 0, 0, q.ldc, ab, bb);
        }
        gmap[key].push_back(src[di]);
    }

    mb_plan *p = new (std::nothrow) mb_plan;
    if (!p) return MB_ERR_HIP;
    p->problems = count;
    p->units = total_units;
    p->idle = idle;
    p->cost_ns = total_ns;
    std::vector<const double *> hA(nd), hB(nd);
    std::vector<double *> hC(nd);
    std::vector<int *> hdst;
    int64_t off = 0;
    for (const auto &kv : gmap) {
        const Key &k = kv.first;
        PlanGroup g{};
        g.op = std::get<0>(k);  // the MB_OP_ codes
        g.off = off;
        g.count = (int64_t)kv.second.size();
        const mb_problem &q0 = problems[kv.second[0]];
        g.ta = std::get<1>(k); g.tb = std::get<2>(k);
        g.m = q0.m; g.n = q0.n; g.k = q0.k;
        g.lda = q0.lda; g.ldb = q0.ldb; g.ldc = q0.ldc;
        g.alpha = q0.alpha; g.beta = q0.beta;
        g.info_off = (int64_t)hdst.size();
        for (int64_t pi : kv.second) {
            const mb_problem &q = problems[pi];
            hA[off] = q.A; hB[off] = q.B; hC[off] = q.C;
            if (g.op == MB_OP_DPOTRF) hdst.push_back(q.info);
            ++off;
        }
        if (g.op == MB_OP_DGEMM) ++p->gemm_groups; else ++p->other_groups;
        // a batched call takes an int batch count: split larger groups
        for (int64_t start = 0; start < g.count; start += INT32_MAX) {
            PlanGroup part = g;
            part.off = g.off + start;
            part.count = std::min<int64_t>(INT32_MAX, g.count - start);
            part.info_off = g.info_off + (g.op == MB_OP_DPOTRF ? start : 0);
            p->groups.push_back(part);
        }
    }
    p->ninfo = (int64_t)hdst.size();

    // ---- device memory: one block ------------------------------------------
    Arena ar;
    const size_t o_units = ar.take(sizeof(FusedTask) * units.size());
    const size_t o_qoff = ar.take(sizeof(int) * qoff.size());
    const size_t o_ctr = ar.take(sizeof(int) * mb::FUSED_QUEUES * mb::FUSED_CTR_STRIDE);
    const size_t o_gA = ar.take(sizeof(void *) * (size_t)nd);
    const size_t o_gB = ar.take(sizeof(void *) * (size_t)nd);
    const size_t o_gC = ar.take(sizeof(void *) * (size_t)nd);
    const size_t o_info = ar.take(sizeof(int) * (size_t)p->ninfo);
    const size_t o_dst = ar.take(sizeof(void *) * (size_t)p->ninfo);

    hipError_t e = hipGetDevice(&p->device);
    if (e == hipSuccess) e = mb::fused_grid(&p->grid, &p->waves_per_cu);
    if (e == hipSuccess) e = hipMalloc((void **)&p->dmem, ar.size);
    if (e != hipSuccess) {
        release(p);
        return MB_ERR_HIP;
    }
    char *b = p->dmem;
    struct Up {
        size_t off;
        const void *src;
        size_t bytes;
    } ups[] = {
        {o_units, units.data(), sizeof(FusedTask) * units.size()},
        {o_qoff, qoff.data(), sizeof(int) * qoff.size()},
        {o_gA, hA.data(), sizeof(void *) * (size_t)nd},
        {o_gB, hB.data(), sizeof(void *) * (size_t)nd},
        {o_gC, hC.data(), sizeof(void *) * (size_t)nd},
        {o_dst, hdst.data(), sizeof(void *) * (size_t)p->ninfo},
    };
    for (const Up &u : ups)
        if (e == hipSuccess && u.bytes)
            e = hipMemcpy(b + u.off, u.src, u.bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemset(b + o_ctr, 0, sizeof(int) * mb::FUSED_QUEUES * mb::FUSED_CTR_STRIDE);
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        release(p);
        return MB_ERR_HIP;
    }
    p->args.tasks = reinterpret_cast<const FusedTask *>(b + o_units);
    p->args.qoff = reinterpret_cast<const int *>(b + o_qoff);
    p->args.counters = reinterpret_cast<int *>(b + o_ctr);
    p->args.potrf_waves = potrf_waves;
    p->gA = reinterpret_cast<const double **>(b + o_gA);
    p->gB = reinterpret_cast<const double **>(b + o_gB);
    p->gC = reinterpret_cast<double **>(b + o_gC);
    p->ginfo = reinterpret_cast<int *>(b + o_info);
    p->ginfo_dst = reinterpret_cast<int **>(b + o_dst);

    if (p->units > 0) {  // an empty plan has nothing to capture
        const int st = capture(p, run_fused, &p->fused_exec);
        if (st != MB_OK) {
            release(p);
            return st;
        }
    }
    *plan = p;
    return MB_OK;
}

int mb_plan_execute_mode(mb_plan *plan, int mode, hipStream_t stream)
{
    if (!plan) return -1;
    if (mode < MB_PLAN_FUSED_GRAPH || mode > MB_PLAN_GROUPED_GRAPH) return -2;
    DeviceGuard guard(plan->device);
    if (!guard.ok) return MB_ERR_HIP;
    switch (mode) {
    case MB_PLAN_FUSED_GRAPH:
        if (!plan->fused_exec)
            return MB_OK;
        return to_status(hipGraphLaunch(plan->fused_exec, stream));
    case MB_PLAN_FUSED:
        return run_fused(plan, stream);
    case MB_PLAN_GROUPED:
        return run_grouped(plan, stream);
    default:
        if (plan->groups.empty())
            return MB_OK;
        if (!plan->grouped_exec) {
            const int st = capture(plan, run_grouped, &plan->grouped_exec);
            if (st != MB_OK)
                return st;
        }
        return to_status(hipGraphLaunch(plan->grouped_exec, stream));
    }
}

int mb_plan_execute(mb_plan *plan, hipStream_t stream)
{
    return mb_plan_execute_mode(plan, MB_PLAN_FUSED_GRAPH, stream);
}

int mb_plan_stats(const mb_plan *plan, int64_t *out, int n)
{
    if (!plan) return -1;
    if (n > 0 && !out) return -2;
    const int64_t v[8] = {plan->problems, plan->units, plan->gemm_groups, plan->other_groups,
                          plan->grid, plan->waves_per_cu, plan->idle, (int64_t)plan->cost_ns};
    for (int i = 0; i < n && i < 8; ++i)
        out[i] = v[i];
    return MB_OK;
}

int mb_plan_destroy(mb_plan *plan)
{
    if (!plan) return MB_OK;
    DeviceGuard guard(plan->device);
    const hipError_t e = hipDeviceSynchronize();
    release(plan);
    return to_status(e);
}

}  // extern "C"
