// fused.hip -- one persistent kernel for an uneven batch of dgemm and dpotrf
// problems of mixed sizes.
//
// The paper switches between kernel variants by operand size (Sec. 2.4) but
// leaves batching aside; a batch whose problems all differ in shape cannot be
// served by per-shape launches without paying one launch per shape.  Here a
// plan (plan.hip) turns the batch into tasks -- one register tile of a dgemm,
// or one whole dpotrf -- sorted by estimated cost and dealt to one queue per
// XCD.  Every wave of the persistent grid is an independent worker: it claims
// the next task of its XCD's queue with one atomic increment, runs it, and
// moves on to the other queues once its own is empty, so the grid drains every
// queue whatever the dispatch order.
//
// The work is latency-bound per wave, so the loop keeps memory requests in
// flight at every step: the index of the task after next is claimed, and the
// next task is fetched, while the current one runs; inside a dgemm tile the operands of k chunk c + 1 are loaded
// while the matrix cores work on chunk c.
//
// dgemm tasks are TM x TN register tiles of 16 x 16 FP64 MFMA blocks computed
// straight from global memory (gemm_regtile.h); dpotrf and Cholesky-adjoint
// tasks run the batched kernels' per-wave routines.
#include "gemm_regtile.h"
#include "potrf_adj_wave.h"
#include "potrf_wave.h"

namespace mb {

// dlaset on columns [j0, j0 + FUSED_LASET_COLS) of the m x n matrix C; k is
// the part (0 strictly upper, 1 strictly lower, 2 all off-diagonal).
__device__ __forceinline__ void laset_task(const FusedTask &t, int lane)
{
    MB_GLOBAL double *C = global_ptr(t.C);
    const int j1 = min(t.j0 + FUSED_LASET_COLS, t.n);
    for (int j = t.j0; j < j1; ++j)
        for (int i = lane; i < t.m; i += 64) {
            const bool sel = i == j || (t.k == 0 ? i < j : (t.k == 1 ? i > j : true));
            if (sel)
                C[(size_t)i + (size_t)j * (size_t)t.ldc] = i == j ? t.beta : t.alpha;
        }
}

// Per-wave LDS of the dpotrf and Cholesky-adjoint tasks.
union TaskSmem {
    PotrfSmem potrf;
    AdjSmem adj;
};

// Run one task (kind is wave-uniform).
__device__ __forceinline__ void run_task(const FusedTask &t, TaskSmem &S, int lane)
{
#define MB_FUSED_CASE(KIND, TA, TB, TM, TN) \
    case KIND:                              \
        regtile<TA, TB, TM, TN>(t, lane);   \
        break;
    switch (t.kind) {
        MB_FUSED_CASE(0, false, false, 1, 1)
        MB_FUSED_CASE(1, false, true, 1, 1)
        MB_FUSED_CASE(2, true, false, 1, 1)
        MB_FUSED_CASE(3, true, true, 1, 1)
        MB_FUSED_CASE(4, false, false, 2, 1)
        MB_FUSED_CASE(5, false, true, 2, 1)
        MB_FUSED_CASE(6, true, false, 2, 1)
        MB_FUSED_CASE(7, true, true, 2, 1)
        MB_FUSED_CASE(8, false, false, 1, 2)
        MB_FUSED_CASE(9, false, true, 1, 2)
        MB_FUSED_CASE(10, true, false, 1, 2)
        MB_FUSED_CASE(11, true, true, 1, 2)
        MB_FUSED_CASE(12, false, false, 2, 2)
        MB_FUSED_CASE(13, false, true, 2, 2)
        MB_FUSED_CASE(14, true, false, 2, 2)
        MB_FUSED_CASE(15, true, true, 2, 2)
    case FUSED_POTRF: {
        // up to five tiles the factor stays in registers (potrf_regs, as the
        // plain launches; its 32-bit offsets need an instance below 4 GiB).
        // Larger orders take the plain-loop left-looking form.  The kernel
        // sits at its 256-register cap: this choice spills 20 bytes per lane,
        // the pipelined loops 92 and the register form also at six and seven
        // tiles 264 (both measured 1-2% slower on the uneven batch).
        const int nt = (t.n + 15) / 16;
        const bool regs = (uint64_t)t.ldc * (uint64_t)t.n * 8u < (1ull << 32);
        int info;
        if (regs && nt == 1)
            info = potrf_regs<1, false>(t.C, (uint32_t)t.ldc, t.n, S.potrf, lane);
        else if (regs && nt == 2)
            info = potrf_regs<2, false>(t.C, (uint32_t)t.ldc, t.n, S.potrf, lane);
        else if (regs && nt == 3)
            info = potrf_regs<3, false>(t.C, (uint32_t)t.ldc, t.n, S.potrf, lane);
        else if (regs && nt == 4)
            info = potrf_regs<4, false>(t.C, (uint32_t)t.ldc, t.n, S.potrf, lane);
        else if (regs && nt == 5)
            info = potrf_regs<5, false>(t.C, (uint32_t)t.ldc, t.n, S.potrf, lane);
        else
            info = potrf_wave<true, 2, false>(t.C, (size_t)t.ldc, t.n, nt, S.potrf, lane);
        if (lane == 0)
            *global_ptr(t.info) = info;
        break;
    }
    case FUSED_POTRF_ADJ:
        potrf_adj_wave(t.A, (size_t)t.lda, t.B, (size_t)t.ldb, t.C, (size_t)t.ldc, t.n,
                       (t.n + 15) / 16, S.adj, lane);
        break;
    case FUSED_LASET:
        laset_task(t, lane);
        break;
    default:
        break;
    }
#undef MB_FUSED_CASE
}

constexpr int FUSED_WAVES = kFusedWaves;  // waves per workgroup, each an independent worker

// Claim the next task of a queue: one atomic per wave, issued by lane 0.  The
// result stays in lane 0's register until claim_get reads it, so the atomic's
// latency overlaps whatever the wave does in between.
__device__ __forceinline__ int claim_issue(int *ctr, int lane)
{
    int v = 0;
    if (lane == 0)
        v = atomicAdd(ctr, 1);
    return v;
}
__device__ __forceinline__ int claim_get(int v) { return __builtin_amdgcn_readfirstlane(v); }

// A task travels as one vector register: lane w < 24 holds dword w of the
// 96-byte record (one coalesced load), and the fields are read out with
// readlane when the task starts.  Two tasks in flight then cost two vector
// registers instead of 48 scalar ones.
__device__ __forceinline__ int task_fetch(const FusedTask *tasks, int idx, int lane)
{
    const MB_GLOBAL int *p = (const MB_GLOBAL int *)global_ptr(tasks + idx);
    return lane < 24 ? p[lane] : 0;
}
__device__ __forceinline__ uint32_t word(int v, int w)
{
    return (uint32_t)__builtin_amdgcn_readlane(v, w);
}
__device__ __forceinline__ uint64_t dword2(int v, int w)
{
    return (uint64_t)word(v, w) | ((uint64_t)word(v, w + 1) << 32);
}
__device__ __forceinline__ FusedTask task_unpack(int v)
{
    FusedTask t;
    t.A = (const double *)dword2(v, 0);
    t.B = (const double *)dword2(v, 2);
    t.C = (double *)dword2(v, 4);
    t.info = (int *)dword2(v, 6);
    t.alpha = __builtin_bit_cast(double, dword2(v, 8));
    t.beta = __builtin_bit_cast(double, dword2(v, 10));
    t.m = (int)word(v, 12);
    t.n = (int)word(v, 13);
    t.k = (int)word(v, 14);
    t.lda = (int)word(v, 15);
    t.ldb = (int)word(v, 16);
    t.ldc = (int)word(v, 17);
    t.kind = (int)word(v, 18);
    t.i0 = (int)word(v, 19);
    t.j0 = (int)word(v, 20);
    return t;
}

// Queue 2 x + c holds the class-c tasks (c = 0 dpotrf, 1 dgemm) meant for
// XCD x.  dpotrf tasks are long and latency-bound, dgemm tiles short and
// bandwidth-bound: the first potrf_waves waves of every workgroup start on
// the dpotrf class and the others on the dgemm class, so that both kinds run
// side by side instead of one phase after the other; a wave whose class is
// drained everywhere moves on to the other class.
__global__ __launch_bounds__(FUSED_WAVES * 64) __attribute__((amdgpu_waves_per_eu(2))) void fused_kernel(const FusedTask *tasks,
                                                                 const int *qoff, int *counters,
                                                                 int potrf_waves)
{
    __shared__ TaskSmem smem[FUSED_WAVES];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    TaskSmem &S = smem[wave];
    const int home = (int)(blockIdx.x % FUSED_XCDS);  // the XCD this workgroup runs on
    const int first = wave < potrf_waves ? 0 : 1;
    for (int pass = 0; pass < FUSED_CLASSES; ++pass) {
        const int cls = pass == 0 ? first : 1 - first;
        for (int xi = 0; xi < FUSED_XCDS; ++xi) {
            const int q = FUSED_CLASSES * ((home + xi) % FUSED_XCDS) + cls;
            const int beg = qoff[q], cnt = qoff[q + 1] - beg;
            int *ctr = counters + q * FUSED_CTR_STRIDE;
            int u = claim_get(claim_issue(ctr, lane));
            if (u >= cnt)
                continue;
            int cur = task_fetch(tasks, beg + u, lane);
            u = claim_get(claim_issue(ctr, lane));
            for (;;) {
                // fetch the next task and claim the one after it; both
                // complete while the current task runs
                const bool more = u < cnt;
                int nxt = 0, raw = 0;
                if (more) {
                    nxt = task_fetch(tasks, beg + u, lane);
                    raw = claim_issue(ctr, lane);
                }
                run_task(task_unpack(cur), S, lane);
                if (!more)
                    break;
                cur = nxt;
                u = claim_get(raw);
            }
        }
    }
}

// Zero the queue counters (a kernel rather than a memset, so that the reset
// can sit in a captured graph).
__global__ void fused_reset_kernel(int *counters)
{
    const int q = threadIdx.x;
    if (q < FUSED_QUEUES)
        counters[q * FUSED_CTR_STRIDE] = 0;
}

// dst[i][0] = src[i]: per-problem info words from a contiguous batch result.
__global__ void scatter_info_kernel(const int *src, int *const *dst, int count)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count)
        *global_ptr(dst[i]) = src[i];
}

hipError_t fused_grid(int *grid, int *waves_per_cu)
{
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fused_kernel, FUSED_WAVES * 64, 0);
    if (e != hipSuccess)
        return e;
    if (per_cu < 1)
        per_cu = 1;
    *grid = cus * per_cu;
    if (waves_per_cu)
        *waves_per_cu = per_cu * FUSED_WAVES;
    return hipSuccess;
}

hipError_t launch_fused(const FusedArgs &a, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(fused_reset_kernel, dim3(1), dim3(64), 0, s, a.counters);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(fused_kernel, dim3((unsigned)grid), dim3(FUSED_WAVES * 64), 0, s, a.tasks,
                       a.qoff, a.counters, a.potrf_waves);
    return hipGetLastError();
}

hipError_t launch_scatter_info(const int *src, int *const *dst, int count, hipStream_t s)
{
    if (count <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(scatter_info_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s,
                       src, dst, count);
    return hipGetLastError();
}

}  // namespace mb
