// gemm_regtile.hip -- batched dgemm in register tiles read straight from
// global memory (gemm_regtile.h): one wave per TM x TN tile of 16 x 16 MFMA
// blocks, four waves per workgroup, the tiles of one instance consecutive.
// The kernel family for thin, flat and small results, where a workgroup
// tile would mostly compute padding and staging in LDS cannot pay off.
#include "gemm_regtile.h"

namespace mb {

constexpr int REG_WAVES = 4;

template <bool TA, bool TB, int TM, int TN>
__global__ __launch_bounds__(REG_WAVES * 64) void gemm_regtile_kernel(GemmArgs p, int tiles_m,
                                                                      int tiles_n, int64_t b0)
{
    const int lane = threadIdx.x & 63;
    const int64_t per = (int64_t)tiles_m * tiles_n;
    const int64_t w = (int64_t)blockIdx.x * REG_WAVES + (threadIdx.x >> 6);
    const int64_t b = b0 + w / per;
    if (b >= p.batch)
        return;
    const int t = (int)(w % per);
    FusedTask task{};
    task.A = inst_ptr(p.A, p.Aarr, p.sA, b);
    task.B = inst_ptr(p.B, p.Barr, p.sB, b);
    task.C = inst_ptr(p.C, p.Carr, p.sC, b);
    task.alpha = p.alpha;
    task.beta = p.beta;
    task.m = p.m;
    task.n = p.n;
    task.k = p.k;
    task.lda = p.lda;
    task.ldb = p.ldb;
    task.ldc = p.ldc;
    task.i0 = (t % tiles_m) * 16 * TM;
    task.j0 = (t / tiles_m) * 16 * TN;
    regtile<TA, TB, TM, TN>(task, lane);
}

template <bool TA, bool TB, int TM, int TN>
static hipError_t launch_t(const GemmArgs &a, hipStream_t s)
{
    const int tiles_m = (a.m + 16 * TM - 1) / (16 * TM);
    const int tiles_n = (a.n + 16 * TN - 1) / (16 * TN);
    const int64_t per = (int64_t)tiles_m * tiles_n;
    // at most 2^30 workgroups per launch; larger batches go in slices
    const int64_t max_inst = std::max<int64_t>(1, ((int64_t)1 << 30) * REG_WAVES / per);
    for (int64_t b0 = 0; b0 < a.batch; b0 += max_inst) {
        const int64_t cnt = std::min<int64_t>(max_inst, a.batch - b0);
        const int64_t blocks = (cnt * per + REG_WAVES - 1) / REG_WAVES;
        GemmArgs sl = a;
        sl.batch = (int)std::min<int64_t>(a.batch, b0 + cnt);
        hipLaunchKernelGGL((gemm_regtile_kernel<TA, TB, TM, TN>), dim3((unsigned)blocks),
                           dim3(REG_WAVES * 64), 0, s, sl, tiles_m, tiles_n, b0);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

template <bool TA, bool TB>
static hipError_t launch_tt(int tm, int tn, const GemmArgs &a, hipStream_t s)
{
    if (tm == 1 && tn == 1) return launch_t<TA, TB, 1, 1>(a, s);
    if (tm == 2 && tn == 1) return launch_t<TA, TB, 2, 1>(a, s);
    if (tm == 1 && tn == 2) return launch_t<TA, TB, 1, 2>(a, s);
    return launch_t<TA, TB, 2, 2>(a, s);
}

hipError_t launch_gemm_regtile(bool ta, bool tb, int tm, int tn, const GemmArgs &a,
                               hipStream_t s)
{
    if (ta)
        return tb ? launch_tt<true, true>(tm, tn, a, s) : launch_tt<true, false>(tm, tn, a, s);
    return tb ? launch_tt<false, true>(tm, tn, a, s) : launch_tt<false, false>(tm, tn, a, s);
}

}  // namespace mb
