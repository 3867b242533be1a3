// potrf.hip -- batched lower Cholesky factorization (dpotrf 'L') on gfx950.
//
// One launch factors the whole batch, one wave per instance (potrf_wave.h),
// several instances per workgroup; the tile count is a template parameter so
// that every loop bound is a constant.
#include "potrf_wave.h"

namespace mb {

template <int NT, int IPB>
__global__ __launch_bounds__(IPB * 64) __attribute__((amdgpu_waves_per_eu(2))) void potrf_lower_kernel(PotrfArgs p)
{
    // orders from 8 tiles keep their first KC pivot steps per pair in LDS
    // (2 KC tiles of 2 KB per wave: 64 KB for four waves, two workgroups per
    // CU -- the two waves per SIMD their registers allow)
    constexpr int KC = NT >= 8 ? 4 : 0;
    __shared__ PotrfSmem smem[IPB];
    __shared__ double pcache[IPB][KC > 0 ? 2 * KC * 256 : 1];
    const int lane = threadIdx.x & 63;
    const int inst = threadIdx.x >> 6;
    const int64_t b = (int64_t)blockIdx.x * IPB + inst;
    if (b >= p.batch)
        return;  // each wave is its own instance: nothing to synchronise with
    double *A = inst_ptr(p.A, p.Aarr, p.sA, b);
    // the pipelined update loops (with the LDS pivot cache) measured 3-12%
    // faster than the plain ones from 8 tiles (n = 128..240) and faster at
    // n = 256..304; below 8 tiles the plain loops keep more waves per SIMD
    constexpr bool PIPE = NT >= 8;
    // panel rows per group: more rows share each load of the pivot columns'
    // tiles (fewer re-reads) at more registers -- 3 with the pipelined loops
    // (4 would spill there), 2 below 8 tiles
    constexpr int G = PIPE ? 3 : 2;
    // first panel rows updated inside the diagonal-block loop (they share its
    // pivot tiles): three rows with the pipelined loops (4.8% faster at
    // n = 256), two where three would spill (odd tile counts, and below 12
    // tiles); the plain-loop orders keep none -- there the extra registers
    // cost a wave per SIMD
    constexpr int G1 = PIPE ? ((NT % 2 == 1 || NT < 12) ? 2 : 3) : 0;
    const int info = potrf_wave<true, G, PIPE, G1, KC>(A, (size_t)p.lda, p.n, NT, smem[inst],
                                                                lane, pcache[inst]);
    if (lane == 0)
        p.info[b] = info;
}

__global__ void fill_info_kernel(int *info, int batch)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < batch)
        info[i] = 0;
}

template <int NT, int IPB>
static hipError_t launch_potrf_t(const PotrfArgs &a, hipStream_t s)
{
    const int64_t blocks = ((int64_t)a.batch + IPB - 1) / IPB;
    hipLaunchKernelGGL((potrf_lower_kernel<NT, IPB>), dim3((unsigned)blocks), dim3(64 * IPB), 0, s,
                       a);
    return hipGetLastError();
}

hipError_t launch_potrf_lower(const PotrfArgs &a, hipStream_t s)
{
    const int nt = (a.n + 15) / 16;
    switch (nt) {
    case 1: return launch_potrf_t<1, 4>(a, s);
    case 2: return launch_potrf_t<2, 4>(a, s);
    case 3: return launch_potrf_t<3, 4>(a, s);
    case 4: return launch_potrf_t<4, 4>(a, s);
    case 5: return launch_potrf_t<5, 4>(a, s);
    case 6: return launch_potrf_t<6, 4>(a, s);
    case 7: return launch_potrf_t<7, 4>(a, s);
    case 8: return launch_potrf_t<8, 4>(a, s);
    case 9: return launch_potrf_t<9, 4>(a, s);
    case 10: return launch_potrf_t<10, 4>(a, s);
    case 11: return launch_potrf_t<11, 4>(a, s);
    case 12: return launch_potrf_t<12, 4>(a, s);
    case 13: return launch_potrf_t<13, 4>(a, s);
    case 14: return launch_potrf_t<14, 4>(a, s);
    case 15: return launch_potrf_t<15, 4>(a, s);
    case 16: return launch_potrf_t<16, 4>(a, s);
    case 17: return launch_potrf_t<17, 4>(a, s);
    case 18: return launch_potrf_t<18, 4>(a, s);
    case 19: return launch_potrf_t<19, 4>(a, s);
    default: return hipErrorInvalidValue;
    }
}

const char *potrf_kernel_name(int n)
{
    static const char *names[20] = {
        "potrf_fill_info", "potrf_nt1", "potrf_nt2", "potrf_nt3", "potrf_nt4", "potrf_nt5",
        "potrf_nt6", "potrf_nt7", "potrf_nt8", "potrf_nt9", "potrf_nt10", "potrf_nt11",
        "potrf_nt12", "potrf_nt13", "potrf_nt14", "potrf_nt15", "potrf_nt16", "potrf_nt17",
        "potrf_nt18", "potrf_nt19"};
    const int nt = (n + 15) / 16;
    return (nt >= 0 && nt <= 19) ? names[nt] : "unsupported";
}

hipError_t launch_fill_info(int *info, int batch, hipStream_t s)
{
    const int64_t blocks = ((int64_t)batch + 255) / 256;
    hipLaunchKernelGGL(fill_info_kernel, dim3((unsigned)blocks), dim3(256), 0, s, info, batch);
    return hipGetLastError();
}

}  // namespace mb
