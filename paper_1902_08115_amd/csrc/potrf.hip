// potrf.hip -- batched lower Cholesky factorization (dpotrf 'L') on gfx950.
//
// One launch factors the whole batch, one wave per instance (potrf_wave.h),
// several instances per workgroup; the tile count is a template parameter so
// that every loop bound is a constant.
#include "potrf_wave.h"

#include <utility>

#ifndef POTRF_ROWS_IPW
#define POTRF_ROWS_IPW 4
#endif

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

// Orders of a few tiles: the factor in registers (potrf_regs).  Up to four
// tiles the kernel fits in 128 registers, four waves per SIMD: a batch of
// 4096 then runs in one round on the 1024 SIMDs instead of leaving a quarter
// of it for a second round of single waves.  FULL: the order is 16 NT.  At 8
// tiles only the FULL form is used (one more register set would halve the
// waves per SIMD).
template <int NT, int IPB, bool FULL>
__global__ __launch_bounds__(IPB * 64) __attribute__((amdgpu_waves_per_eu(NT <= 4 ? 4 : 1))) void potrf_regs_kernel(PotrfArgs p)
{
    __shared__ PotrfSmem smem[IPB];
    const int lane = threadIdx.x & 63;
    // the instance is uniform over the wave: its base address stays scalar
    const int inst = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t b = (int64_t)blockIdx.x * IPB + inst;
    if (b >= p.batch)
        return;
    double *A = inst_ptr(p.A, p.Aarr, p.sA, b);
    const int info = potrf_regs<NT, FULL>(A, (uint32_t)p.lda, p.n, smem[inst], lane);
    if (lane == 0)
        p.info[b] = info;
}

// ---- orders up to 32: four instances per wave, whole rows in lanes ----------
// (the order 32 itself runs the register kernel unless an instance spans 4 GiB)
// For small orders what costs is the chain of N elimination steps, not
// arithmetic.  Lane (g, i) of a wave holds rows i and, from order 17, i + 16
// of instance 4w + g whole (entries right of the diagonal read from the lower
// triangle, by symmetry), so the pivot row of step C -- row C, in lane C % 16
// of the lane's own group of 16 -- reaches the group by one DPP broadcast per
// entry, each broadcast serves both rows of a lane, and each instruction
// serves four instances.  The order N is a template parameter: exactly N
// steps, with every register index a constant.  No matrix cores, no LDS.

// Elimination step C on rows i + 16 s (s < S) held whole in R[s][0..N):
// rows below C get l_kC = R[C] / sqrt(piv) and lose (R[C] / piv) times the
// pivot row right of C; row C itself becomes [.., sqrt(piv), 0 ..] (the
// update clears the entries right of its diagonal); rows above C have
// R[C] = 0 and do not change.  A step at a pivot that is not positive, or
// after one, changes nothing (zero multiplier; fc keeps the first failing
// column).  Branch-free: the four instances of a wave fail independently.
template <int N, int S, int C>
__device__ __forceinline__ void rows_step(double (&R)[S][N], int &fc)
{
    constexpr int CL = C % 16, CS = C / 16;
    const double piv = row_bcast<CL>(R[CS][C]);
    const bool live = fc == N;
    const bool act = live && piv > 0.0;
    fc = (live && !act) ? C : fc;
    const double rs = rsqrt_nr(act ? piv : 1.0);
    double l[S], lr[S];
#pragma unroll
    for (int k = 0; k < S; ++k) {
        l[k] = R[k][C] * rs;
        lr[k] = act ? l[k] * rs : 0.0;
    }
    // all broadcasts first, each into its own register: they are independent,
    // and a shared temporary would make every broadcast wait for the fma
    // before it
    double pr[N];
#pragma unroll
    for (int q = C + 1; q < N; ++q)
        pr[q] = row_bcast<CL>(R[CS][q]);
#pragma unroll
    for (int q = C + 1; q < N; ++q) {
#pragma unroll
        for (int k = 0; k < S; ++k)
            R[k][q] = fma(-lr[k], pr[q], R[k][q]);
    }
#pragma unroll
    for (int k = 0; k < S; ++k)
        R[k][C] = act ? l[k] : R[k][C];
}

template <int N, int S, int... C>
__device__ __forceinline__ void rows_steps(double (&R)[S][N], int &fc,
                                           std::integer_sequence<int, C...>)
{
    (rows_step<N, S, C>(R, fc), ...);
}

template <int N, int IPW>
__global__ __launch_bounds__(256) void potrf_rows_kernel(PotrfArgs p)
{
    constexpr int S = (N + 15) / 16;  // rows per lane
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = lane & 15, g = lane >> 4;
    // IPW instances per wave: groups g >= IPW repeat group g % IPW and store
    // nothing (fewer instances per wave: more waves to hide memory latency)
    const int64_t b = ((int64_t)blockIdx.x * 4 + wave) * IPW + (g % IPW);
    // lanes of a missing instance, and rows past N, compute on zero rows
    // (their results are never stored), so every lane takes part in the
    // broadcasts
    const bool inst = b < p.batch;
    const MB_GLOBAL double *A =
        global_ptr((const double *)inst_ptr(p.A, p.Aarr, p.sA, inst ? b : 0));
    const size_t lda = (size_t)p.lda;
    // every load is unconditional, from an address inside instance b (or
    // instance 0 for a missing one; rows past N read row N-1), and only the
    // value is selected: a load under a branch makes the compiler wait for it
    // before the next one is issued
    double R[S][N];
#pragma unroll
    for (int k = 0; k < S; ++k) {
        const int ii = i + 16 * k;
        const bool row = inst && ii < N;
        const size_t ic = (size_t)min(ii, N - 1);
#pragma unroll
        for (int q = 0; q < N; ++q) {
            const double v = A[(size_t)q <= ic ? ic + (size_t)q * lda : (size_t)q + ic * lda];
            R[k][q] = row ? v : 0.0;
        }
    }
    int fc = N;
    rows_steps<N, S>(R, fc, std::make_integer_sequence<int, N>{});
    if (inst && g < IPW) {
        MB_GLOBAL double *Aw = global_ptr(inst_ptr(p.A, p.Aarr, p.sA, b));
#pragma unroll
        for (int k = 0; k < S; ++k) {
            const int ii = i + 16 * k;
#pragma unroll
            for (int q = 0; q < N; ++q)
                if (ii < N && q <= ii && q < fc)
                    Aw[(size_t)ii + (size_t)q * lda] = R[k][q];
        }
        if (i == 0)
            p.info[b] = fc == N ? 0 : fc + 1;
    }
}

template <int N>
static hipError_t launch_potrf_rows(const PotrfArgs &a, hipStream_t s)
{
    constexpr int IPW = POTRF_ROWS_IPW;
    const int64_t blocks = ((int64_t)a.batch + 4 * IPW - 1) / (4 * IPW);  // four waves per workgroup
    hipLaunchKernelGGL((potrf_rows_kernel<N, IPW>), dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <int... N>
static hipError_t launch_potrf_rows_n(int n, const PotrfArgs &a, hipStream_t s,
                                      std::integer_sequence<int, N...>)
{
    hipError_t e = hipErrorInvalidValue;
    (void)((n == N + 1 ? (e = launch_potrf_rows<N + 1>(a, s), true) : false) || ...);
    return e;
}

__global__ void fill_info_kernel(int *info, int batch)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < batch)
        info[i] = 0;
}

template <int NT, int IPB>
static hipError_t launch_potrf_regs(const PotrfArgs &a, hipStream_t s)
{
    const int64_t blocks = ((int64_t)a.batch + IPB - 1) / IPB;
    if (a.n == 16 * NT)
        hipLaunchKernelGGL((potrf_regs_kernel<NT, IPB, true>), dim3((unsigned)blocks),
                           dim3(64 * IPB), 0, s, a);
    else
        hipLaunchKernelGGL((potrf_regs_kernel<NT, IPB, false>), dim3((unsigned)blocks),
                           dim3(64 * IPB), 0, s, a);
    return hipGetLastError();
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
    // at the order 32 the two full tiles in registers beat the rows kernel
    // (17.4 against 18.8 us for 4096 instances); at 17..31 and at 16 the rows
    // kernel is faster
    if (a.n == 32 && (uint64_t)a.lda * (uint64_t)a.n * 8u < (1ull << 32))
        return launch_potrf_regs<2, 1>(a, s);
    if (a.n <= POTRF_ROWS_MAX_N)
        return launch_potrf_rows_n(a.n, a, s, std::make_integer_sequence<int, POTRF_ROWS_MAX_N>{});
    const int nt = (a.n + 15) / 16;
    // the register-resident kernel up to 7 tiles, and at 8 tiles for the
    // order 128 (two waves per SIMD; a partial eighth tile needs one more
    // register set and one wave per SIMD, where it measured slower than
    // potrf_lower); it addresses an instance with 32-bit offsets
    const bool regs = (nt <= 7 || a.n == 128) &&
                      (uint64_t)a.lda * (uint64_t)a.n * 8u < (1ull << 32);
    // one instance (one wave) per workgroup: 2-4% faster than four at the
    // orders 64, 96 and 128, the same elsewhere
    if (regs) {
        switch (nt) {
        case 3: return launch_potrf_regs<3, 1>(a, s);
        case 4: return launch_potrf_regs<4, 1>(a, s);
        case 5: return launch_potrf_regs<5, 1>(a, s);
        case 6: return launch_potrf_regs<6, 1>(a, s);
        case 7: return launch_potrf_regs<7, 1>(a, s);
        case 8: return launch_potrf_regs<8, 1>(a, s);
        default: break;
        }
    }
    switch (nt) {
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
        "potrf_fill_info", "potrf_rows", "potrf_rows2", "potrf_nt3", "potrf_nt4", "potrf_nt5",
        "potrf_nt6", "potrf_nt7", "potrf_nt8", "potrf_nt9", "potrf_nt10", "potrf_nt11",
        "potrf_nt12", "potrf_nt13", "potrf_nt14", "potrf_nt15", "potrf_nt16", "potrf_nt17",
        "potrf_nt18", "potrf_nt19"};
    if (n == 32)
        return "potrf_nt2";  // the register kernel (the rows kernel below it)
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
