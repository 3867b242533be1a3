// gemm_packed.hip -- LDS-staged ("packed") batched dgemm on FP64 matrix cores.
//
// The analogue of the paper's algorithmic variants 'C'/'B' (Sec. 2.2, Table 1):
// the factors are packed, k-panel by k-panel, into an on-chip buffer whose
// layout suits the compute kernel, transposing while packing so that every
// trans case runs the same inner kernel (Sec. 2.2 "transposed while packed";
// Sec. 3.2.1: one shared inner kernel for all variants).  On gfx950 the buffer
// is LDS and the inner kernel is a v_mfma_f64_16x16x4 rank-4 update.
//
// Packed layout: for a BK x BM slice of op(A) and a BK x BN slice of op(B),
// element (q, i) lives at As[q*SA + i] and (q, j) at Bs[q*SB + j] (k-major,
// the "nt" arrangement of both factors).  The MFMA is issued with op(B) as its
// left operand and op(A) as its right one, so it accumulates C^T tiles whose
// result registers hold, in lane l, C[16*ti + l%16][16*tj + 4*(l/16) + r]:
// consecutive lanes own consecutive rows, and the epilogue reads and writes C
// in 128-byte column segments.
//
// Global->LDS staging maps consecutive threads to consecutive addresses of
// the operand as stored (rows for 'N' A / 'T' B, k for 'T' A / 'N' B), and the
// next k-panel is prefetched into registers while the current one is consumed.
// Two launch shapes share the code:
//   * SMALL (IPB > 1): each wave owns one whole instance (C up to 16*TM x 16*TN),
//     IPB instances per workgroup, wave-local synchronisation only;
//   * TILED (IPB == 1): WM x WN waves cooperate on a BM x BN tile of one
//     instance, workgroup barriers, XCD-aware tile order.
#include "mb_internal.h"

namespace mb {

template <bool TA, bool TB, int WM, int WN, int TM, int TN, int IPB>
struct PackedCfg {
    static constexpr int BM = WM * TM * 16;
    static constexpr int BN = WN * TN * 16;
    static constexpr int BK = 16;
    static constexpr int SA = BM + 1;  // odd row stride: transposed stores hit distinct banks
    static constexpr int SB = BN + 1;
    static constexpr int NTHR = WM * WN * 64;  // threads per instance group
    static constexpr int EA = BM * BK / NTHR;  // staged elements per thread
    static constexpr int EB = BN * BK / NTHR;
    static_assert(EA * NTHR == BM * BK && EB * NTHR == BN * BK, "tile/threads mismatch");
    static_assert(IPB == 1 || (WM == 1 && WN == 1), "SMALL shape is one wave per instance");
};

template <class Cfg, bool TA>
__device__ __forceinline__ void load_a(double (&ra)[Cfg::EA], const double *A, size_t lda, int m,
                                       int k, int i0, int kb, int tid)
{
#pragma unroll
    for (int u = 0; u < Cfg::EA; ++u) {
        const int e = tid + u * Cfg::NTHR;
        int i, q;
        if (!TA) {  // A[i + q*lda]: consecutive threads along i
            i = e % Cfg::BM;
            q = e / Cfg::BM;
        } else {  // A[q + i*lda]: consecutive threads along q
            q = e % Cfg::BK;
            i = e / Cfg::BK;
        }
        const int gi = i0 + i, gq = kb + q;
        double v = 0.0;
        if (gi < m && gq < k)
            v = TA ? A[(size_t)gq + (size_t)gi * lda] : A[(size_t)gi + (size_t)gq * lda];
        ra[u] = v;
    }
}

template <class Cfg, bool TA>
__device__ __forceinline__ void store_a(const double (&ra)[Cfg::EA], double *As, int tid)
{
#pragma unroll
    for (int u = 0; u < Cfg::EA; ++u) {
        const int e = tid + u * Cfg::NTHR;
        int i, q;
        if (!TA) {
            i = e % Cfg::BM;
            q = e / Cfg::BM;
        } else {
            q = e % Cfg::BK;
            i = e / Cfg::BK;
        }
        As[q * Cfg::SA + i] = ra[u];
    }
}

template <class Cfg, bool TB>
__device__ __forceinline__ void load_b(double (&rb)[Cfg::EB], const double *B, size_t ldb, int n,
                                       int k, int j0, int kb, int tid)
{
#pragma unroll
    for (int u = 0; u < Cfg::EB; ++u) {
        const int e = tid + u * Cfg::NTHR;
        int j, q;
        if (TB) {  // B[j + q*ldb]: consecutive threads along j
            j = e % Cfg::BN;
            q = e / Cfg::BN;
        } else {  // B[q + j*ldb]: consecutive threads along q
            q = e % Cfg::BK;
            j = e / Cfg::BK;
        }
        const int gj = j0 + j, gq = kb + q;
        double v = 0.0;
        if (gj < n && gq < k)
            v = TB ? B[(size_t)gj + (size_t)gq * ldb] : B[(size_t)gq + (size_t)gj * ldb];
        rb[u] = v;
    }
}

template <class Cfg, bool TB>
__device__ __forceinline__ void store_b(const double (&rb)[Cfg::EB], double *Bs, int tid)
{
#pragma unroll
    for (int u = 0; u < Cfg::EB; ++u) {
        const int e = tid + u * Cfg::NTHR;
        int j, q;
        if (TB) {
            j = e % Cfg::BN;
            q = e / Cfg::BN;
        } else {
            q = e % Cfg::BK;
            j = e / Cfg::BK;
        }
        Bs[q * Cfg::SB + j] = rb[u];
    }
}

template <bool TA, bool TB, int WM, int WN, int TM, int TN, int IPB>
__global__ __launch_bounds__(WM *WN *IPB * 64) void gemm_packed_kernel(GemmArgs p, int tiles_m,
                                                                       int tiles_n)
{
    using Cfg = PackedCfg<TA, TB, WM, WN, TM, TN, IPB>;
    constexpr bool WAVE_ONLY = (IPB > 1);
    __shared__ double smem[IPB][Cfg::BK * Cfg::SA + Cfg::BK * Cfg::SB];

    const int lane = threadIdx.x & 63;
    int grp, tid;  // instance group within the block, thread id within it
    int64_t b;
    int tm, tn;
    if constexpr (WAVE_ONLY) {
        grp = threadIdx.x >> 6;
        tid = lane;
        b = (int64_t)blockIdx.x * IPB + grp;
        if (b >= p.batch)
            return;
        tm = tn = 0;
    } else {
        grp = 0;
        tid = threadIdx.x;
        const int bid = xcd_remap(blockIdx.x, gridDim.x);
        const int per_inst = tiles_m * tiles_n;
        b = bid / per_inst;
        const int rem = bid - (int)b * per_inst;
        tn = rem / tiles_m;
        tm = rem - tn * tiles_m;
    }
    double *As = &smem[grp][0];
    double *Bs = &smem[grp][Cfg::BK * Cfg::SA];

    const double *A = inst_ptr(p.A, p.Aarr, p.sA, b);
    const double *B = inst_ptr(p.B, p.Barr, p.sB, b);
    double *C = inst_ptr(p.C, p.Carr, p.sC, b);
    const size_t lda = (size_t)p.lda, ldb = (size_t)p.ldb, ldc = (size_t)p.ldc;
    const int m = p.m, n = p.n, k = p.k;
    const int i0 = tm * Cfg::BM, j0 = tn * Cfg::BN;

    const int wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;
    const int lr = lane & 15, lg = lane >> 4;

    d4 acc[TM][TN];
#pragma unroll
    for (int ti = 0; ti < TM; ++ti)
#pragma unroll
        for (int tj = 0; tj < TN; ++tj)
            acc[ti][tj] = d4{0.0, 0.0, 0.0, 0.0};

    double ra[Cfg::EA], rb[Cfg::EB];
    load_a<Cfg, TA>(ra, A, lda, m, k, i0, 0, tid);
    load_b<Cfg, TB>(rb, B, ldb, n, k, j0, 0, tid);

    for (int kb = 0; kb < k; kb += Cfg::BK) {
        store_a<Cfg, TA>(ra, As, tid);
        store_b<Cfg, TB>(rb, Bs, tid);
        group_sync<WAVE_ONLY>();
        if (kb + Cfg::BK < k) {
            load_a<Cfg, TA>(ra, A, lda, m, k, i0, kb + Cfg::BK, tid);
            load_b<Cfg, TB>(rb, B, ldb, n, k, j0, kb + Cfg::BK, tid);
        }
#pragma unroll
        for (int s = 0; s < Cfg::BK / 4; ++s) {
            const int q = 4 * s + lg;
            double fa[TM], fb[TN];
#pragma unroll
            for (int ti = 0; ti < TM; ++ti)
                fa[ti] = As[q * Cfg::SA + (wm * TM + ti) * 16 + lr];
#pragma unroll
            for (int tj = 0; tj < TN; ++tj)
                fb[tj] = Bs[q * Cfg::SB + (wn * TN + tj) * 16 + lr];
#pragma unroll
            for (int ti = 0; ti < TM; ++ti)
#pragma unroll
                for (int tj = 0; tj < TN; ++tj)
                    acc[ti][tj] = mfma16(fb[tj], fa[ti], acc[ti][tj]);
        }
        group_sync<WAVE_ONLY>();
    }

    // epilogue: C <= alpha*acc + beta*C, masked to the m x n window
    const double alpha = p.alpha, beta = p.beta;
#pragma unroll
    for (int ti = 0; ti < TM; ++ti) {
        const int gi = i0 + (wm * TM + ti) * 16 + lr;
#pragma unroll
        for (int tj = 0; tj < TN; ++tj) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gj = j0 + (wn * TN + tj) * 16 + lg + 4 * r;
                if (gi < m && gj < n) {
                    double *c = C + (size_t)gi + (size_t)gj * ldc;
                    const double v = acc[ti][tj][r];
                    *c = (beta == 0.0) ? alpha * v : fma(alpha, v, beta * (*c));
                }
            }
        }
    }
}

template <bool TA, bool TB, int WM, int WN, int TM, int TN, int IPB>
static hipError_t launch_cfg(const GemmArgs &a, hipStream_t s)
{
    using Cfg = PackedCfg<TA, TB, WM, WN, TM, TN, IPB>;
    if constexpr (IPB > 1) {
        const int64_t blocks = ((int64_t)a.batch + IPB - 1) / IPB;
        hipLaunchKernelGGL((gemm_packed_kernel<TA, TB, WM, WN, TM, TN, IPB>), dim3((unsigned)blocks),
                           dim3(64 * IPB), 0, s, a, 1, 1);
    } else {
        const int tiles_m = (a.m + Cfg::BM - 1) / Cfg::BM;
        const int tiles_n = (a.n + Cfg::BN - 1) / Cfg::BN;
        const int64_t blocks = (int64_t)a.batch * tiles_m * tiles_n;
        if (blocks > 0x7fffffff)
            return hipErrorInvalidValue;
        hipLaunchKernelGGL((gemm_packed_kernel<TA, TB, WM, WN, TM, TN, 1>), dim3((unsigned)blocks),
                           dim3(64 * WM * WN), 0, s, a, tiles_m, tiles_n);
    }
    return hipGetLastError();
}

// Tile configuration by operand size (the packed family's own size classes).
enum PackedConfig { PK_WAVE16 = 0, PK_WAVE32 = 1, PK_TILE64 = 2 };

static PackedConfig packed_config(int m, int n)
{
    const int mx = m > n ? m : n;
    if (mx <= 16)
        return PK_WAVE16;
    if (mx <= 32)
        return PK_WAVE32;
    return PK_TILE64;
}

template <bool TA, bool TB>
static hipError_t launch_packed_t(const GemmArgs &a, hipStream_t s)
{
    switch (packed_config(a.m, a.n)) {
    case PK_WAVE16: return launch_cfg<TA, TB, 1, 1, 1, 1, 4>(a, s);
    case PK_WAVE32: return launch_cfg<TA, TB, 1, 1, 2, 2, 4>(a, s);
    default: return launch_cfg<TA, TB, 2, 2, 2, 2, 1>(a, s);
    }
}

hipError_t launch_gemm_packed(bool ta, bool tb, const GemmArgs &a, hipStream_t s)
{
    if (!ta && !tb)
        return launch_packed_t<false, false>(a, s);
    if (!ta && tb)
        return launch_packed_t<false, true>(a, s);
    if (ta && !tb)
        return launch_packed_t<true, false>(a, s);
    return launch_packed_t<true, true>(a, s);
}

const char *packed_kernel_name(int m, int n)
{
    switch (packed_config(m, n)) {
    case PK_WAVE16: return "gemm_packed_wave16";
    case PK_WAVE32: return "gemm_packed_wave32";
    default: return "gemm_packed_tile64";
    }
}

}  // namespace mb
