// potrf.hip -- batched lower Cholesky factorization (dpotrf 'L') on gfx950.
//
// The paper builds LAPACK routines as nested loops around tailored kernels
// rather than on top of BLAS calls (Sec. 1, Sec. 3.1), with the factorization
// kernel composed of the shared dgemm_nt rank-k inner loop, a subtraction
// (alpha = -1, beta = 1), a register-resident factorization of the diagonal
// block and a lower-triangle store (Sec. 3.2.1); off-diagonal blocks use the
// right-variant triangular solve, which vectorizes across rows (Sec. 3.1.3).
//
// gfx950 design: one kernel launch factors every instance of the batch; one
// group of NW waves factors one instance, blocked in 16 x 16 tiles (the FP64
// MFMA tile), right-looking, with the whole lower triangle resident in the
// matrix-core accumulator registers of the group's waves (tile (I,K) is owned
// by wave t % NW, t its column-major index among lower tiles).  Step J:
//   1. the owner of tile (J,J) factors it in registers, lanes over rows and
//      readlane broadcasts (inner_edge_dpotrf), and also forms L_JJ^{-1};
//   2. panel tiles (I,J), I > J: X = A_IJ * L_JJ^{-T}, four MFMA steps whose
//      right operand is the tile's own accumulator registers (right-variant
//      solve expressed as a product with the inverted diagonal block);
//   3. trailing tiles (I,K), J < K <= I: acc -= X_I * X_K^T, four MFMA steps
//      reading both panel tiles from LDS (the dgemm_nt inner update).
// The matrix is read once and written once; the strict upper triangle is never
// accessed.  Orders that are not a multiple of 16 are padded with the identity,
// which the factorization leaves unchanged.  The first non-positive (or NaN)
// pivot stops the instance and is reported as info = column + 1 (LAPACK).
#include <limits.h>

#include "mb_internal.h"

namespace mb {

template <int NT, int PB>
struct PotrfSmem {
    double col[2][16];        // column being eliminated (diagonal tile)
    double xrow[2][16];       // row of L^{-1} being propagated (diagonal tile)
    double W[4][64];          // L_JJ^{-1} in MFMA left-operand order, per k-step
    double P[PB][NT][4][64];  // panel tiles X_I in accumulator order [reg][lane]
    int fail;                 // first failing global column, INT_MAX if none
};

// Factor one 16x16 diagonal tile held in accumulator order -- lane (g, i),
// register r holds T[i][g + 4r] -- by one whole wave (inner_edge_dpotrf).
// Column c is eliminated in step c: its current values are published through
// LDS, every lane forms l_ic = T[i][c]/l_cc for its row and l_qc for its four
// columns q, and updates its own entries T[i][q] -= l_ic*l_qc (c < q <= i).
// Alongside, X = L^{-1} is accumulated in the same order as the product of
// inverted column factors (X <= C_c^{-1} X with C_c the identity except for
// column c of L): row c is scaled by 1/l_cc and rows i > c lose l_ic times it.
// Row c of X is published with column c+1 of T, so each step costs a single
// LDS round trip.  A failing pivot at column c is recorded in S.fail; columns
// c..15 are then replaced by the identity so that L stays invertible.
// On exit t holds L (upper part zero) and x holds L^{-1}, both in accumulator
// order -- which is exactly the left-operand order the panel MFMA needs.
template <class Smem>
__device__ __forceinline__ void factor_diag_tile(d4 &t, d4 &x, Smem &S, int J, int lane)
{
    const int i = lane & 15, g = lane >> 4;
#pragma unroll
    for (int r = 0; r < 4; ++r)
        x[r] = (i == g + 4 * r) ? 1.0 : 0.0;
    bool failed = false;
    double lic_prev = 0.0;  // l_{i,c-1} of the previous step
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        const int buf = c & 1;
        // publish column c of T and (from step 1 on) the scaled row c-1 of X
        if (g == (c & 3))
            S.col[buf][i] = t[c >> 2];
        if (c > 0 && i == c - 1) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
                S.xrow[buf][g + 4 * r] = x[r];
        }
        wave_lds_sync();
        // X update of step c-1: rows i > c-1 lose l_{i,c-1} * (scaled row c-1)
        if (c > 0 && i > c - 1) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
                x[r] = fma(-lic_prev, S.xrow[buf][g + 4 * r], x[r]);
        }
        const double piv = S.col[buf][c];
        if (!failed && !(piv > 0.0)) {
            failed = true;  // uniform: every lane read the same pivot
            if (lane == 0)
                S.fail = 16 * J + c;
        }
        double ljj = 1.0, rinv = 1.0;
        if (!failed) {
            ljj = sqrt(piv);
            rinv = 1.0 / ljj;
        }
        // l_ic for this lane's row (zero above the diagonal and after a failure)
        double lic;
        if (i == c)
            lic = ljj;
        else if (i > c && !failed)
            lic = S.col[buf][i] * rinv;
        else
            lic = 0.0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int q = g + 4 * r;
            if (q > c && q <= i && !failed)
                t[r] = fma(-lic, S.col[buf][q] * rinv, t[r]);
        }
        if (g == (c & 3))
            t[c >> 2] = (i >= c) ? lic : 0.0;
        if (i == c) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
                x[r] *= rinv;
        }
        lic_prev = (i > c) ? lic : 0.0;
    }
    // zero the strict upper part of L (entries of T never touched above)
#pragma unroll
    for (int r = 0; r < 4; ++r)
        if (g + 4 * r > i)
            t[r] = 0.0;
}

template <int NT, int NW, int IPB>
__global__ __launch_bounds__(NW *IPB * 64) void potrf_lower_kernel(PotrfArgs p)
{
    constexpr int T = NT * (NT + 1) / 2;
    constexpr int SLOTS = (T + NW - 1) / NW;
    constexpr bool WAVE_ONLY = (NW == 1);
    constexpr int PB = WAVE_ONLY ? 1 : 2;
    static_assert(IPB == 1 || NW == 1, "several instances per block only with one wave each");
    __shared__ PotrfSmem<NT, PB> smem[IPB];

    const int lane = threadIdx.x & 63;
    const int wib = threadIdx.x >> 6;
    const int inst = wib / NW;
    const int w = __builtin_amdgcn_readfirstlane(wib - inst * NW);
    const int64_t b = (int64_t)blockIdx.x * IPB + inst;
    if (b >= p.batch)
        return;  // IPB > 1 implies NW == 1: this whole wave is idle
    PotrfSmem<NT, PB> &S = smem[inst];
    double *A = inst_ptr(p.A, p.Aarr, p.sA, b);
    const int n = p.n;
    const size_t lda = (size_t)p.lda;
    const int lr = lane & 15, lg = lane >> 4;

    // slot -> tile (I, K); -1 when the slot is unused
    int tI[SLOTS], tK[SLOTS];
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        int t = w + s * NW;
        tI[s] = -1;
        tK[s] = -1;
        if (t < T) {
            int K = 0;
            while (t >= NT - K) {
                t -= NT - K;
                ++K;
            }
            tK[s] = K;
            tI[s] = K + t;
        }
    }

    // load the owned tiles in accumulator order: lane (lg, lr), reg r holds
    // element (16I + lr, 16K + lg + 4r); identity outside the n x n matrix and
    // zeros in the strict upper part of diagonal tiles.
    d4 acc[SLOTS];
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            double v = 0.0;
            if (tI[s] >= 0) {
                const int gi = 16 * tI[s] + lr, gc = 16 * tK[s] + lg + 4 * r;
                if (gi < n && gc < n) {
                    if (gi >= gc)
                        v = A[(size_t)gi + (size_t)gc * lda];
                } else if (gi == gc) {
                    v = 1.0;
                }
            }
            acc[s][r] = v;
        }
    }
    if (w == 0 && lane == 0)
        S.fail = INT_MAX;
    group_sync<WAVE_ONLY>();

    for (int J = 0; J < NT; ++J) {
        const int pb = WAVE_ONLY ? 0 : (J & 1);
        // 1. diagonal tile: its owner factors it and forms L_JJ^{-1}
        {
            bool own = false;
            d4 t = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s = 0; s < SLOTS; ++s) {
                if (tI[s] == J && tK[s] == J) {
                    own = true;
                    t = acc[s];
                }
            }
            if (own) {
                d4 x;
                factor_diag_tile(t, x, S, J, lane);
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    S.W[r][lane] = x[r];
                // store the lower part of L_JJ (columns before a failing pivot only)
                wave_lds_sync();
                const int fail_col = S.fail;
                const int gi = 16 * J + lr;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int gc = 16 * J + lg + 4 * r;
                    if (gi < n && gc <= gi && gc < fail_col)
                        A[(size_t)gi + (size_t)gc * lda] = t[r];
                }
            }
        }
        group_sync<WAVE_ONLY>();
        // 2. panel tiles: X = A_IJ * L_JJ^{-T}; after a failing pivot only the
        //    columns before it are meaningful and stored
        const int fail_col = S.fail;
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            if (tK[s] == J && tI[s] > J) {
                d4 x = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    x = mfma16(S.W[q][lane], acc[s][q], x);
                acc[s] = x;
                const int gi = 16 * tI[s] + lr;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    S.P[pb][tI[s]][r][lane] = x[r];
                    const int gc = 16 * J + lg + 4 * r;
                    if (gi < n && gc < n && gc < fail_col)
                        A[(size_t)gi + (size_t)gc * lda] = x[r];
                }
            }
        }
        group_sync<WAVE_ONLY>();
        // a failure at this step's pivot ends the instance; a later step's
        // diagonal owner may already be writing S.fail, hence the bound
        if (S.fail < 16 * (J + 1))
            break;
        // 3. trailing update: acc(I,K) -= X_I * X_K^T for J < K <= I
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            if (tK[s] > J) {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    acc[s] = mfma16(-S.P[pb][tK[s]][q][lane], S.P[pb][tI[s]][q][lane], acc[s]);
            }
        }
        if constexpr (WAVE_ONLY)
            wave_lds_sync();
    }
    if (w == 0 && lane == 0)
        p.info[b] = (S.fail == INT_MAX) ? 0 : S.fail + 1;
}

__global__ void fill_info_kernel(int *info, int batch)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < batch)
        info[i] = 0;
}

template <int NT, int NW, int IPB>
static hipError_t launch_potrf_t(const PotrfArgs &a, hipStream_t s)
{
    const int64_t blocks = ((int64_t)a.batch + IPB - 1) / IPB;
    hipLaunchKernelGGL((potrf_lower_kernel<NT, NW, IPB>), dim3((unsigned)blocks),
                       dim3(64 * NW * IPB), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_potrf_lower(const PotrfArgs &a, hipStream_t s)
{
    const int nt = (a.n + 15) / 16;
    switch (nt) {
    case 1: return launch_potrf_t<1, 1, 4>(a, s);
    case 2: return launch_potrf_t<2, 1, 4>(a, s);
    case 3: return launch_potrf_t<3, 1, 4>(a, s);
    case 4: return launch_potrf_t<4, 1, 4>(a, s);
    case 5: return launch_potrf_t<5, 4, 1>(a, s);
    case 6: return launch_potrf_t<6, 4, 1>(a, s);
    case 7: return launch_potrf_t<7, 4, 1>(a, s);
    case 8: return launch_potrf_t<8, 4, 1>(a, s);
    case 9: return launch_potrf_t<9, 8, 1>(a, s);
    case 10: return launch_potrf_t<10, 8, 1>(a, s);
    case 11: return launch_potrf_t<11, 8, 1>(a, s);
    case 12: return launch_potrf_t<12, 8, 1>(a, s);
    case 13: return launch_potrf_t<13, 16, 1>(a, s);
    case 14: return launch_potrf_t<14, 16, 1>(a, s);
    case 15: return launch_potrf_t<15, 16, 1>(a, s);
    case 16: return launch_potrf_t<16, 16, 1>(a, s);
    case 17: return launch_potrf_t<17, 16, 1>(a, s);
    case 18: return launch_potrf_t<18, 16, 1>(a, s);
    case 19: return launch_potrf_t<19, 16, 1>(a, s);
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
