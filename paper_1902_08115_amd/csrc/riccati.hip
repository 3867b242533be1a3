// riccati.hip -- batched backward Riccati recursion in the factorized form of
// Sec. 5.2: for each independent problem, Lc_N = chol(Q_N), then for
// n = N-1 .. 0
//   C_n = [B_n^T; A_n^T] * Lc_{n+1}                 (dtrmm_rlnn)
//   F_n = chol([R_n S_n; S_n^T Q_n] + C_n C_n^T)    (dsyrk_ln + dpotrf_l)
//   Lc_n = bottom-right nx x nx block of F_n.
//
// One wave runs one problem's whole recursion, so the stages -- which depend
// on each other -- never leave the wave, and the batch supplies the
// parallelism.  The paper credits part of its API's advantage on this
// workload to a routine that fuses dsyrk with the following dpotrf
// (Sec. 5.2); here the fusion is complete: the C_n C_n^T terms are added into
// the same accumulators as the left-looking Cholesky update, so the matrix
// R + C C^T is never written out.  Per stage:
//   1. dtrmm: every 16 x 16 tile of C_n is a sum of MFMA tile products of
//      BAt_n and the lower factor of the previous stage (read transposed
//      through the cache; its upper triangle is masked, never read); C_n is
//      needed in full while the factor is formed, so its tiles are kept in a
//      lane-private order -- in the wave's part of LDS when they fit (at most
//      six tiles), else in the wave's workspace slot (one coalesced 512-byte
//      row per register);
//   2. fused dsyrk + dpotrf by block column J: tile (I,J) of RSQ_n plus
//      sum_K C(I,K) C(J,K)^T minus sum_{K<J} F(I,K) F(J,K)^T, then the
//      diagonal tile factored in registers (factor_diag_tile) and the panel
//      solved against its inverse -- the structure of potrf_wave.h, with the
//      syrk terms in the same accumulation.
// Problems with nu + nx <= 16 take a register-resident variant (below).
// Otherwise the grid is a fixed set of waves (at most what the device holds at once),
// each owning one workspace slot and taking problems b = w, w + W, ... in
// turn; all problems have the same shape, so the static split is balanced,
// and a slot is rewritten problem after problem while it is still cached.
#include <limits.h>

#include <atomic>
#include <mutex>

#include <type_traits>

#include "potrf_wave.h"

namespace mb {

// waves (independent workers) per workgroup: one measured 1-5% faster than
// four at the (24,12), (40,20) and (64,32) shapes and the same at (8,4)
constexpr int RIC_WPB = 1;

// acc + X * Y^T for tiles in accumulator order.
__device__ __forceinline__ d4 add_xyT(d4 acc, const d4 &x, const d4 &y)
{
#pragma unroll
    for (int s = 0; s < 4; ++s)
        acc = mfma16(y[s], x[s], acc);
    return acc;
}

// Tile (I, T) of the rows x cols matrix X, zero outside it.
__device__ __forceinline__ d4 load_rect(const MB_GLOBAL double *X, size_t ld, int rows, int cols,
                                        int I, int T, int lr, int lg)
{
    d4 t;
    const int gi = 16 * I + lr;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int gc = 16 * T + lg + 4 * r;
        t[r] = (gi < rows && gc < cols) ? X[(size_t)gi + (size_t)gc * ld] : 0.0;
    }
    return t;
}

// Y with Y[i][c] = L(16T + c, 16K + i) for the nx x nx lower factor L (its
// strictly upper part reads as zero, outside the matrix zero): the transpose
// of tile (T, K), so that X * Y^T multiplies by L(T, K).
__device__ __forceinline__ d4 load_lower_t(const MB_GLOBAL double *L, size_t ld, int nx, int T, int K,
                                           int lr, int lg)
{
    d4 t;
    const int col = 16 * K + lr;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = 16 * T + lg + 4 * r;
        t[r] = (row < nx && col < nx && row >= col) ? L[(size_t)row + (size_t)col * ld] : 0.0;
    }
    return t;
}

// Where C lives: tile (I, K) of C holds register r of lane l at
// (I * ntk + K) * 256 + r * 64 + l, either in the wave's slot of the global
// workspace or, when the tiles fit, in the wave's part of LDS.  Each lane
// reads back only what it wrote, so after the dtrmm a wave-level fence
// suffices (global: the stores must complete; LDS: the LDS counter).
struct GlobalC {
    MB_GLOBAL double *W;
    int ntk;
    __device__ __forceinline__ d4 load(int I, int K, int lane) const
    {
        const MB_GLOBAL double *p = W + ((size_t)I * ntk + K) * 256 + lane;
        return d4{p[0], p[64], p[128], p[192]};
    }
    __device__ __forceinline__ void store(int I, int K, const d4 &t, int lane) const
    {
        MB_GLOBAL double *p = W + ((size_t)I * ntk + K) * 256 + lane;
        p[0] = t[0];
        p[64] = t[1];
        p[128] = t[2];
        p[192] = t[3];
    }
    __device__ __forceinline__ void sync() const { wave_mem_sync(); }
};
struct LdsC {
    double *W;  // this wave's LDS block
    int ntk;
    __device__ __forceinline__ d4 load(int I, int K, int lane) const
    {
        const double *p = W + (I * ntk + K) * 256 + lane;
        return d4{p[0], p[64], p[128], p[192]};
    }
    __device__ __forceinline__ void store(int I, int K, const d4 &t, int lane) const
    {
        double *p = W + (I * ntk + K) * 256 + lane;
        p[0] = t[0];
        p[64] = t[1];
        p[128] = t[2];
        p[192] = t[3];
    }
    __device__ __forceinline__ void sync() const { wave_lds_sync(); }
};

// The inner sums below take their operand tiles RIC_CHUNK at a time, all
// loads of a chunk issued before its first MFMA, so that one memory latency
// covers RIC_CHUNK tile products; indices past the end are clamped (a cached
// reload) and their products skipped.
constexpr int RIC_CHUNK = 4;

// C = BAt * L into the workspace: BAt is m x nx, L the nx x nx lower factor;
// ntm = ceil(m / 16) by ntx = ceil(nx / 16) tiles, zero outside m x nx.
template <class CS>
__device__ __forceinline__ void trmm_wave(const MB_GLOBAL double *BAt, size_t ldb, const MB_GLOBAL double *L,
                                          size_t ldl, int m, int nx, int ntm, int ntx, const CS &W,
                                          int lane)
{
    const int lr = lane & 15, lg = lane >> 4;
    for (int I = 0; I < ntm; ++I)
        for (int K = 0; K < ntx; ++K) {
            d4 acc = d4{0.0, 0.0, 0.0, 0.0};
            for (int T0 = K; T0 < ntx; T0 += RIC_CHUNK) {
                d4 x[RIC_CHUNK], y[RIC_CHUNK];
#pragma unroll
                for (int u = 0; u < RIC_CHUNK; ++u) {
                    const int T = min(T0 + u, ntx - 1);
                    x[u] = load_rect(BAt, ldb, m, nx, I, T, lr, lg);
                    y[u] = load_lower_t(L, ldl, nx, T, K, lr, lg);
                }
#pragma unroll
                for (int u = 0; u < RIC_CHUNK; ++u)
                    if (T0 + u < ntx)
                        acc = add_xyT(acc, x[u], y[u]);
            }
            W.store(I, K, acc, lane);
        }
    W.sync();
}

// acc + sum_{K < ntk} C(I,K) C(J,K)^T.
template <class CS>
__device__ __forceinline__ d4 syrk_terms(d4 acc, const CS &W, int ntk, int I, int J, int lane)
{
    for (int K0 = 0; K0 < ntk; K0 += RIC_CHUNK) {
        d4 a[RIC_CHUNK], b[RIC_CHUNK];
#pragma unroll
        for (int u = 0; u < RIC_CHUNK; ++u) {
            const int K = min(K0 + u, ntk - 1);
            a[u] = W.load(I, K, lane);
            b[u] = I == J ? a[u] : W.load(J, K, lane);
        }
#pragma unroll
        for (int u = 0; u < RIC_CHUNK; ++u)
            if (K0 + u < ntk)
                acc = add_xyT(acc, a[u], b[u]);
    }
    return acc;
}

// acc - sum_{K < J} F(I,K) F(J,K)^T from the factor already written.
__device__ __forceinline__ d4 potrf_terms(d4 acc, const MB_GLOBAL double *F, size_t ldf, int m, int I,
                                          int J, int lr, int lg)
{
    for (int K0 = 0; K0 < J; K0 += RIC_CHUNK) {
        d4 a[RIC_CHUNK], b[RIC_CHUNK];
#pragma unroll
        for (int u = 0; u < RIC_CHUNK; ++u) {
            const int K = min(K0 + u, J - 1);
            a[u] = load_tile(F, ldf, m, I, K, lr, lg, false);
            b[u] = I == J ? a[u] : load_tile(F, ldf, m, J, K, lr, lg, false);
        }
#pragma unroll
        for (int u = 0; u < RIC_CHUNK; ++u)
            if (K0 + u < J)
                acc = update_nt(acc, a[u], b[u]);
    }
    return acc;
}

// F = chol(S + C C^T) for the m x m symmetric S (lower triangle read) and the
// ntk tile columns of C in the workspace (ntk = 0: F = chol(S)).  Only the
// lower triangle of F is written, and at a failing pivot only the columns
// before it.  Returns the LAPACK info (0, or the failing column + 1).
template <class CS>
__device__ __forceinline__ int syrk_potrf_wave(const MB_GLOBAL double *Sm, size_t lds, MB_GLOBAL double *F,
                                               size_t ldf, int m, int nt, const CS &W, int ntk,
                                               PotrfSmem &S, int lane)
{
    const int lr = lane & 15, lg = lane >> 4;
    if (lane == 0)
        S.fail = INT_MAX;
    wave_lds_sync();
    for (int J = 0; J < nt; ++J) {
        d4 t = load_tile(Sm, lds, m, J, J, lr, lg, true);
        t = potrf_terms(syrk_terms(t, W, ntk, J, J, lane), F, ldf, m, J, J, lr, lg);
        d4 w;
        factor_diag_tile<true>(t, w, S, J, lane, m - 16 * J);
        wave_lds_sync();
        const int fail_col = S.fail;
        store_diag(F, ldf, m, J, t, fail_col, lr, lg);
        for (int I = J + 1; I < nt; ++I) {
            d4 a = load_tile(Sm, lds, m, I, J, lr, lg, false);
            a = potrf_terms(syrk_terms(a, W, ntk, I, J, lane), F, ldf, m, I, J, lr, lg);
            store_tile(F, ldf, m, I, J, solve_right(a, w), fail_col, lr, lg);
        }
        // later block columns, and the next stage, read these tiles back
        wave_mem_sync();
        if (fail_col != INT_MAX)
            break;
    }
    return (S.fail == INT_MAX) ? 0 : S.fail + 1;
}

// LDS_TILES > 0: C lives in LDS (at most LDS_TILES tiles per wave); 0: in
// the global workspace.
template <int LDS_TILES>
__global__ __launch_bounds__(RIC_WPB * 64) void riccati_kernel(RiccatiArgs p, int waves)
{
    __shared__ PotrfSmem smem[RIC_WPB];
    __shared__ double cbuf[RIC_WPB][LDS_TILES > 0 ? LDS_TILES * 256 : 1];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int w = blockIdx.x * RIC_WPB + wave;
    if (w >= waves)
        return;
    PotrfSmem &S = smem[wave];
    const int nx = p.nx, nu = p.nu, N = p.N, m = nx + nu;
    const int ntm = (m + 15) / 16, ntx = (nx + 15) / 16;
    using CS = typename std::conditional<(LDS_TILES > 0), LdsC, GlobalC>::type;
    CS W;
    if constexpr (LDS_TILES > 0)
        W = LdsC{cbuf[wave], ntx};
    else
        W = GlobalC{global_ptr(p.work) + (size_t)w * ((size_t)ntm * ntx * 256), ntx};
    const GlobalC none{nullptr, 0};
    for (int64_t b = w; b < p.batch; b += waves) {
        MB_GLOBAL int *info = global_ptr(p.info) + b * (N + 1);
        const MB_GLOBAL double *QN = global_ptr(p.QN) + b * p.sQ;
        MB_GLOBAL double *LN = global_ptr(p.LN) + b * p.sL;
        int st = syrk_potrf_wave(QN, (size_t)p.ldq, LN, (size_t)p.ldl, nx, ntx, none, 0, S, lane);
        if (lane == 0)
            info[N] = st;
        int n = N - 1;
        const MB_GLOBAL double *Lc = LN;
        size_t ldlc = (size_t)p.ldl;
        for (; st == 0 && n >= 0; --n) {
            const MB_GLOBAL double *BAt = global_ptr(p.BAt) + b * p.sBAt + n * p.stBAt;
            const MB_GLOBAL double *RSQ = global_ptr(p.RSQ) + b * p.sRSQ + n * p.stRSQ;
            MB_GLOBAL double *F = global_ptr(p.F) + b * p.sF + n * p.stF;
            trmm_wave(BAt, (size_t)p.ldbat, Lc, ldlc, m, nx, ntm, ntx, W, lane);
            st = syrk_potrf_wave(RSQ, (size_t)p.ldrsq, F, (size_t)p.ldf, m, ntm, W, ntx, S, lane);
            if (lane == 0)
                info[n] = st;
            Lc = F + (size_t)nu + (size_t)nu * (size_t)p.ldf;
            ldlc = (size_t)p.ldf;
        }
        // stages below a failure are not computed
        for (int q = lane; q <= n; q += 64)
            info[q] = -1;
    }
}

// Problems with m = nu + nx <= 16: every stage is one 16 x 16 tile, and the
// whole recursion stays in the wave's registers.  Each stage's tile is
// factored by the blocked elimination of the register kernels (factor_tall,
// the columns past the stage's order skipped).  The next stage's BAt and
// RSQ tiles are loaded while the current stage is factored; the factor of
// P_n -- needed transposed by the next stage's dtrmm -- goes from the
// factored tile to the next operand through LDS, so stages exchange nothing
// through global memory (F is only written).
struct RicSmallSmem {
    PotrfSmem potrf;
    double t[16][17];  // factored tile, for the shifted transpose
};

// Y with Y[i][c] = F(nu + c, nu + i) for c, i < nx (else 0): the next dtrmm
// operand (the transpose of the bottom-right nx x nx block) of the factored
// tile f, held in accumulator order.
__device__ __forceinline__ d4 next_operand(const d4 &f, RicSmallSmem &S, int nx, int nu, int lane)
{
    const int i = lane & 15, g = lane >> 4;
#pragma unroll
    for (int r = 0; r < 4; ++r)
        S.t[i][g + 4 * r] = f[r];
    wave_lds_sync();
    d4 y;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int c = g + 4 * r;
        y[r] = (i < nx && c < nx) ? S.t[nu + c][nu + i] : 0.0;
    }
    wave_lds_sync();
    return y;
}

__global__ __launch_bounds__(RIC_WPB * 64) void riccati_small_kernel(RiccatiArgs p)
{
    __shared__ RicSmallSmem smem[RIC_WPB];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t b = (int64_t)blockIdx.x * RIC_WPB + wave;
    if (b >= p.batch)
        return;
    RicSmallSmem &S = smem[wave];
    const int lr = lane & 15, lg = lane >> 4;
    const int nx = p.nx, nu = p.nu, N = p.N, m = nx + nu;
    MB_GLOBAL int *info = global_ptr(p.info) + b * (N + 1);
    const MB_GLOBAL double *BAt = global_ptr(p.BAt) + b * p.sBAt;
    const MB_GLOBAL double *RSQ = global_ptr(p.RSQ) + b * p.sRSQ;
    MB_GLOBAL double *F = global_ptr(p.F) + b * p.sF;

    MB_GLOBAL double *LN = global_ptr(p.LN) + b * p.sL;
    // Iteration n = N factors Q_N (its dtrmm operand is zero); iterations
    // n < N are the stages.  The operands of iteration n - 1 are loaded while
    // iteration n runs.
    d4 x_next = d4{0.0, 0.0, 0.0, 0.0}, y = x_next;
    d4 r_next = load_tile(global_ptr(p.QN) + b * p.sQ, (size_t)p.ldq, nx, 0, 0, lr, lg, true);
    int n = N, st = 0;
    for (; n >= 0; --n) {
        const d4 x = x_next, rq = r_next;
        if (n > 0) {
            x_next = load_rect(BAt + (n - 1) * p.stBAt, (size_t)p.ldbat, m, nx, 0, 0, lr, lg);
            r_next = load_tile(RSQ + (n - 1) * p.stRSQ, (size_t)p.ldrsq, m, 0, 0, lr, lg, true);
        }
        const d4 c = add_xyT(d4{0.0, 0.0, 0.0, 0.0}, x, y);  // C_n = BAt_n Lc_{n+1}
        d4 f = add_xyT(rq, c, c);                            // RSQ_n + C_n C_n^T
        if (lane == 0)
            S.potrf.fail = INT_MAX;
        wave_lds_sync();
        d4 P0[1];
        factor_tall<0, true>(f, P0, S.potrf, 0, lane, n == N ? nx : m);
        wave_lds_sync();
        const int fail = S.potrf.fail;
        const bool term = n == N;
        store_diag(term ? LN : F + n * p.stF, term ? (size_t)p.ldl : (size_t)p.ldf, term ? nx : m, 0, f,
                   fail, lr, lg);
        st = fail == INT_MAX ? 0 : fail + 1;
        if (lane == 0)
            info[n] = st;
        if (st != 0)
            break;
        y = next_operand(f, S, nx, term ? 0 : nu, lane);
    }
    // stages below a failure are not computed
    for (int q = lane; q < n; q += 64)
        info[q] = -1;
}

// ---- m up to 96, nx up to 64: every stage in registers -------------------------
// One wave per problem, no workspace: per stage the dtrmm result C (NTM x
// NTX tiles), the matrix M = RSQ + C C^T (its lower NTM (NTM + 1) / 2 tiles)
// and the factor live in registers, so nothing is stored and read back
// within a stage; F is written once, column block by column block, and
// the next stage reads the factor's bottom-right block Lc back once (L2-hot,
// coalesced, transposed through LDS).  The tile counts are template
// parameters: every tile index is a constant.

// Y[i][c] = X(16T + c, 16K + i) for the nx x nx lower matrix X (zero above
// the diagonal and outside nx): tile (T, K) loaded in its own order -- every
// lane loads from its element's position clamped into the matrix (a 32-bit
// offset from the scalar base), the value selected -- and transposed
// through LDS.
__device__ __forceinline__ d4 ric_lower_t(const MB_GLOBAL double *X, uint32_t ld, int nx, int T,
                                          int K, RicSmallSmem &S, int lane)
{
    const int i = lane & 15, g = lane >> 4;
    const int row = 16 * T + i;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int col = 16 * K + g + 4 * r;
        const double v = ld_off(X, off32(min(row, nx - 1), min(col, nx - 1), ld));
        S.t[i][g + 4 * r] = (row < nx && col < nx && row >= col) ? v : 0.0;
    }
    wave_lds_sync();
    d4 y;
#pragma unroll
    for (int r = 0; r < 4; ++r)
        y[r] = S.t[g + 4 * r][i];
    wave_lds_sync();
    return y;
}

// Tile (I, T) of the rows x cols matrix X, zero outside it; unconditional
// clamped loads (32-bit offsets from the scalar base), the value selected.
__device__ __forceinline__ d4 ric_rect(const MB_GLOBAL double *X, uint32_t ld, int rows, int cols,
                                       int I, int T, int lr, int lg)
{
    d4 t;
    const int gi = 16 * I + lr;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int gc = 16 * T + lg + 4 * r;
        const double v = ld_off(X, off32(min(gi, rows - 1), min(gc, cols - 1), ld));
        t[r] = (gi < rows && gc < cols) ? v : 0.0;
    }
    return t;
}

// Factor the n x n matrix held in T (lower tiles; NT = ceil(n / 16)) in
// registers, left-looking (as potrf_regs), writing the lower triangle of the
// factor to X column block by column block.  Returns the LAPACK info.
template <int NT, int J>
__device__ __forceinline__ bool ric_column(d4 (&T)[NT][NT], MB_GLOBAL double *X, uint32_t ld, int n,
                                           PotrfSmem &S, int lane, int &fail_col)
{
    const int lr = lane & 15, lg = lane >> 4;
#pragma unroll
    for (int I = J; I < NT; ++I)
#pragma unroll
        for (int K = 0; K < J; ++K)
            T[I][J] = update_nt(T[I][J], T[I][K], T[J][K]);
    constexpr int NP = NT - 1 - J;
    d4 P[NP > 0 ? NP : 1];
#pragma unroll
    for (int p = 0; p < NP; ++p)
        P[p] = T[J + 1 + p][J];
    factor_tall<NP, NP == 0>(T[J][J], P, S, J, lane, n - 16 * J);
    wave_lds_sync();
    fail_col = __builtin_amdgcn_readfirstlane(S.fail);
    store_tile32<false>(X, ld, n, J, J, T[J][J], true, fail_col, lr, lg);
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        T[J + 1 + p][J] = P[p];
        store_tile32<false>(X, ld, n, J + 1 + p, J, P[p], false, fail_col, lr, lg);
    }
    return fail_col == INT_MAX;
}

template <int NT, int... J>
__device__ __forceinline__ int ric_factor(d4 (&T)[NT][NT], MB_GLOBAL double *X, uint32_t ld, int n,
                                          PotrfSmem &S, int lane, std::integer_sequence<int, J...>)
{
    if (lane == 0)
        S.fail = INT_MAX;
    wave_lds_sync();
    int fail_col = INT_MAX;
    (ric_column<NT, J>(T, X, ld, n, S, lane, fail_col) && ...);
    return (fail_col == INT_MAX) ? 0 : fail_col + 1;
}

template <int NTM, int NTX>
__global__ __launch_bounds__(RIC_WPB * 64) void riccati_regs_kernel(RiccatiArgs p)
{
    // PIN: the stage's loads are issued a row of C, resp. a tile of M, at a
    // time (scheduling barriers); otherwise the compiler hoists them as far
    // as it can.  Measured per shape (fused ms, 10 stages): pinned (24,12)
    // 2.63 against 2.98, (64,32) 7.42 against 7.78; hoisted (40,20) 3.02
    // against 3.47.
    constexpr bool PIN = !(NTM == 4 && NTX == 3);
    constexpr bool PRE = NTM >= 6;
    __shared__ RicSmallSmem smem[RIC_WPB];
    const int lane0 = threadIdx.x & 63;
    // the problem is uniform over the wave: its addresses stay scalar
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t b = (int64_t)blockIdx.x * RIC_WPB + wave;
    if (b >= p.batch)
        return;
    RicSmallSmem &S = smem[wave];
    const int nx = p.nx, nu = p.nu, N = p.N, m = nx + nu;
    MB_GLOBAL int *info = global_ptr(p.info) + b * (N + 1);
    MB_GLOBAL double *LN = global_ptr(p.LN) + b * p.sL;
    int st;
    {
        const int lane = lane0;
        const int lr = lane & 15, lg = lane >> 4;
        // terminal factor Lc_N = chol(Q_N)
        const MB_GLOBAL double *QN = global_ptr(p.QN) + b * p.sQ;
        d4 T[NTX][NTX];
#pragma unroll
        for (int I = 0; I < NTX; ++I)
#pragma unroll
            for (int K = 0; K <= I; ++K)
                T[I][K] = ric_rect(QN, (uint32_t)p.ldq, nx, nx, I, K, lr, lg);
        st = ric_factor<NTX>(T, LN, (uint32_t)p.ldl, nx, S.potrf, lane,
                             std::make_integer_sequence<int, NTX>{});
    }
    if (lane0 == 0)
        info[N] = st;
    int n = N - 1;
    const MB_GLOBAL double *Lc = LN;
    uint32_t ldlc = (uint32_t)p.ldl;
    for (; st == 0 && n >= 0; --n) {
        const MB_GLOBAL double *BAt = global_ptr(p.BAt) + b * p.sBAt + n * p.stBAt;
        const MB_GLOBAL double *RSQ = global_ptr(p.RSQ) + b * p.sRSQ + n * p.stRSQ;
        MB_GLOBAL double *F = global_ptr(p.F) + b * p.sF + n * p.stF;
        // an opaque copy of the lane index per stage: the element offsets and
        // masks derived from it are formed where they are used instead of
        // being hoisted out of the stage loop (all of them, held in registers
        // for the whole recursion)
        int lane = lane0;
        asm volatile("" : "+v"(lane));
        const int lr = lane & 15, lg = lane >> 4;
        // PRE: the stage's RSQ tiles are loaded first, into M, so that their
        // latency overlaps the fence and the dtrmm (at six row tiles, one
        // wave per SIMD, where nothing else hides it)
        d4 M[NTM][NTM];
        if constexpr (PRE) {
#pragma unroll
            for (int I = 0; I < NTM; ++I)
#pragma unroll
                for (int J = 0; J <= I; ++J)
                    M[I][J] = ric_rect(RSQ, (uint32_t)p.ldrsq, m, m, I, J, lr, lg);
            __builtin_amdgcn_sched_barrier(0);
        }
        // the previous factor's stores are complete before it is read back
        wave_mem_sync();
        d4 Y[NTX][NTX];  // Y[T][K] = Lc(T, K)^T, T >= K
#pragma unroll
        for (int K = 0; K < NTX; ++K)
#pragma unroll
            for (int T = K; T < NTX; ++T)
                Y[T][K] = ric_lower_t(Lc, ldlc, nx, T, K, S, lane);
        // C = BAt Lc
        d4 C[NTM][NTX];
#pragma unroll
        for (int I = 0; I < NTM; ++I) {
            d4 x[NTX];
#pragma unroll
            for (int T = 0; T < NTX; ++T)
                x[T] = ric_rect(BAt, (uint32_t)p.ldbat, m, nx, I, T, lr, lg);
#pragma unroll
            for (int K = 0; K < NTX; ++K) {
                d4 acc = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int T = K; T < NTX; ++T)
                    acc = add_xyT(acc, x[T], Y[T][K]);
                C[I][K] = acc;
            }
            if constexpr (PIN)
                __builtin_amdgcn_sched_barrier(0);
        }
        // M = RSQ + C C^T (lower tiles)
#pragma unroll
        for (int I = 0; I < NTM; ++I)
#pragma unroll
            for (int J = 0; J <= I; ++J) {
                d4 acc = PRE ? M[I][J] : ric_rect(RSQ, (uint32_t)p.ldrsq, m, m, I, J, lr, lg);
#pragma unroll
                for (int K = 0; K < NTX; ++K)
                    acc = add_xyT(acc, C[I][K], C[J][K]);
                M[I][J] = acc;
                if constexpr (PIN)
                    __builtin_amdgcn_sched_barrier(0);
            }
        st = ric_factor<NTM>(M, F, (uint32_t)p.ldf, m, S.potrf, lane,
                             std::make_integer_sequence<int, NTM>{});
        if (lane == 0)
            info[n] = st;
        Lc = F + (size_t)nu + (size_t)nu * (size_t)p.ldf;
        ldlc = (uint32_t)p.ldf;
    }
    // stages below a failure are not computed
    for (int q = lane0; q <= n; q += 64)
        info[q] = -1;
}

// The register-resident kernel's shapes (its 32-bit offsets need every
// operand instance below 4 GiB).  At six by four tiles it holds 381
// registers: one wave per SIMD, still faster than the workspace kernel.
static bool riccati_regs(const RiccatiArgs &a)
{
    const int m = a.nx + a.nu;
    const auto fits = [](int ld, int cols) { return (uint64_t)ld * (uint64_t)cols * 8u < (1ull << 32); };
    return m > 16 && m <= 96 && a.nx >= 1 && a.nx <= 64 && fits(a.ldf, m) && fits(a.ldl, a.nx) &&
           fits(a.ldbat, a.nx) && fits(a.ldrsq, m) && fits(a.ldq, a.nx);
}

template <int NTM, int NTX>
static void launch_riccati_regs_t(const RiccatiArgs &a, hipStream_t s)
{
    const int64_t blocks = (a.batch + RIC_WPB - 1) / RIC_WPB;
    hipLaunchKernelGGL((riccati_regs_kernel<NTM, NTX>), dim3((unsigned)blocks), dim3(RIC_WPB * 64),
                       0, s, a);
}

static hipError_t launch_riccati_regs(const RiccatiArgs &a, hipStream_t s)
{
    const int ntm = (a.nx + a.nu + 15) / 16, ntx = (a.nx + 15) / 16;
    switch (ntm * 4 + ntx) {
    case 2 * 4 + 1: launch_riccati_regs_t<2, 1>(a, s); break;
    case 2 * 4 + 2: launch_riccati_regs_t<2, 2>(a, s); break;
    case 3 * 4 + 1: launch_riccati_regs_t<3, 1>(a, s); break;
    case 3 * 4 + 2: launch_riccati_regs_t<3, 2>(a, s); break;
    case 3 * 4 + 3: launch_riccati_regs_t<3, 3>(a, s); break;
    case 4 * 4 + 1: launch_riccati_regs_t<4, 1>(a, s); break;
    case 4 * 4 + 2: launch_riccati_regs_t<4, 2>(a, s); break;
    case 4 * 4 + 3: launch_riccati_regs_t<4, 3>(a, s); break;
    case 5 * 4 + 1: launch_riccati_regs_t<5, 1>(a, s); break;
    case 5 * 4 + 2: launch_riccati_regs_t<5, 2>(a, s); break;
    case 5 * 4 + 3: launch_riccati_regs_t<5, 3>(a, s); break;
    case 5 * 4 + 4: launch_riccati_regs_t<5, 4>(a, s); break;
    case 6 * 4 + 1: launch_riccati_regs_t<6, 1>(a, s); break;
    case 6 * 4 + 2: launch_riccati_regs_t<6, 2>(a, s); break;
    case 6 * 4 + 3: launch_riccati_regs_t<6, 3>(a, s); break;
    case 6 * 4 + 4: launch_riccati_regs_t<6, 4>(a, s); break;
    case 4 * 4 + 4: launch_riccati_regs_t<4, 4>(a, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int64_t riccati_slot_doubles(int nx, int nu)
{
    const int64_t ntm = (nx + nu + 15) / 16, ntx = (nx + 15) / 16;
    return ntm * ntx * 256;
}

// C in LDS when its tiles fit this many per wave (12 KB: LDS then does not
// lower the occupancy the kernel's registers allow)
constexpr int RIC_LDS_TILES = 6;

static bool riccati_lds(int nx, int nu)
{
    return ((nx + nu + 15) / 16) * ((nx + 15) / 16) <= RIC_LDS_TILES;
}

hipError_t riccati_max_waves(int nx, int nu, int *waves)
{
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = riccati_lds(nx, nu)
                ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                      &per_cu, riccati_kernel<RIC_LDS_TILES>, RIC_WPB * 64, 0)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, riccati_kernel<0>,
                                                               RIC_WPB * 64, 0);
    if (e != hipSuccess)
        return e;
    *waves = std::max(1, cus * std::max(per_cu, 1) * RIC_WPB);
    return hipSuccess;
}

hipError_t launch_riccati(const RiccatiArgs &a, int waves, hipStream_t s)
{
    if (a.nx + a.nu <= 16) {
        const int64_t blocks = (a.batch + RIC_WPB - 1) / RIC_WPB;
        hipLaunchKernelGGL(riccati_small_kernel, dim3((unsigned)blocks), dim3(RIC_WPB * 64), 0, s,
                           a);
        return hipGetLastError();
    }
    if (riccati_regs(a))
        return launch_riccati_regs(a, s);
    const unsigned blocks = (unsigned)((waves + RIC_WPB - 1) / RIC_WPB);
    if (riccati_lds(a.nx, a.nu))
        hipLaunchKernelGGL(riccati_kernel<RIC_LDS_TILES>, dim3(blocks), dim3(RIC_WPB * 64), 0, s, a,
                           waves);
    else
        hipLaunchKernelGGL(riccati_kernel<0>, dim3(blocks), dim3(RIC_WPB * 64), 0, s, a, waves);
    return hipGetLastError();
}

// ---- device scratch of the allocation-free entry point -----------------------
// mb_riccati_strided_batched_noalloc takes its workspace slots from this
// file-scope array instead of a caller's buffer.  Each device holds its own
// copy (RIC_SCRATCH_BYTES, from the first load of this library until the
// process ends) at its own address.  In host code the name `scratch` stands
// for a host-side shadow, not for device memory: host code must only pass
// the address riccati_scratch() resolves.  Every call on one device shares
// the array, so calls that overlap in time on one device race.  The kernel
// writes every slot element before reading it within each problem, so the
// array needs no clearing between calls.
static __device__ __align__(256) double scratch[RIC_SCRATCH_BYTES / sizeof(double)];

hipError_t riccati_scratch(void **ptr, size_t *bytes)
{
    constexpr int MAX_DEVICES = 64;
    static std::atomic<void *> addr[MAX_DEVICES];
    static std::mutex mu;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (dev < 0 || dev >= MAX_DEVICES)
        return hipErrorInvalidDevice;
    void *p = addr[dev].load(std::memory_order_acquire);
    if (!p) {
        // resolved once per device, with that device current
        std::lock_guard<std::mutex> lock(mu);
        p = addr[dev].load(std::memory_order_relaxed);
        if (!p) {
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess)
                return e;
            if (!p)
                return hipErrorInvalidSymbol;
            addr[dev].store(p, std::memory_order_release);
        }
    }
    *ptr = p;
    *bytes = RIC_SCRATCH_BYTES;
    return hipSuccess;
}

}  // namespace mb
