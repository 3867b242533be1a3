// potrf_wave.h -- one wave factors one lower Cholesky instance (dpotrf 'L').
//
// Shared by the batched kernel (potrf.hip) and the fused persistent kernel
// (fused.hip).  The paper builds LAPACK routines as nested loops around
// tailored kernels rather than on top of BLAS calls (Sec. 1, Sec. 3.1), with
// the factorization kernel composed of the shared dgemm_nt rank-k inner loop,
// a subtraction (alpha = -1, beta = 1), a register-resident factorization of
// the diagonal block and a lower-triangle store (Sec. 3.2.1); off-diagonal
// blocks use the right-variant triangular solve, which vectorizes across rows
// (Sec. 3.1.3).
//
// gfx950 design: blocked in 16 x 16 tiles (the FP64 MFMA tile) and
// left-looking, so only a few tiles live in the wave's registers and many
// instances share a CU (their serial pivot chains hide behind each other's
// matrix-core work).  Tiles are held in accumulator order -- lane (g, i),
// register r holds element (16I + i, 16J + g + 4r).  With PAIR, block columns
// are processed two at a time, so every factored tile loaded for the update
// serves both (half the re-reads of the factor, more registers); with G1 the
// first G1 panel rows are updated in the diagonal block's loop, which loads
// the pivot tiles L(J,K), L(J1,K) they need anyway; with KC the diagonal
// block's loop also leaves the pivot tiles of its first KC steps in LDS, from
// where the later panel groups take them.  For one block column J:
//   1. tile(J,J) of A minus L(J,K) * L(J,K)^T for every factored block column
//      K < J: four MFMA steps per K whose operands are the registers s of
//      L(J,K) loaded from the factor already written (the k index of step s in
//      lane group g is g + 4s: the accumulator order itself, so no reshuffle);
//   2. factor the diagonal tile in registers and form L_JJ^{-1} alongside
//      (inner_edge_dpotrf); write the lower part of L_JJ;
//   3. panel tiles I > J, two at a time: tile(I,J) of A minus
//      L(I,K) * L(J,K)^T for K < J (the dgemm_nt inner update, alpha = -1,
//      beta = 1), then L(I,J) = tile(I,J) * L_JJ^{-T}, four MFMA steps with
//      L_JJ^{-1} (also in accumulator order) as the left operand -- the
//      right-variant solve expressed as a product with the inverted diagonal
//      block; write L(I,J).
// Only the lower triangle is read or written.  Orders that are not a multiple
// of 16 are padded with the identity, which the factorization leaves
// unchanged.  The first non-positive (or NaN) pivot stops the instance and is
// reported as info = column + 1 (LAPACK).
#pragma once

#include <limits.h>

#include <utility>

#include "mb_internal.h"

namespace mb {

// Per-wave LDS of the diagonal-tile factorization: the lower triangle of the
// tile, packed by columns (element (a, b), a >= b, at tri_pos(a, b)), so that
// every lane can read its whole symmetric row.
struct PotrfSmem {
    double tile[136];
    int fail;  // first failing global column, INT_MAX if none
};

__device__ __forceinline__ int tri_pos(int a, int b)
{
    return 16 * b - (b * (b - 1)) / 2 + (a - b);
}

// 1/sqrt(a) for a positive normal a: the hardware estimate y (relative error
// about 2^-24) refined by one third-order step of the Newton iteration for
// f(y) = 1/y^2 - a, y <- y (1 + e/2 + 3 e^2 / 8) with e = 1 - a y^2 (error
// e^3; the result measured within 1 ulp of the exact value over 2^20 inputs
// spanning 2^-100 .. 2^100).  Four dependent operations after the estimate,
// where two second-order steps take eight.
__device__ __forceinline__ double rsqrt_nr(double a)
{
    const double y = __builtin_amdgcn_rsq(a);
    const double e = fma(-(a * y), y, 1.0);
    return fma(y * e, fma(0.375, e, 0.5), y);
}

// 1/a for a normal a: the hardware estimate refined by two Newton-Raphson
// steps y <- y + y (1 - a y).
__device__ __forceinline__ double rcp_nr(double a)
{
    double y = __builtin_amdgcn_rcp(a);
#pragma unroll
    for (int k = 0; k < 2; ++k)
        y = fma(y, fma(-a, y, 1.0), y);
    return y;
}

// Lane C of every row of 16 lanes, broadcast to the whole row (one 64-bit DPP
// move, row_newbcast).
template <int C>
__device__ __forceinline__ double row_bcast(double v)
{
    return __builtin_amdgcn_mov_dpp(v, 0x150 + C, 0xF, 0xF, true);
}

// Value of v in lane `src` (every lane may name a different source; the LDS
// crossbar, no LDS memory).
__device__ __forceinline__ double lane_read(double v, int src)
{
    const int2 w = __builtin_bit_cast(int2, v);
    const int addr = src * 4;
    int2 r;
    r.x = __builtin_amdgcn_ds_bpermute(addr, w.x);
    r.y = __builtin_amdgcn_ds_bpermute(addr, w.y);
    return __builtin_bit_cast(double, r);
}

// Elimination step C of the diagonal-tile factorization, on tiles in
// accumulator order (lane (g, i), register r: row i, column g + 4r).  T is
// the whole symmetric trailing matrix; every finished row and column of it
// is zero (up to rounding), so the step needs no masks:
//   l_iC = T[i][C] / sqrt(T[C][C]);  T[i][q] -= (T[i][C] / T[C][C]) T[C][q]
// for every i, q -- which also clears row and column C.  T[C][q] is register
// r of lane (g, C), the same group and register: one DPP broadcast within the
// row of 16; T[i][C] is register C/4 of lane (C%4, i): one crossbar read;
// the pivot is T[C][C] of lane (g, C), broadcast likewise.  Column C of the factor goes to register C/4
// of group C%4 of lo (zero above the diagonal).  With INV, X = L^{-1} (same
// order) is updated alongside, X <= C_C^{-1} X for the column factor C_C of L:
// row C is divided by l_CC and rows i > C lose l_iC / l_CC times the old row
// C -- one fma with the DPP-broadcast old row C (multiplier 1 - 1/l_CC on row
// C; rows i < C have multiplier T[i][C] / T[C][C] = 0).  A step past `cols`
// is skipped; a step at a pivot that is not positive, or after one, is
// inactive: zero multipliers, and lo keeps its identity column.  The first
// failing column goes to fc.  No data-dependent branches: the state never
// needs merging.
template <int C, bool INV, bool SKIP>
__device__ __forceinline__ void elim_step(d4 &t, d4 &lo, d4 &x, int lane, int cols, int &fc)
{
    constexpr int RC = C >> 2, GC = C & 3;
    // with SKIP, columns past the order (identity padding) are skipped by a
    // scalar branch (cols is uniform over the wave); without it they run as
    // inactive steps, which keeps the registers of callers whose tiles are
    // mostly full from being spent on merging the branches
    if (SKIP && C >= cols)
        return;
    // an opaque copy of the lane index: the lane masks below are then formed
    // where they are used (one compare each) instead of being hoisted out of
    // the callers' loops, 48 of them held in scalar registers
    asm volatile("" : "+v"(lane));
    const int i = lane & 15, g = lane >> 4;
    const double col = lane_read(t[RC], 16 * GC + i);  // T[i][C]
    const double piv = row_bcast<C>(col);              // T[C][C]
    const bool live = (SKIP || C < cols) && fc == 16;
    const bool act = live && piv > 0.0;
    fc = (live && !act) ? C : fc;
    // an inactive step takes rs = 1 exactly (so 1 - rs = 0)
    const double rs = rsqrt_nr(act ? piv : 1.0);
    const double l = col * rs;
    const double lr = act ? l * rs : 0.0;
    // the broadcasts first, each into its own register: they are
    // independent, and a shared temporary would make every broadcast wait
    // for the fma before it
    d4 tb, xb;
#pragma unroll
    for (int r = 0; r < 4; ++r)
        tb[r] = row_bcast<C>(t[r]);
    if (INV) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
            xb[r] = row_bcast<C>(x[r]);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
        t[r] = fma(-lr, tb[r], t[r]);
    if (g == GC && act)
        lo[RC] = (i >= C) ? l : 0.0;
    // an opaque copy: the select above is done here, in place; otherwise it
    // is deferred to the end of the factorization, with all sixteen lane
    // masks held until then (about 40 more registers)
    {
        double v = lo[RC];
        asm volatile("" : "+v"(v));
        lo[RC] = v;
    }
    if (INV) {
        const double ms = (i == C) ? 1.0 - rs : lr;
#pragma unroll
        for (int r = 0; r < 4; ++r)
            x[r] = fma(-ms, xb[r], x[r]);
    }
}

template <bool INV, bool SKIP, int... C>
__device__ __forceinline__ void elim_steps(d4 &t, d4 &lo, d4 &x, int lane, int cols, int &fc,
                                           std::integer_sequence<int, C...>)
{
    (elim_step<C, INV, SKIP>(t, lo, x, lane, cols, fc), ...);
}

// Factor one 16x16 diagonal tile held in accumulator order -- lane (g, i),
// register r holds T[i][g + 4r], lower triangle valid -- by one whole wave
// (inner_edge_dpotrf).  The tile is made symmetric through LDS (entries right
// of the diagonal read back from the lower triangle), then the columns are
// eliminated in order (elim_step).  Only the first `cols` columns are
// eliminated: the rest of the tile is the identity padding of an order that
// is not a multiple of 16 (SKIP: callers whose tiles are mostly partial skip
// the remaining steps by a scalar branch).  A failing pivot at column c is
// recorded in S.fail (as 16 J + c); columns c..15 of L are then the identity,
// so that L stays invertible.  On exit t holds L (upper part zero) and, with INV, x holds
// L^{-1}, both in accumulator order -- exactly the left-operand order the
// panel MFMA needs.
template <bool INV, bool SKIP = false, class Smem>
__device__ __forceinline__ void factor_diag_tile(d4 &t, d4 &x, Smem &S, int J, int lane,
                                                 int cols = 16)
{
    const int i = lane & 15, g = lane >> 4;
#pragma unroll
    for (int r = 0; r < 4; ++r)
        if (i >= g + 4 * r)
            S.tile[tri_pos(i, g + 4 * r)] = t[r];
    wave_lds_sync();
    d4 lo;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int q = g + 4 * r;
        t[r] = S.tile[q <= i ? tri_pos(i, q) : tri_pos(q, i)];
        lo[r] = (q == i) ? 1.0 : 0.0;
        x[r] = lo[r];
    }
    int fc = 16;
    elim_steps<INV, SKIP>(t, lo, x, lane, cols, fc, std::make_integer_sequence<int, 16>{});
    if (fc < 16 && lane == 0)
        S.fail = 16 * J + fc;
    t = lo;
}

// Step C = 4K + c of factor_tall: register K of every tile holds the four
// columns 4K .. 4K + 3 (lane group g: column 4K + g), so the step touches that
// register only.  Column C of the trailing diagonal tile, T[i][C], comes
// through the crossbar (register K of lane (c, i)); the pivot T[C][C] and row
// C of the block, T[C][4K + g], by DPP broadcasts from lane C of each row of
// 16.  l = T[i][C] / sqrt(piv) goes to group c of lo (column C of L), and
// the block's later columns lose (T[i][C] / piv) T[C][q].  Every panel tile
// does the same with its own column P[i][C]: l_P = P[i][C] / sqrt(piv) to
// column C of its factor, P[i][q] -= l_P T[C][q] / sqrt(piv).  A pivot that
// is not positive makes l_CC a NaN (1/sqrt of it is a NaN or infinite), and
// every later step computes on NaNs; the failure is found from the diagonal
// of L at the end (only columns before it are ever stored; the columns of L
// and of the panel factors before it never mix with the NaNs).
template <int K, int c, int NP>
__device__ __forceinline__ void tall_step(d4 &t, d4 &lo, d4 *P, d4 *LP, int lane)
{
    constexpr int C = 4 * K + c;
    const int i = lane & 15, g = lane >> 4;
    const double col = lane_read(t[K], 16 * c + i);  // T[i][C]
    const double piv = row_bcast<C>(col);           // T[C][C]
    const double rs = rsqrt_nr(piv);
    const double l = col * rs;
    const double tb = row_bcast<C>(t[K]);  // T[C][4K + g]
    t[K] = fma(-(l * rs), tb, t[K]);
    lo[K] = (g == c) ? l : lo[K];
    if (NP > 0) {
        const double tbs = tb * rs;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const double pc = lane_read(P[p][K], 16 * c + i);  // P[i][C]
            const double lp = pc * rs;
            P[p][K] = fma(-lp, tbs, P[p][K]);
            LP[p][K] = (g == c) ? lp : LP[p][K];
        }
    }
}

template <int K, int NP, bool SKIP>
__device__ __forceinline__ void tall_block(d4 &t, d4 &lo, d4 *P, d4 *LP, int lane, int cols)
{
    if (!SKIP || 4 * K + 0 < cols)
        tall_step<K, 0, NP>(t, lo, P, LP, lane);
    if (!SKIP || 4 * K + 1 < cols)
        tall_step<K, 1, NP>(t, lo, P, LP, lane);
    if (!SKIP || 4 * K + 2 < cols)
        tall_step<K, 2, NP>(t, lo, P, LP, lane);
    if (!SKIP || 4 * K + 3 < cols)
        tall_step<K, 3, NP>(t, lo, P, LP, lane);
    if constexpr (K < 3) {
        // the block's four columns of L update everything to their right at
        // once: T -= L_K L_K^T and P -= L_P,K L_K^T, one rank-4 MFMA each
        // (registers up to K receive garbage; they are finished)
        t = mfma16(-lo[K], lo[K], t);
#pragma unroll
        for (int p = 0; p < NP; ++p)
            P[p] = mfma16(-lo[K], LP[p][K], P[p]);
    }
}

// Factor the diagonal tile t (lower triangle valid, accumulator order) and
// solve the NP panel tiles P below it, P <= P L^{-T}, by one wave: the
// right-looking blocked form of the column elimination -- four elimination
// steps per block of four columns on one register (tall_step), then the
// rank-4 update of everything to the right by the matrix cores.  The panel
// tiles go through the same elimination (the right-variant solve, Sec.
// 3.1.3), so no inverse is formed.  Columns at and past `cols` are the
// identity padding of an order that is not a multiple of 16: with SKIP they
// are skipped by scalar branches, otherwise they run as exact identity steps.
// A failing pivot at column c is recorded in S.fail (as 16 J + c).  On exit t
// holds L (upper part zero) and P the panel of L.
template <int NP, bool SKIP, class Smem>
__device__ __forceinline__ void factor_tall(d4 &t, d4 *P, Smem &S, int J, int lane, int cols)
{
    const int i = lane & 15, g = lane >> 4;
#pragma unroll
    for (int r = 0; r < 4; ++r)
        if (i >= g + 4 * r)
            S.tile[tri_pos(i, g + 4 * r)] = t[r];
    wave_lds_sync();
    d4 lo, LP[NP > 0 ? NP : 1];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int q = g + 4 * r;
        t[r] = S.tile[q <= i ? tri_pos(i, q) : tri_pos(q, i)];
        lo[r] = (q == i) ? 1.0 : 0.0;
    }
    tall_block<0, NP, SKIP>(t, lo, P, LP, lane, cols);
    tall_block<1, NP, SKIP>(t, lo, P, LP, lane, cols);
    tall_block<2, NP, SKIP>(t, lo, P, LP, lane, cols);
    tall_block<3, NP, SKIP>(t, lo, P, LP, lane, cols);
    // the first column whose diagonal entry of L is not a positive number
    // (lane (g, i) holds l_ii in register r when i = g + 4r)
    bool bad = false;
#pragma unroll
    for (int r = 0; r < 4; ++r)
        bad |= (i == g + 4 * r) & !(lo[r] > 0.0);
    const uint64_t bm = __builtin_amdgcn_ballot_w64(bad);
    const uint32_t cm = (uint32_t)(bm | (bm >> 16) | (bm >> 32) | (bm >> 48)) & 0xFFFFu;
#pragma unroll
    for (int r = 0; r < 4; ++r)
        t[r] = (i < g + 4 * r) ? 0.0 : lo[r];
#pragma unroll
    for (int p = 0; p < NP; ++p)
        P[p] = LP[p];
    if (cm != 0 && lane == 0)
        S.fail = 16 * J + __builtin_ctz(cm);
}

// Load tile (I, K) in accumulator order.  diag: the tile of A on the
// diagonal (strict upper part read as zero); outside the n x n matrix the
// identity is used.
__device__ __forceinline__ d4 load_tile(const MB_GLOBAL double *A, size_t lda, int n, int I, int K,
                                        int lr, int lg, bool diag)
{
    d4 t;
    const int gi = 16 * I + lr;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int gc = 16 * K + lg + 4 * r;
        double v = 0.0;
        if (gi < n && gc < n) {
            if (!diag || gi >= gc)
                v = A[(size_t)gi + (size_t)gc * lda];
        } else if (gi == gc) {
            v = 1.0;
        }
        t[r] = v;
    }
    return t;
}

// Byte offset of element (r, c) of a matrix that spans less than 4 GiB: one
// 32-bit register per address (scalar base + vector offset), instead of a
// 64-bit address per element.
__device__ __forceinline__ uint32_t off32(int r, int c, uint32_t lda)
{
    return ((uint32_t)r + (uint32_t)c * lda) * 8u;
}

__device__ __forceinline__ double ld_off(const MB_GLOBAL double *A, uint32_t off)
{
    return *(const MB_GLOBAL double *)((const MB_GLOBAL char *)A + off);
}

__device__ __forceinline__ void st_off(MB_GLOBAL double *A, uint32_t off, double v)
{
    *(MB_GLOBAL double *)((MB_GLOBAL char *)A + off) = v;
}

// A wave-uniform address held in scalar registers: a per-register base for
// loads and stores that then share one lane offset (without this the
// compiler folds the base into a 64-bit vector address per base).
template <class T>
__device__ __forceinline__ T *scalar_ptr(T *p)
{
    const uint64_t a = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    return (T *)(((uint64_t)hi << 32) | lo);
}

// load_tile for a matrix of less than 4 GiB.  With FULL (the order is a
// multiple of 16) every element is inside the matrix: plain loads, no
// selects.  Otherwise every lane loads unconditionally, from its element's
// position clamped into the matrix, and only the value is selected (a load
// under a branch ends a basic block, and the compiler then waits for all
// outstanding loads before the first use of any of them); outside the
// matrix the tile is the identity.  The strict upper part of a diagonal
// tile is loaded as it is: the factorization never reads it.
template <bool FULL>
__device__ __forceinline__ d4 load_tile32(const MB_GLOBAL double *A, uint32_t lda, int n, int I,
                                          int K, int lr, int lg)
{
    d4 t;
    const int gi = 16 * I + lr;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int gc = 16 * K + lg + 4 * r;
        if (FULL) {
            // a scalar base per register plus one lane offset for all loads
            const MB_GLOBAL double *At =
                scalar_ptr(A + (16 * I + (16 * K + 4 * r) * (size_t)lda));
            t[r] = ld_off(At, off32(lr, lg, lda));
        } else {
            const double v = ld_off(A, off32(min(gi, n - 1), min(gc, n - 1), lda));
            const bool in = gi < n && gc < n;
            t[r] = in ? v : ((gi == gc) ? 1.0 : 0.0);
        }
    }
    return t;
}

// Store tile (I, J) of L (its lower part if diag), columns before fail_col,
// for a matrix of less than 4 GiB (FULL: the order is a multiple of 16).
template <bool FULL>
__device__ __forceinline__ void store_tile32(MB_GLOBAL double *A, uint32_t lda, int n, int I, int J,
                                             const d4 &t, bool diag, int fail_col, int lr, int lg)
{
    const int gi = 16 * I + lr;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int gc = 16 * J + lg + 4 * r;
        if ((FULL || (gi < n && gc < n)) && gc < fail_col && (!diag || gc <= gi)) {
            MB_GLOBAL double *At = scalar_ptr(A + (16 * I + (16 * J + 4 * r) * (size_t)lda));
            st_off(At, off32(lr, lg, lda), t[r]);
        }
    }
}

// Store the lower part of a diagonal tile (columns before a failing pivot).
__device__ __forceinline__ void store_diag(MB_GLOBAL double *A, size_t lda, int n, int J, const d4 &t,
                                           int fail_col, int lr, int lg)
{
    const int gi = 16 * J + lr;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int gc = 16 * J + lg + 4 * r;
        if (gi < n && gc <= gi && gc < fail_col)
            A[(size_t)gi + (size_t)gc * lda] = t[r];
    }
}

// Store an off-diagonal tile (I, J) of L (columns before a failing pivot).
__device__ __forceinline__ void store_tile(MB_GLOBAL double *A, size_t lda, int n, int I, int J, const d4 &t,
                                           int fail_col, int lr, int lg)
{
    const int gi = 16 * I + lr;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int gc = 16 * J + lg + 4 * r;
        if (gi < n && gc < n && gc < fail_col)
            A[(size_t)gi + (size_t)gc * lda] = t[r];
    }
}

// tile * W^T with W = L_JJ^{-1} in accumulator order (the right-variant solve).
__device__ __forceinline__ d4 solve_right(const d4 &tile, const d4 &w)
{
    d4 xo = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 4; ++s)
        xo = mfma16(w[s], tile[s], xo);
    return xo;
}

// acc -= X * Y^T for two tiles in accumulator order.
__device__ __forceinline__ d4 update_nt(d4 acc, const d4 &x, const d4 &y)
{
#pragma unroll
    for (int s = 0; s < 4; ++s)
        acc = mfma16(-y[s], x[s], acc);
    return acc;
}

// A tile kept in LDS in accumulator order: slot t, register r, lane.  Each
// lane reads back only the values it wrote itself.
__device__ __forceinline__ void lds_put_tile(double *pc, int t, const d4 &x, int lane)
{
#pragma unroll
    for (int r = 0; r < 4; ++r)
        pc[(t * 4 + r) * 64 + lane] = x[r];
}

__device__ __forceinline__ d4 lds_get_tile(const double *pc, int t, int lane)
{
    d4 x;
#pragma unroll
    for (int r = 0; r < 4; ++r)
        x[r] = pc[(t * 4 + r) * 64 + lane];
    return x;
}

// Factor the n x n lower triangle of A (nt = ceil(n / 16) tiles) with the
// calling wave; returns the LAPACK info (0, or the failing column + 1).  S is
// this wave's private LDS block.  With KC > 0, pc is this wave's LDS slot of
// 2 KC tiles: the diagonal block's loop keeps the
// pivot tiles L(J,K), L(J1,K) of its first KC steps there, and every later
// panel group takes those steps from LDS instead of reading them again.
template <bool PAIR, int G = 2, bool PIPE = true, int G1 = 0, int KC = 0>
__device__ __forceinline__ int potrf_wave(double *Ain, size_t lda, int n, int NT, PotrfSmem &S,
                                          int lane, double *pc = nullptr)
{
    MB_GLOBAL double *A = global_ptr(Ain);
    // G: panel row tiles updated together (register footprint grows with G)
    const int lr = lane & 15, lg = lane >> 4;
    constexpr int STEP = PAIR ? 2 : 1;
    if (lane == 0)
        S.fail = INT_MAX;
    wave_lds_sync();

    // With PAIR block columns are taken two at a time (J and J1 = J + 1):
    // every factored tile L(I,K) loaded for the update then serves both.
    for (int J = 0; J < NT; J += STEP) {
        const bool two = PAIR && J + 1 < NT;
        const int J1 = J + 1;
        // --- the 2x2 diagonal block: tiles (J,J), (J1,J), (J1,J1) ---
        d4 t00 = load_tile(A, lda, n, J, J, lr, lg, true);
        d4 t10 = d4{0.0, 0.0, 0.0, 0.0}, t11 = d4{0.0, 0.0, 0.0, 0.0};
        if (two) {
            t10 = load_tile(A, lda, n, J1, J, lr, lg, false);
            t11 = load_tile(A, lda, n, J1, J1, lr, lg, true);
        }
        // The update loops below are software-pipelined: the tiles of step
        // K + 1 are loaded while the MFMAs of step K run (the index is clamped
        // at the last step -- a cached reload instead of a branch).  Row tile
        // NT lies past the matrix and loads as zeros without a memory access,
        // which stands in for J1 when there is no second column.
        // (PIPE = false keeps the plain loops, which need fewer registers.)
        const int R1 = two ? J1 : NT;
        // With G1 > 0 the first G1 panel rows below the pair are updated in
        // the same loop: they need exactly the pivot tiles L(J,K), L(J1,K)
        // that the diagonal block loads, so those are read once per pair
        // instead of once more for the first panel group.
        constexpr int NF = G1 > 0 ? G1 : 1;
        const int F0 = J + STEP;
        d4 f0[NF], f1[NF];
#pragma unroll
        for (int g = 0; g < NF; ++g) {
            const bool in = G1 > 0 && F0 + g < NT;
            f0[g] = in ? load_tile(A, lda, n, F0 + g, J, lr, lg, false) : d4{0.0, 0.0, 0.0, 0.0};
            f1[g] = (in && two) ? load_tile(A, lda, n, F0 + g, J1, lr, lg, false)
                                : d4{0.0, 0.0, 0.0, 0.0};
        }
        if (!PIPE) {
            for (int K = 0; K < J; ++K) {
                const d4 l0 = load_tile(A, lda, n, J, K, lr, lg, false);
                t00 = update_nt(t00, l0, l0);
                d4 l1 = d4{0.0, 0.0, 0.0, 0.0};
                if (two) {
                    l1 = load_tile(A, lda, n, J1, K, lr, lg, false);
                    t10 = update_nt(t10, l1, l0);
                    t11 = update_nt(t11, l1, l1);
                }
                if (KC > 0 && K < KC) {
                    lds_put_tile(pc, 2 * K, l0, lane);
                    lds_put_tile(pc, 2 * K + 1, l1, lane);
                }
                if constexpr (G1 > 0) {
#pragma unroll
                    for (int g = 0; g < NF; ++g) {
                        if (F0 + g < NT) {
                            const d4 lf = load_tile(A, lda, n, F0 + g, K, lr, lg, false);
                            f0[g] = update_nt(f0[g], lf, l0);
                            if (two)
                                f1[g] = update_nt(f1[g], lf, l1);
                        }
                    }
                }
            }
        }
        if (PIPE && J > 0) {
            d4 p0 = load_tile(A, lda, n, J, 0, lr, lg, false);
            d4 p1 = load_tile(A, lda, n, R1, 0, lr, lg, false);
            d4 pf[NF];
#pragma unroll
            for (int g = 0; g < NF; ++g)
                pf[g] = G1 > 0 ? load_tile(A, lda, n, F0 + g, 0, lr, lg, false) : d4{0.0, 0.0, 0.0, 0.0};
            for (int K = 0; K < J; ++K) {
                const d4 l0 = p0, l1 = p1;
                if (KC > 0 && K < KC) {
                    lds_put_tile(pc, 2 * K, l0, lane);
                    lds_put_tile(pc, 2 * K + 1, l1, lane);
                }
                d4 lf[NF];
#pragma unroll
                for (int g = 0; g < NF; ++g)
                    lf[g] = pf[g];
                const int Kn = min(K + 1, J - 1);
                p0 = load_tile(A, lda, n, J, Kn, lr, lg, false);
                p1 = load_tile(A, lda, n, R1, Kn, lr, lg, false);
                if constexpr (G1 > 0) {
#pragma unroll
                    for (int g = 0; g < NF; ++g)
                        pf[g] = load_tile(A, lda, n, F0 + g, Kn, lr, lg, false);
                }
                t00 = update_nt(t00, l0, l0);
                if (two) {
                    t10 = update_nt(t10, l1, l0);
                    t11 = update_nt(t11, l1, l1);
                }
                if constexpr (G1 > 0) {
#pragma unroll
                    for (int g = 0; g < NF; ++g) {
                        if (F0 + g < NT) {
                            f0[g] = update_nt(f0[g], lf[g], l0);
                            if (two)
                                f1[g] = update_nt(f1[g], lf[g], l1);
                        }
                    }
                }
            }
        }
        d4 w0, w1 = d4{0.0, 0.0, 0.0, 0.0};
        factor_diag_tile<true>(t00, w0, S, J, lane, n - 16 * J);
        wave_lds_sync();
        int fail_col = S.fail;
        store_diag(A, lda, n, J, t00, fail_col, lr, lg);
        d4 l10 = d4{0.0, 0.0, 0.0, 0.0};
        if (two) {
            l10 = solve_right(t10, w0);
            store_tile(A, lda, n, J1, J, l10, fail_col, lr, lg);
            if (fail_col == INT_MAX) {
                t11 = update_nt(t11, l10, l10);
                factor_diag_tile<true>(t11, w1, S, J1, lane, n - 16 * J1);
                wave_lds_sync();
                fail_col = S.fail;
                store_diag(A, lda, n, J1, t11, fail_col, lr, lg);
            }
        }
        if constexpr (G1 > 0) {
#pragma unroll
            for (int g = 0; g < NF; ++g) {
                if (F0 + g < NT) {
                    const d4 x0 = solve_right(f0[g], w0);
                    store_tile(A, lda, n, F0 + g, J, x0, fail_col, lr, lg);
                    if (two) {
                        const d4 x1 = solve_right(update_nt(f1[g], x0, l10), w1);
                        store_tile(A, lda, n, F0 + g, J1, x1, fail_col, lr, lg);
                    }
                }
            }
        }
        // --- panel rows I > J1 (after the first G1), G at a time, both columns ---
        for (int I0 = J + STEP + G1; I0 < NT; I0 += G) {
            d4 a0[G], a1[G];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const bool in = I0 + g < NT;
                a0[g] = in ? load_tile(A, lda, n, I0 + g, J, lr, lg, false) : d4{0.0, 0.0, 0.0, 0.0};
                a1[g] = (in && two) ? load_tile(A, lda, n, I0 + g, J1, lr, lg, false)
                                    : d4{0.0, 0.0, 0.0, 0.0};
            }
            if (!PIPE) {
                // steps below Kc take the pivot tiles from the LDS cache
                const int Kc = KC > 0 ? min(J, KC) : 0;
                for (int K = 0; K < Kc; ++K) {
                    const d4 l0 = lds_get_tile(pc, 2 * K, lane);
                    const d4 l1 = lds_get_tile(pc, 2 * K + 1, lane);
#pragma unroll
                    for (int g = 0; g < G; ++g) {
                        if (I0 + g < NT) {
                            const d4 li = load_tile(A, lda, n, I0 + g, K, lr, lg, false);
                            a0[g] = update_nt(a0[g], li, l0);
                            if (two)
                                a1[g] = update_nt(a1[g], li, l1);
                        }
                    }
                }
                for (int K = Kc; K < J; ++K) {
                    const d4 l0 = load_tile(A, lda, n, J, K, lr, lg, false);
                    const d4 l1 = two ? load_tile(A, lda, n, J1, K, lr, lg, false)
                                      : d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int g = 0; g < G; ++g) {
                        if (I0 + g < NT) {
                            const d4 li = load_tile(A, lda, n, I0 + g, K, lr, lg, false);
                            a0[g] = update_nt(a0[g], li, l0);
                            if (two)
                                a1[g] = update_nt(a1[g], li, l1);
                        }
                    }
                }
            } else if (J > 0) {
                // steps below Kc take the pivot tiles from the LDS cache
                const int Kc = KC > 0 ? min(J, KC) : 0;
                d4 pi[G];
#pragma unroll
                for (int g = 0; g < G; ++g)
                    pi[g] = load_tile(A, lda, n, I0 + g, 0, lr, lg, false);
                for (int K = 0; K < Kc; ++K) {
                    const d4 l0 = lds_get_tile(pc, 2 * K, lane);
                    const d4 l1 = lds_get_tile(pc, 2 * K + 1, lane);
                    d4 li[G];
#pragma unroll
                    for (int g = 0; g < G; ++g)
                        li[g] = pi[g];
                    const int Kn = min(K + 1, J - 1);
#pragma unroll
                    for (int g = 0; g < G; ++g)
                        pi[g] = load_tile(A, lda, n, I0 + g, Kn, lr, lg, false);
#pragma unroll
                    for (int g = 0; g < G; ++g) {
                        if (I0 + g < NT) {
                            a0[g] = update_nt(a0[g], li[g], l0);
                            if (two)
                                a1[g] = update_nt(a1[g], li[g], l1);
                        }
                    }
                }
                d4 p0 = d4{0.0, 0.0, 0.0, 0.0}, p1 = d4{0.0, 0.0, 0.0, 0.0};
                if (Kc < J) {
                    p0 = load_tile(A, lda, n, J, Kc, lr, lg, false);
                    p1 = load_tile(A, lda, n, R1, Kc, lr, lg, false);
                }
                for (int K = Kc; K < J; ++K) {
                    const d4 l0 = p0, l1 = p1;
                    d4 li[G];
#pragma unroll
                    for (int g = 0; g < G; ++g)
                        li[g] = pi[g];
                    const int Kn = min(K + 1, J - 1);
                    p0 = load_tile(A, lda, n, J, Kn, lr, lg, false);
                    p1 = load_tile(A, lda, n, R1, Kn, lr, lg, false);
#pragma unroll
                    for (int g = 0; g < G; ++g)
                        pi[g] = load_tile(A, lda, n, I0 + g, Kn, lr, lg, false);
#pragma unroll
                    for (int g = 0; g < G; ++g) {
                        if (I0 + g < NT) {
                            a0[g] = update_nt(a0[g], li[g], l0);
                            if (two)
                                a1[g] = update_nt(a1[g], li[g], l1);
                        }
                    }
                }
            }
#pragma unroll
            for (int g = 0; g < G; ++g) {
                if (I0 + g < NT) {
                    const d4 x0 = solve_right(a0[g], w0);
                    store_tile(A, lda, n, I0 + g, J, x0, fail_col, lr, lg);
                    if (two) {
                        const d4 x1 = solve_right(update_nt(a1[g], x0, l10), w1);
                        store_tile(A, lda, n, I0 + g, J1, x1, fail_col, lr, lg);
                    }
                }
            }
        }
        if (fail_col != INT_MAX || J + STEP >= NT)
            break;
        // the next steps read these block columns back
        wave_mem_sync();
    }
    return (S.fail == INT_MAX) ? 0 : S.fail + 1;
}

// Small orders (a few tiles): the factor kept in registers, every tile read
// once and written once.  Block column J (left-looking): the loads of column
// J + 1 are issued, the tiles of column J lose L(I,K) L(J,K)^T for the
// earlier columns K (factor tiles still in registers), then the diagonal
// tile is factored and the panel below it solved in one blocked elimination
// (factor_tall).  No tile is stored and read back, so there is no memory
// fence and no re-read; only the factor tiles still needed by later columns
// and one column of prefetched tiles are live at a time.  Tile indices are compile-time constants (NT is a template
// parameter), so the tiles stay in registers.  A failing pivot ends the
// factorization after its block column's panel solve; only columns before it
// are stored.  The matrix must span less than 4 GiB (32-bit offsets).
// Block column J of potrf_regs; returns false at a failing pivot.  On entry
// T[I][J] (I >= J) holds the loaded tiles of the column and T[I][K] (K < J)
// the factor tiles of the earlier columns.
template <int NT, bool FULL, int J>
__device__ __forceinline__ bool regs_column(d4 (&T)[NT][NT], MB_GLOBAL double *A, uint32_t lda,
                                            int n, PotrfSmem &S, int lane, int &fail_col)
{
    const int lr = lane & 15, lg = lane >> 4;
    // the next column's loads are in flight while this one is factored
#pragma unroll
    for (int I = J + 1; I < NT && J + 1 < NT; ++I)
        T[I][J + 1] = load_tile32<FULL>(A, lda, n, I, J + 1, lr, lg);
    // left-looking update by the factor tiles of the earlier columns
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
    // only the last diagonal tile can be partial (its steps past the order
    // are skipped)
    factor_tall<NP, !FULL && NP == 0>(T[J][J], P, S, J, lane, n - 16 * J);
    wave_lds_sync();
    fail_col = __builtin_amdgcn_readfirstlane(S.fail);
    // block column J is final: its stores drain while the later columns are
    // factored
    store_tile32<FULL>(A, lda, n, J, J, T[J][J], true, fail_col, lr, lg);
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        T[J + 1 + p][J] = P[p];
        store_tile32<FULL>(A, lda, n, J + 1 + p, J, P[p], false, fail_col, lr, lg);
    }
    return fail_col == INT_MAX;
}

template <int NT, bool FULL, int... J>
__device__ __forceinline__ void regs_columns(d4 (&T)[NT][NT], MB_GLOBAL double *A, uint32_t lda,
                                             int n, PotrfSmem &S, int lane, int &fail_col,
                                             std::integer_sequence<int, J...>)
{
    (regs_column<NT, FULL, J>(T, A, lda, n, S, lane, fail_col) && ...);
}

// FULL: n == 16 NT.
template <int NT, bool FULL>
__device__ __forceinline__ int potrf_regs(double *Ain, uint32_t lda, int n, PotrfSmem &S, int lane)
{
    MB_GLOBAL double *A = global_ptr(Ain);
    const int lr = lane & 15, lg = lane >> 4;
    d4 T[NT][NT];
#pragma unroll
    for (int I = 0; I < NT; ++I)
        T[I][0] = load_tile32<FULL>(A, lda, n, I, 0, lr, lg);
    if (lane == 0)
        S.fail = INT_MAX;
    wave_lds_sync();
    int fail_col = INT_MAX;
    regs_columns<NT, FULL>(T, A, lda, n, S, lane, fail_col, std::make_integer_sequence<int, NT>{});
    return (fail_col == INT_MAX) ? 0 : fail_col + 1;
}

}  // namespace mb
