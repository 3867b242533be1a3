// gemm_packed.hip -- LDS-staged ("packed") batched dgemm on FP64 matrix cores.
//
// The analogue of the paper's algorithmic variants 'C'/'B' (Sec. 2.2, Table 1):
// the factors are packed, k-panel by k-panel, into an on-chip buffer whose
// layout suits the compute kernel, transposing while packing so that every
// trans case runs the same inner kernel (Sec. 2.2: transposition is free while
// packing; Sec. 3.2.1: one shared inner kernel behind all routines).  On gfx950
// the buffer is LDS and the inner kernel is a v_mfma_f64_16x16x4 rank-4 update.
//
// Packed layout: a BK (16 or 32) deep slice of op(A) (BM x BK) and of op(B)^T
// (BN x BK) is stored row by row with k contiguous, As[i][q] and Bs[j][q], row
// stride SK = BK + 2 doubles (conflict-free 16-byte accesses of 16 consecutive
// rows).
// Both factors are therefore in the "nt" arrangement the paper's kernels use.
//
// Inner kernel: the k index seen by MFMA step s in lane group g = lane/16 is
// q = 4g + s, so every lane fetches its four steps' operands as four
// consecutive doubles of one packed row (two 128-bit LDS reads per 16x16
// tile).  The MFMA is issued with op(B) as its left operand and op(A) as its
// right one, so it accumulates C^T: result register r of lane l holds
// C[16*ti + l%16][16*tj + l/16 + 4r] -- consecutive lanes own consecutive rows
// and the epilogue reads/writes C in 128-byte column segments.
//
// Pipeline: the next k-panel is loaded from global memory into registers while
// the current one is multiplied; with two LDS buffers (DB = 2) one workgroup
// barrier per k-panel suffices.  Each thread stages pairs of consecutive k of
// one row and writes them with one 16-byte LDS store; operands contiguous
// along k are also read with 16-byte global loads when every address is
// 16-byte aligned and k is even (VEC = 2).
//   * Loads go through a raw buffer resource based at the panel's origin:
//     an element outside the matrix gets an offset beyond the resource's
//     record count, which the hardware answers with zero, so the staging code
//     has no branches and the compiler interleaves the next panel's loads with
//     the current panel's MFMAs (the order is pinned with scheduling-group
//     hints).  Leading dimensions above 2^21 fall back to 64-bit addressing
//     with clamped pointers (still branch-free).
//   * While a wave issues its MFMAs it raises its wave priority, so that the
//     waves sharing a SIMD take turns on the matrix core instead of all
//     reaching their barrier at the same time.
//   * C is loaded just before the last k-panel (beta != 0), so its registers
//     are not live during the loop and four workgroups of the 64 x 64 tile fit
//     on a CU.
//
// Launch shapes:
//   * WAVE (IPB > 1): each wave owns one whole instance (C up to 16*TM x 16*TN),
//     IPB instances per workgroup, wave-local synchronisation only;
//   * TILE (IPB == 1): WM x WN waves cooperate on a BM x BN tile of one
//     instance; tiles of one instance are numbered consecutively and mapped to
//     one XCD (shared L2).
#include "mb_internal.h"

#include <cstdint>
#include <type_traits>

namespace mb {

// Raw buffer resource over a panel (record count just under 2 GiB); an offset
// at or beyond kOob reads as zero without touching memory.
constexpr unsigned kOob = 0x80000000u;
// Largest leading dimension for 32-bit buffer offsets: 127 rows or columns of
// a tile at that stride stay below the record count.
constexpr int kBufMaxLd = 1 << 21;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const double *p)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<double *>(p), (short)0, 0x7ffffff0,
                                             0x00020000);
}
// The same with a record count of nrec bytes: offsets at or beyond it read as zero.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc_n(const double *p, unsigned nrec)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<double *>(p), (short)0, (int)nrec,
                                             0x00020000);
}
__device__ __forceinline__ double buf_ld8(__amdgpu_buffer_rsrc_t r, unsigned off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ double2 buf_ld16(__amdgpu_buffer_rsrc_t r, unsigned off)
{
    return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}
// 64-bit form: an invalid element reads the (valid) base address, then is zeroed.
__device__ __forceinline__ double ptr_ld8(const double *base, const double *p, bool in)
{
    const double v = *(in ? p : base);
    return in ? v : 0.0;
}

template <int WM_, int WN_, int TM_, int TN_, int IPB_, int BK_, int DB_>
struct PackedCfg {
    static constexpr int WM = WM_, WN = WN_, TM = TM_, TN = TN_, IPB = IPB_;
    static constexpr int BM = WM * TM * 16;
    static constexpr int BN = WN * TN * 16;
    static constexpr int BK = BK_;             // k depth of one packed panel (16 or 32)
    static constexpr int DB = DB_;             // LDS buffers (2: one barrier per panel)
    static constexpr int SK = BK + 2;          // packed row stride (doubles)
    static constexpr int NTHR = WM * WN * 64;  // threads per instance group
    static constexpr int LDS_A = BM * SK;
    static constexpr int LDS_B = BN * SK;
    static_assert(IPB == 1 || (WM == 1 && WN == 1), "WAVE shape is one wave per instance");
    static_assert(BK == 16 || BK == 32, "panel depth");
    static_assert(DB == 1 || DB == 2, "buffers");
};

// Stage a ROWS x BK slice of op(X) (rows r0.., k from kb) through registers.
// op(X)(row, q) = X[row + q*ld] when the rows are contiguous in memory (!T),
// X[q + row*ld] when k is contiguous (T).  Every thread moves the pair
// (row, q), (row, q+1) and writes it to LDS with one 16-byte store.
//   !T: consecutive threads take consecutive rows, so each of the two 8-byte
//       loads is coalesced across the wave;
//   T:  consecutive threads take consecutive k pairs; one 16-byte load when
//       VEC16 (every address 16-byte aligned, k even), else two 8-byte loads.
template <int ROWS, int NTHR, bool T, bool VEC16, int BK>
struct Stage {
    static constexpr int PAIRS = ROWS * BK / 2;
    static constexpr int PER = PAIRS / NTHR;
    static_assert(PAIRS % NTHR == 0, "staging must divide evenly");
    double v[PER][2];

    __device__ __forceinline__ static void coords(int e, int &row, int &q)
    {
        if (!T) {
            row = e % ROWS;
            q = 2 * (e / ROWS);
        } else {
            q = 2 * (e % (BK / 2));
            row = e / (BK / 2);
        }
    }

    // global loads per thread and panel
    static constexpr int LOADS = (T && VEC16) ? PER : 2 * PER;

    // Stage the panel at k offset kb; rows r0.. of op(X) with nrows rows and
    // k columns, zero outside.  BUF: 32-bit offsets into a buffer resource
    // based at the panel's origin (ld <= kBufMaxLd); else clamped pointers.
    template <bool BUF, bool KFULL = false>
    __device__ __forceinline__ void load(const double *X, size_t ld, int nrows, int k, int r0,
                                         int kb, int tid)
    {
        const double *base = T ? X + kb + (size_t)r0 * ld : X + r0 + (size_t)kb * ld;
        const __amdgpu_buffer_rsrc_t rs = make_rsrc(base);
        const unsigned ldb = (unsigned)ld * 8u;
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            int row, q;
            coords(tid + u * NTHR, row, q);
            const bool rin = r0 + row < nrows;
            // KFULL: the panel lies wholly inside k (only the row test remains)
            const bool in0 = rin && (KFULL || kb + q < k), in1 = rin && (KFULL || kb + q + 1 < k);
            if (!T) {
                if (BUF) {
                    // column q of the panel lies at [q ldb, (q + 1) ldb): the record
                    // count (k - kb) ldb zeroes the columns past k, so only the
                    // loop-invariant row test stays in the per-element offset
                    // (capped at the full record count, which then holds every
                    // column of the panel: k - kb exceeds it)
                    const unsigned kr = k - kb > 0 ? (unsigned)(k - kb) : 0u;
                    const unsigned nrec = kr < 0x7ffffff0u / ldb ? kr * ldb : 0x7ffffff0u;
                    const __amdgpu_buffer_rsrc_t rk = make_rsrc_n(base, nrec);
                    const unsigned off = rin ? (unsigned)row * 8u + (unsigned)q * ldb : kOob;
                    v[u][0] = buf_ld8(rk, off);
                    v[u][1] = buf_ld8(rk, off + ldb);
                } else {
                    const double *ptr = base + row + (size_t)q * ld;
                    v[u][0] = ptr_ld8(base, ptr, in0);
                    v[u][1] = ptr_ld8(base, ptr + ld, in1);
                }
            } else if (BUF) {
                const unsigned off = (unsigned)q * 8u + (unsigned)row * ldb;
                if (VEC16) {
                    // k is even on this path: a pair is either whole or outside
                    const double2 w = buf_ld16(rs, in1 ? off : kOob);
                    v[u][0] = w.x;
                    v[u][1] = w.y;
                } else {
                    v[u][0] = buf_ld8(rs, in0 ? off : kOob);
                    v[u][1] = buf_ld8(rs, in1 ? off + 8u : kOob);
                }
            } else {
                const double *ptr = base + q + (size_t)row * ld;
                v[u][0] = ptr_ld8(base, ptr, in0);
                v[u][1] = ptr_ld8(base, ptr + 1, in1);
            }
        }
    }

    template <int SK>
    __device__ __forceinline__ void store(double *S, int tid) const
    {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            int row, q;
            coords(tid + u * NTHR, row, q);
            *reinterpret_cast<double2 *>(&S[row * SK + q]) = double2{v[u][0], v[u][1]};
        }
    }
};

// Operands of one 16-deep step of a packed panel for this wave's tiles: lane
// (lr, lg) takes k = kk + 4*lg .. +3 of row lr of each of its tiles.  Waves
// with eight or more MFMA tiles read and multiply them in two halves of two k
// (one 16-byte LDS read per tile and half), which keeps half the operand
// registers live -- three waves per SIMD instead of two; smaller waves read
// all four k at once (measured faster there: fewer waits on LDS).
template <class Cfg>
struct Frags {
    static constexpr int TM = Cfg::TM, TN = Cfg::TN, SK = Cfg::SK;
    static constexpr bool HALF = TM * TN >= 8;
    const double *As, *Bs;
    double a[HALF ? 1 : TM][4], b[HALF ? 1 : TN][4];

    __device__ __forceinline__ void read(const double *S, int kk, int wm, int wn, int lr, int lg)
    {
        As = &S[(wm * TM * 16 + lr) * SK + kk + 4 * lg];
        Bs = &S[Cfg::LDS_A + (wn * TN * 16 + lr) * SK + kk + 4 * lg];
        if constexpr (!HALF) {
#pragma unroll
            for (int ti = 0; ti < TM; ++ti) {
                const double2 x = *reinterpret_cast<const double2 *>(As + ti * 16 * SK);
                const double2 y = *reinterpret_cast<const double2 *>(As + ti * 16 * SK + 2);
                a[ti][0] = x.x;
                a[ti][1] = x.y;
                a[ti][2] = y.x;
                a[ti][3] = y.y;
            }
#pragma unroll
            for (int tj = 0; tj < TN; ++tj) {
                const double2 x = *reinterpret_cast<const double2 *>(Bs + tj * 16 * SK);
                const double2 y = *reinterpret_cast<const double2 *>(Bs + tj * 16 * SK + 2);
                b[tj][0] = x.x;
                b[tj][1] = x.y;
                b[tj][2] = y.x;
                b[tj][3] = y.y;
            }
        }
    }

    __device__ __forceinline__ void mma(d4 (&acc)[TM][TN]) const
    {
        if constexpr (!HALF) {
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int ti = 0; ti < TM; ++ti)
#pragma unroll
                    for (int tj = 0; tj < TN; ++tj)
                        acc[ti][tj] = mfma16(b[tj][s], a[ti][s], acc[ti][tj]);
        } else {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                double2 x[TM], y[TN];
#pragma unroll
                for (int ti = 0; ti < TM; ++ti)
                    x[ti] = *reinterpret_cast<const double2 *>(As + ti * 16 * SK + 2 * h);
#pragma unroll
                for (int tj = 0; tj < TN; ++tj)
                    y[tj] = *reinterpret_cast<const double2 *>(Bs + tj * 16 * SK + 2 * h);
#pragma unroll
                for (int ti = 0; ti < TM; ++ti)
#pragma unroll
                    for (int tj = 0; tj < TN; ++tj)
                        acc[ti][tj] = mfma16(y[tj].x, x[ti].x, acc[ti][tj]);
#pragma unroll
                for (int ti = 0; ti < TM; ++ti)
#pragma unroll
                    for (int tj = 0; tj < TN; ++tj)
                        acc[ti][tj] = mfma16(y[tj].y, x[ti].y, acc[ti][tj]);
            }
        }
    }
};

// This wave's C tiles in accumulator order; zero outside the m x n window and
// when beta == 0 (C is then not read).
template <class Cfg, bool BUF>
__device__ __forceinline__ void load_c(const double *C, size_t ldc, int m, int n, int i0, int j0,
                                       int wm, int wn, int lr, int lg, double beta,
                                       d4 (&cin)[Cfg::TM][Cfg::TN])
{
    const double *base = C + i0 + (size_t)j0 * ldc;
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(base);
    const unsigned ldb = (unsigned)ldc * 8u;
#pragma unroll
    for (int ti = 0; ti < Cfg::TM; ++ti) {
        const int li = (wm * Cfg::TM + ti) * 16 + lr;
#pragma unroll
        for (int tj = 0; tj < Cfg::TN; ++tj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int lj = (wn * Cfg::TN + tj) * 16 + lg + 4 * r;
                const bool in = beta != 0.0 && i0 + li < m && j0 + lj < n;
                cin[ti][tj][r] = BUF ? buf_ld8(rs, in ? (unsigned)li * 8u + (unsigned)lj * ldb : kOob)
                                     : ptr_ld8(base, base + li + (size_t)lj * ldc, in);
            }
    }
}

// Scheduling hints for the MFMA block of a staging panel: one global load and
// a few address instructions after each of the first MFMAs, the rest of the
// MFMAs after them.
template <int NMFMA, int NLOAD>
__device__ __forceinline__ void interleave_loads()
{
    constexpr int P = NLOAD < NMFMA ? NLOAD : NMFMA;
#pragma unroll
    for (int z = 0; z < P; ++z) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
        __builtin_amdgcn_sched_group_barrier(0x002, 5, 0);  // VALU
        __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);  // VMEM read
    }
    if constexpr (NMFMA > P)
        __builtin_amdgcn_sched_group_barrier(0x008, NMFMA - P, 0);
}

template <bool TA, bool TB, class Cfg, int VEC, bool BUF>
__global__ __launch_bounds__(Cfg::NTHR *Cfg::IPB) void gemm_packed_kernel(GemmArgs p, int tiles_m,
                                                                          int tiles_n)
{
    constexpr int WM = Cfg::WM, TM = Cfg::TM, TN = Cfg::TN, IPB = Cfg::IPB;
    constexpr int BK = Cfg::BK, DB = Cfg::DB;
    constexpr bool WAVE_ONLY = (IPB > 1);
    constexpr int SK = Cfg::SK;
    __shared__ __align__(16) double smem[IPB][DB][Cfg::LDS_A + Cfg::LDS_B];

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

    using SA = Stage<Cfg::BM, Cfg::NTHR, TA, VEC == 2, BK>;   // op(A): rows i; 'T' A: k contiguous
    using SB = Stage<Cfg::BN, Cfg::NTHR, !TB, VEC == 2, BK>;  // op(B)^T: rows j; 'N' B: k contiguous
    SA sa;
    SB sb;
    sa.template load<BUF>(A, lda, m, k, i0, 0, tid);
    sb.template load<BUF>(B, ldb, n, k, j0, 0, tid);
    sa.template store<SK>(&smem[grp][0][0], tid);
    sb.template store<SK>(&smem[grp][0][Cfg::LDS_A], tid);
    group_sync<WAVE_ONLY>();

    // k loop: every panel but the last also stages the next one; the staging
    // loads are issued among the first MFMAs of the panel's first 16 steps.
    const int klast = ((k - 1) / BK) * BK;
    // one panel at k offset kb read from LDS buffer CUR (a constant, so the
    // LDS addresses are immediate offsets); it stages panel kb + BK into the
    // other buffer (DB == 2) or, after a barrier, into the same one
    auto panel = [&](int kb, auto curc, auto fullc) __attribute__((always_inline)) {
        constexpr int CUR = decltype(curc)::value;
        constexpr bool KF = decltype(fullc)::value;
        const double *S = &smem[grp][CUR][0];
#pragma unroll
        for (int kk = 0; kk < BK; kk += 16) {
            Frags<Cfg> f;
            f.read(S, kk, wm, wn, lr, lg);
            __builtin_amdgcn_s_setprio(1);
            if (kk == 0) {
                sa.template load<BUF, KF>(A, lda, m, k, i0, kb + BK, tid);
                sb.template load<BUF, KF>(B, ldb, n, k, j0, kb + BK, tid);
                f.mma(acc);
                interleave_loads<4 * TM * TN, SA::LOADS + SB::LOADS>();
            } else {
                f.mma(acc);
            }
            __builtin_amdgcn_s_setprio(0);
        }
        constexpr int NXT = (DB == 2) ? (CUR ^ 1) : 0;
        if constexpr (DB == 1)
            group_sync<WAVE_ONLY>();  // everyone is done reading the single buffer
        sa.template store<SK>(&smem[grp][NXT][0], tid);
        sb.template store<SK>(&smem[grp][NXT][Cfg::LDS_A], tid);
        group_sync<WAVE_ONLY>();
    };
    using B0 = std::integral_constant<int, 0>;
    using B1 = std::integral_constant<int, 1>;
    using KPart = std::false_type;
    // panels 0 .. P - 1 run here; panel p stages panel p + 1, which lies wholly
    // inside k unless it is the last one (p = P - 1): with KPEEL the loads of an
    // operand stored along k ('T' A, 'N' B) skip the k test (the last one keeps
    // it; the other operand is bounded by its record count anyway).  Register counts keep it to the
    // workgroup tiles with 16-byte buffer loads and either one buffer of
    // 16-deep panels or at most four MFMA tiles per wave: elsewhere the extra
    // copy of the panel cost a wave per SIMD.
    constexpr bool KPEEL = (TA || !TB) && !WAVE_ONLY && BUF && VEC == 2 &&
                           ((DB == 1 && BK == 16) || TM * TN <= 4);
    using KF = std::integral_constant<bool, KPEEL>;
    const int P = klast / BK;
    int cur = 0;
    if constexpr (KPEEL) {
        if constexpr (DB == 2) {
            if (P > 0) {
                // two panels per trip: buffers 0 then 1
                int p = 0;
                for (; p + 2 < P; p += 2) {
                    panel(p * BK, B0{}, KF{});
                    panel((p + 1) * BK, B1{}, KF{});
                }
                if (p + 1 < P) {
                    panel(p * BK, B0{}, KF{});
                    ++p;
                }
                if (p & 1)
                    panel(p * BK, B1{}, KPart{});
                else
                    panel(p * BK, B0{}, KPart{});
                cur = P & 1;
            }
        } else {
            int p = 0;
            for (; p + 1 < P; ++p)
                panel(p * BK, B0{}, KF{});
            if (P > 0)
                panel(p * BK, B0{}, KPart{});
        }
    } else if constexpr (DB == 2) {
        // two panels per trip: buffers 0 then 1
        int kb = 0;
        for (; kb + BK < klast; kb += 2 * BK) {
            panel(kb, B0{}, KPart{});
            panel(kb + BK, B1{}, KPart{});
        }
        if (kb < klast) {
            panel(kb, B0{}, KPart{});
            cur = 1;
        }
    } else {
        for (int kb = 0; kb < klast; kb += BK)
            panel(kb, B0{}, KPart{});
    }

    // C is needed only by the epilogue: its loads overlap the last panel.
    const double alpha = p.alpha, beta = p.beta;
    d4 cin[TM][TN];
    load_c<Cfg, BUF>(C, ldc, m, n, i0, j0, wm, wn, lr, lg, beta, cin);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
        Frags<Cfg> f;
        f.read(&smem[grp][cur][0], kk, wm, wn, lr, lg);
        __builtin_amdgcn_s_setprio(1);
        f.mma(acc);
        __builtin_amdgcn_s_setprio(0);
    }

    // epilogue: C <= alpha*acc + beta*C, masked to the m x n window
#pragma unroll
    for (int ti = 0; ti < TM; ++ti) {
        const int gi = i0 + (wm * TM + ti) * 16 + lr;
#pragma unroll
        for (int tj = 0; tj < TN; ++tj) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gj = j0 + (wn * TN + tj) * 16 + lg + 4 * r;
                if (gi < m && gj < n) {
                    const double v = acc[ti][tj][r];
                    C[(size_t)gi + (size_t)gj * ldc] =
                        (beta == 0.0) ? alpha * v : fma(alpha, v, beta * cin[ti][tj][r]);
                }
            }
        }
    }
}

// ---------------------------------------------------------------- launch ---

// The menu of packed configurations.  Each entry: waves (WM x WN), MFMA tiles
// per wave (TM x TN), instances per workgroup (IPB > 1: one wave per instance),
// panel depth BK and LDS buffers DB.  The default choice per size class is the
// measured table in gemm_tuned.h (written by the autotuner).
#define MB_PACKED_CONFIGS(X)                                                                \
    X(0, "wave16", 1, 1, 1, 1, 4, 16, 1)                                                     \
    X(1, "wave32", 1, 1, 2, 2, 4, 16, 1)                                                     \
    X(2, "wave48", 1, 1, 3, 3, 2, 16, 1)                                                     \
    X(3, "tile64_k16", 2, 2, 2, 2, 1, 16, 1)                                                 \
    X(4, "tile64_k32", 2, 2, 2, 2, 1, 32, 1)                                                 \
    X(5, "tile64_k16_db", 2, 2, 2, 2, 1, 16, 2)                                              \
    X(6, "tile96_k16", 2, 2, 3, 3, 1, 16, 1)                                                 \
    X(7, "tile128_w4", 2, 2, 4, 4, 1, 16, 1)                                                 \
    X(8, "tile128_w8", 2, 4, 4, 2, 1, 16, 1)                                                 \
    X(9, "tile128_w8_db", 2, 4, 4, 2, 1, 16, 2)                                              \
    X(10, "tile64x128_w8", 2, 4, 2, 2, 1, 16, 1)                                             \
    X(11, "tile96_k32", 2, 2, 3, 3, 1, 32, 1)                                                 \
    X(12, "tile128_w8_k32", 2, 4, 4, 2, 1, 32, 1)                                            \
    X(13, "tile64x128_w8_k32", 2, 4, 2, 2, 1, 32, 1)                                         \
    X(14, "tile128_w4_k32", 2, 2, 4, 4, 1, 32, 1)                                            \
    X(15, "tile128x64_w4", 2, 2, 4, 2, 1, 16, 1)                                             \
    X(16, "tile128x64_w4_db", 2, 2, 4, 2, 1, 16, 2)                                          \
    X(17, "tile64x128_w4", 2, 2, 2, 4, 1, 16, 1)                                             \
    X(18, "tile64x128_w8_db", 2, 4, 2, 2, 1, 16, 2)

#define MB_COUNT_CFG(id, name, wm, wn, tm, tn, ipb, bk, db) +1
constexpr int kPackedConfigs = 0 MB_PACKED_CONFIGS(MB_COUNT_CFG);

// 16-byte global loads need every instance base, stride and leading dimension
// of A and B to keep 16-byte alignment (pointer arrays are not inspected on
// the host: they use 8-byte loads), and an even k (whole pairs).
static bool vec2_ok(const GemmArgs &a)
{
    if (a.Aarr || a.Barr)
        return false;
    const uintptr_t pa = (uintptr_t)a.A, pb = (uintptr_t)a.B;
    return (pa % 16 == 0) && (pb % 16 == 0) && (a.lda % 2 == 0) && (a.ldb % 2 == 0) &&
           (a.sA % 2 == 0) && (a.sB % 2 == 0) && (a.k % 2 == 0);
}

// 32-bit buffer offsets cover every leading dimension up to kBufMaxLd.
static bool buf_ok(const GemmArgs &a)
{
    return a.lda <= kBufMaxLd && a.ldb <= kBufMaxLd && a.ldc <= kBufMaxLd;
}

template <bool TA, bool TB, class Cfg, bool BUF = true>
static hipError_t launch_cfg(const GemmArgs &a, hipStream_t s)
{
    const bool v2 = vec2_ok(a);
    int tiles_m = 1, tiles_n = 1;
    int64_t blocks;
    if constexpr (Cfg::IPB > 1) {
        blocks = ((int64_t)a.batch + Cfg::IPB - 1) / Cfg::IPB;
        if (a.m > Cfg::BM || a.n > Cfg::BN)
            return hipErrorInvalidValue;  // a wave owns a whole instance
    } else {
        tiles_m = (a.m + Cfg::BM - 1) / Cfg::BM;
        tiles_n = (a.n + Cfg::BN - 1) / Cfg::BN;
        blocks = (int64_t)a.batch * tiles_m * tiles_n;
    }
    if (blocks > 0x7fffffff)
        return hipErrorInvalidValue;
    const dim3 grid((unsigned)blocks), block(Cfg::NTHR * Cfg::IPB);
    if (v2)
        hipLaunchKernelGGL((gemm_packed_kernel<TA, TB, Cfg, 2, BUF>), grid, block, 0, s, a,
                           tiles_m, tiles_n);
    else
        hipLaunchKernelGGL((gemm_packed_kernel<TA, TB, Cfg, 1, BUF>), grid, block, 0, s, a,
                           tiles_m, tiles_n);
    return hipGetLastError();
}

template <bool TA, bool TB>
static hipError_t launch_config_t(int config, const GemmArgs &a, hipStream_t s)
{
    // beyond 32-bit offsets: the 64 x 64 tile with 64-bit addressing
    if (!buf_ok(a) && config >= 0 && config < kPackedConfigs)
        return launch_cfg<TA, TB, PackedCfg<2, 2, 2, 2, 1, 16, 1>, false>(a, s);
    switch (config) {
#define MB_CASE_CFG(id, name, wm, wn, tm, tn, ipb, bk, db)                                     \
    case id:                                                                                \
        return launch_cfg<TA, TB, PackedCfg<wm, wn, tm, tn, ipb, bk, db>>(a, s);
        MB_PACKED_CONFIGS(MB_CASE_CFG)
#undef MB_CASE_CFG
    default:
        return hipErrorInvalidValue;
    }
}

int packed_config_count() { return kPackedConfigs; }

const char *packed_config_name(int config)
{
    switch (config) {
#define MB_NAME_CFG(id, name, wm, wn, tm, tn, ipb, bk, db) \
    case id:                                              \
        return "gemm_packed_" name;
        MB_PACKED_CONFIGS(MB_NAME_CFG)
#undef MB_NAME_CFG
    default:
        return "illegal";
    }
}

// Largest C a configuration can take in one wave (WAVE shapes) or 0 (TILE).
int packed_config_wave_limit(int config)
{
    switch (config) {
#define MB_LIM_CFG(id, name, wm, wn, tm, tn, ipb, bk, db) \
    case id:                                             \
        return ipb > 1 ? tm * 16 : 0;
        MB_PACKED_CONFIGS(MB_LIM_CFG)
#undef MB_LIM_CFG
    default:
        return -1;
    }
}

hipError_t launch_gemm_packed_config(int config, bool ta, bool tb, const GemmArgs &a,
                                     hipStream_t s)
{
    if (!ta && !tb)
        return launch_config_t<false, false>(config, a, s);
    if (!ta && tb)
        return launch_config_t<false, true>(config, a, s);
    if (ta && !tb)
        return launch_config_t<true, false>(config, a, s);
    return launch_config_t<true, true>(config, a, s);
}

}  // namespace mb
