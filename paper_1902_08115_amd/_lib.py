"""ctypes binding of libmi355blas.so (the C ABI declared in include/mi355blas.h).

Argument marshalling only: every arithmetic step runs in the HIP kernels of
the shared library.  Importing this module raises if the library has not been
built -- there is no fallback of any kind.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("MB_LIBRARY", os.path.join(_HERE, "lib", "libmi355blas.so"))

MB_OK = 0
MB_ERR_HIP = -1000
MB_ERR_UNSUPPORTED = -1001
MB_ERR_INVALID_PROBLEM = -1002
MB_ERR_SCRATCH = -1003
VARIANT_AUTO, VARIANT_DIRECT, VARIANT_PACKED, VARIANT_REGTILE = 0, 1, 2, 3
OP_DGEMM, OP_DPOTRF, OP_DPOTRF_ADJOINT, OP_DLASET = 0, 1, 2, 3
PLAN_FUSED_GRAPH, PLAN_FUSED, PLAN_GROUPED, PLAN_GROUPED_GRAPH = 0, 1, 2, 3
PLAN_STATS = ("problems", "units", "gemm_groups", "other_groups", "workgroups", "waves_per_cu",
              "idle", "cost_ns")

# every symbol the header declares, in declaration order
EXPORTS = (
    "mb_dgemm", "mb_dgemm_strided_batched", "mb_dgemm_batched",
    "mb_dgemm_strided_batched_ex", "mb_dgemm_batched_ex", "mb_dgemm_strided_batched_config",
    "mb_dgemm_config_count", "mb_dgemm_config_name", "mb_dgemm_config_max_mn", "mb_dgemm_select",
    "mb_dgemm_kernel_name", "mb_dpotrf", "mb_dpotrf_strided_batched", "mb_dpotrf_batched",
    "mb_dpotrf_kernel_name",
    "mb_dgemm_backward_strided_batched", "mb_dpotrf_l_backward_strided_batched",
    "mb_dpotrf_l_backward_batched", "mb_dlaset_strided_batched", "mb_dlaset_batched",
    "mb_plan_create", "mb_plan_create_ex", "mb_plan_execute", "mb_plan_execute_mode", "mb_plan_stats",
    "mb_plan_destroy",
    "mb_dgemm_", "mb_dpotrf_",
    "mb_dtrmm_rlnn_strided_batched", "mb_dsyrk_ln_strided_batched",
    "mb_riccati_strided_batched", "mb_riccati_strided_batched_noalloc",
    "mb_riccati_workspace_size",
    "mb_ceiling_fp64", "mb_ceiling_hbm",
    "mb_status_string", "mb_version",
)


class PlanOptions(ctypes.Structure):
    """struct mb_plan_options (negative fields keep the tuned defaults)."""
    _fields_ = [("tile_two_min", ctypes.c_int), ("potrf_waves", ctypes.c_int)]


class Problem(ctypes.Structure):
    """struct mb_problem (one problem of an uneven batch; device pointers)."""
    _fields_ = [
        ("op", ctypes.c_int),
        ("transa", ctypes.c_char), ("transb", ctypes.c_char), ("uplo", ctypes.c_char),
        ("reserved", ctypes.c_char),
        ("m", ctypes.c_int), ("n", ctypes.c_int), ("k", ctypes.c_int),
        ("lda", ctypes.c_int), ("ldb", ctypes.c_int), ("ldc", ctypes.c_int),
        ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
        ("A", ctypes.c_void_p), ("B", ctypes.c_void_p), ("C", ctypes.c_void_p),
        ("info", ctypes.c_void_p),
    ]


_STRING_FNS = ("mb_status_string", "mb_dgemm_kernel_name", "mb_dpotrf_kernel_name",
               "mb_dgemm_config_name")


class MbError(RuntimeError):
    def __init__(self, fn: str, status: int):
        self.status = status
        msg = status_string(status)
        if -64 < status < 0:
            msg = f"illegal value of argument {-status}"
        super().__init__(f"{fn} returned {status}: {msg}")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"mi355blas HIP library not found at {LIB_PATH}; build it first "
            "(python -m paper_1902_08115_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    c_int, c_double, c_char, c_i64, vp = (ctypes.c_int, ctypes.c_double, ctypes.c_char,
                                          ctypes.c_int64, ctypes.c_void_p)
    lib.mb_dgemm.argtypes = [c_char, c_char, c_int, c_int, c_int, c_double, vp, c_int, vp, c_int,
                             c_double, vp, c_int, vp]
    lib.mb_dgemm_strided_batched.argtypes = [c_char, c_char, c_int, c_int, c_int, c_double,
                                             vp, c_int, c_i64, vp, c_int, c_i64, c_double,
                                             vp, c_int, c_i64, c_int, vp]
    lib.mb_dgemm_strided_batched_ex.argtypes = lib.mb_dgemm_strided_batched.argtypes[:-1] + [
        c_int, vp]
    lib.mb_dgemm_batched.argtypes = [c_char, c_char, c_int, c_int, c_int, c_double, vp, c_int,
                                     vp, c_int, c_double, vp, c_int, c_int, vp]
    lib.mb_dgemm_batched_ex.argtypes = lib.mb_dgemm_batched.argtypes[:-1] + [c_int, vp]
    lib.mb_dgemm_strided_batched_config.argtypes = lib.mb_dgemm_strided_batched_ex.argtypes
    lib.mb_dgemm_config_count.argtypes = []
    lib.mb_dgemm_config_name.argtypes = [c_int]
    lib.mb_dgemm_config_max_mn.argtypes = [c_int]
    lib.mb_dgemm_select.argtypes = [c_char, c_char, c_int, c_int, c_int]
    lib.mb_dpotrf.argtypes = [c_char, c_int, vp, c_int, vp, vp]
    lib.mb_dpotrf_strided_batched.argtypes = [c_char, c_int, vp, c_int, c_i64, vp, c_int, vp]
    lib.mb_dpotrf_batched.argtypes = [c_char, c_int, vp, c_int, vp, c_int, vp]
    lib.mb_status_string.argtypes = [c_int]
    lib.mb_dgemm_kernel_name.argtypes = [c_char, c_char, c_int, c_int, c_int, c_int]
    lib.mb_dpotrf_kernel_name.argtypes = [c_int]
    lib.mb_version.argtypes = []
    lib.mb_ceiling_fp64.argtypes = [c_int, c_int, c_int, vp, vp, vp]
    lib.mb_ceiling_hbm.argtypes = [c_int, vp, vp, c_i64, c_int, vp, vp, vp]
    lib.mb_dgemm_backward_strided_batched.argtypes = [
        c_char, c_char, c_int, c_int, c_int, c_double, vp, c_int, c_i64, vp, c_int, c_i64,
        vp, c_int, c_i64, vp, c_int, c_i64, vp, c_int, c_i64, c_int, vp]
    lib.mb_dpotrf_l_backward_strided_batched.argtypes = [c_int, vp, c_int, c_i64, vp, c_int, c_i64,
                                                         vp, c_int, c_i64, c_int, vp]
    lib.mb_dpotrf_l_backward_batched.argtypes = [c_int, vp, c_int, vp, c_int, vp, c_int, c_int, vp]
    lib.mb_dlaset_strided_batched.argtypes = [c_char, c_int, c_int, c_double, c_double, vp, c_int,
                                              c_i64, c_int, vp]
    lib.mb_dlaset_batched.argtypes = [c_char, c_int, c_int, c_double, c_double, vp, c_int, c_int,
                                      vp]
    lib.mb_plan_create.argtypes = [vp, c_i64, ctypes.POINTER(vp), ctypes.POINTER(c_i64)]
    lib.mb_plan_create_ex.argtypes = [vp, c_i64, vp, ctypes.POINTER(vp), ctypes.POINTER(c_i64)]
    lib.mb_plan_execute.argtypes = [vp, vp]
    lib.mb_plan_execute_mode.argtypes = [vp, c_int, vp]
    lib.mb_plan_stats.argtypes = [vp, ctypes.POINTER(c_i64), c_int]
    lib.mb_plan_destroy.argtypes = [vp]
    P = ctypes.POINTER
    lib.mb_dgemm_.argtypes = [P(c_char), P(c_char), P(c_int), P(c_int), P(c_int), P(c_double), vp,
                              P(c_int), vp, P(c_int), P(c_double), vp, P(c_int)]
    lib.mb_dpotrf_.argtypes = [P(c_char), P(c_int), vp, P(c_int), vp]
    lib.mb_dtrmm_rlnn_strided_batched.argtypes = [c_int, c_int, c_double, vp, c_int, c_i64, vp,
                                                  c_int, c_i64, c_int, vp]
    lib.mb_dsyrk_ln_strided_batched.argtypes = [c_int, c_int, c_double, vp, c_int, c_i64, c_double,
                                                vp, c_int, c_i64, c_int, vp]
    lib.mb_riccati_strided_batched.argtypes = [
        c_int, c_int, c_int, vp, c_int, c_i64, c_i64, vp, c_int, c_i64, c_i64, vp, c_int, c_i64,
        vp, c_int, c_i64, c_i64, vp, c_int, c_i64, vp, vp, ctypes.c_size_t, c_int, vp]
    lib.mb_riccati_strided_batched_noalloc.argtypes = [
        c_int, c_int, c_int, vp, c_int, c_i64, c_i64, vp, c_int, c_i64, c_i64, vp, c_int, c_i64,
        vp, c_int, c_i64, c_i64, vp, c_int, c_i64, vp, c_int, vp]
    lib.mb_riccati_workspace_size.argtypes = [c_int, c_int, c_int, ctypes.POINTER(ctypes.c_size_t)]
    for name in EXPORTS:
        getattr(lib, name).restype = ctypes.c_char_p if name in _STRING_FNS else c_int
    return lib


lib = _load()


def status_string(status: int) -> str:
    return lib.mb_status_string(int(status)).decode()


def _ch(x: str) -> bytes:
    return x.encode() if isinstance(x, str) else x


def dgemm(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, stream=0) -> int:
    return lib.mb_dgemm(_ch(transa), _ch(transb), m, n, k, float(alpha), A, lda, B, ldb,
                        float(beta), C, ldc, stream)


def dgemm_strided_batched(transa, transb, m, n, k, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc,
                          sC, batch, stream=0, variant=None) -> int:
    if variant is None:
        return lib.mb_dgemm_strided_batched(_ch(transa), _ch(transb), m, n, k, float(alpha), A,
                                            lda, sA, B, ldb, sB, float(beta), C, ldc, sC, batch,
                                            stream)
    return lib.mb_dgemm_strided_batched_ex(_ch(transa), _ch(transb), m, n, k, float(alpha), A,
                                           lda, sA, B, ldb, sB, float(beta), C, ldc, sC, batch,
                                           int(variant), stream)


def dgemm_batched(transa, transb, m, n, k, alpha, Aarr, lda, Barr, ldb, beta, Carr, ldc, batch,
                  stream=0, variant=None) -> int:
    if variant is None:
        return lib.mb_dgemm_batched(_ch(transa), _ch(transb), m, n, k, float(alpha), Aarr, lda,
                                    Barr, ldb, float(beta), Carr, ldc, batch, stream)
    return lib.mb_dgemm_batched_ex(_ch(transa), _ch(transb), m, n, k, float(alpha), Aarr, lda,
                                   Barr, ldb, float(beta), Carr, ldc, batch, int(variant), stream)


def dgemm_strided_batched_config(transa, transb, m, n, k, alpha, A, lda, sA, B, ldb, sB, beta, C,
                                 ldc, sC, batch, config, stream=0) -> int:
    return lib.mb_dgemm_strided_batched_config(_ch(transa), _ch(transb), m, n, k, float(alpha), A,
                                               lda, sA, B, ldb, sB, float(beta), C, ldc, sC,
                                               batch, int(config), stream)


def dgemm_config_count() -> int:
    return lib.mb_dgemm_config_count()


def dgemm_config_name(config) -> str:
    return lib.mb_dgemm_config_name(int(config)).decode()


def dgemm_config_max_mn(config) -> int:
    return lib.mb_dgemm_config_max_mn(int(config))


def dgemm_select(transa, transb, m, n, k) -> int:
    return lib.mb_dgemm_select(_ch(transa), _ch(transb), m, n, k)


def dgemm_kernel_name(transa, transb, m, n, k, variant=0) -> str:
    return lib.mb_dgemm_kernel_name(_ch(transa), _ch(transb), m, n, k, int(variant)).decode()


def dpotrf_kernel_name(n) -> str:
    return lib.mb_dpotrf_kernel_name(int(n)).decode()


def dpotrf(uplo, n, A, lda, info, stream=0) -> int:
    return lib.mb_dpotrf(_ch(uplo), n, A, lda, info, stream)


def dpotrf_strided_batched(uplo, n, A, lda, sA, info, batch, stream=0) -> int:
    return lib.mb_dpotrf_strided_batched(_ch(uplo), n, A, lda, sA, info, batch, stream)


def dpotrf_batched(uplo, n, Aarr, lda, info, batch, stream=0) -> int:
    return lib.mb_dpotrf_batched(_ch(uplo), n, Aarr, lda, info, batch, stream)


def dgemm_backward_strided_batched(transa, transb, m, n, k, alpha, A, lda, sA, B, ldb, sB, dC,
                                   lddc, sdC, dA, ldda, sdA, dB, lddb, sdB, batch,
                                   stream=0) -> int:
    return lib.mb_dgemm_backward_strided_batched(_ch(transa), _ch(transb), m, n, k, float(alpha),
                                                 A, lda, sA, B, ldb, sB, dC, lddc, sdC, dA, ldda,
                                                 sdA, dB, lddb, sdB, batch, stream)


def dpotrf_l_backward_strided_batched(n, L, ldl, sL, Lbar, ldlb, sLbar, Abar, ldab, sAbar, batch,
                                      stream=0) -> int:
    return lib.mb_dpotrf_l_backward_strided_batched(n, L, ldl, sL, Lbar, ldlb, sLbar, Abar, ldab,
                                                    sAbar, batch, stream)


def dpotrf_l_backward_batched(n, Larr, ldl, Lbararr, ldlb, Abararr, ldab, batch, stream=0) -> int:
    return lib.mb_dpotrf_l_backward_batched(n, Larr, ldl, Lbararr, ldlb, Abararr, ldab, batch,
                                            stream)


def dlaset_strided_batched(uplo, m, n, alpha, beta, A, lda, sA, batch, stream=0) -> int:
    return lib.mb_dlaset_strided_batched(_ch(uplo), m, n, float(alpha), float(beta), A, lda, sA,
                                         batch, stream)


def dlaset_batched(uplo, m, n, alpha, beta, Aarr, lda, batch, stream=0) -> int:
    return lib.mb_dlaset_batched(_ch(uplo), m, n, float(alpha), float(beta), Aarr, lda, batch,
                                 stream)


def dgemm_fortran(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc) -> int:
    """mb_dgemm_: scalars by pointer (None passes a NULL pointer), null stream."""
    def ref(ctype, v):
        return None if v is None else ctypes.byref(ctype(v))
    return lib.mb_dgemm_(ref(ctypes.c_char, _ch(transa) if transa is not None else None),
                         ref(ctypes.c_char, _ch(transb) if transb is not None else None),
                         ref(ctypes.c_int, m), ref(ctypes.c_int, n), ref(ctypes.c_int, k),
                         ref(ctypes.c_double, alpha), A, ref(ctypes.c_int, lda), B,
                         ref(ctypes.c_int, ldb), ref(ctypes.c_double, beta), C,
                         ref(ctypes.c_int, ldc))


def dpotrf_fortran(uplo, n, A, lda, info) -> int:
    """mb_dpotrf_: scalars by pointer (None passes a NULL pointer), null stream."""
    def ref(ctype, v):
        return None if v is None else ctypes.byref(ctype(v))
    return lib.mb_dpotrf_(ref(ctypes.c_char, _ch(uplo) if uplo is not None else None),
                          ref(ctypes.c_int, n), A, ref(ctypes.c_int, lda), info)


def dtrmm_rlnn_strided_batched(m, n, alpha, A, lda, sA, B, ldb, sB, batch, stream=0) -> int:
    return lib.mb_dtrmm_rlnn_strided_batched(m, n, float(alpha), A, lda, sA, B, ldb, sB, batch,
                                             stream)


def dsyrk_ln_strided_batched(n, k, alpha, A, lda, sA, beta, C, ldc, sC, batch, stream=0) -> int:
    return lib.mb_dsyrk_ln_strided_batched(n, k, float(alpha), A, lda, sA, float(beta), C, ldc, sC,
                                           batch, stream)


def riccati_strided_batched(nx, nu, N, BAt, ldbat, stBAt, sBAt, RSQ, ldrsq, stRSQ, sRSQ, QN, ldq,
                            sQ, F, ldf, stF, sF, LN, ldl, sL, info, work, work_bytes, batch,
                            stream=0) -> int:
    return lib.mb_riccati_strided_batched(nx, nu, N, BAt, ldbat, stBAt, sBAt, RSQ, ldrsq, stRSQ,
                                          sRSQ, QN, ldq, sQ, F, ldf, stF, sF, LN, ldl, sL, info,
                                          work, work_bytes, batch, stream)


def riccati_strided_batched_noalloc(nx, nu, N, BAt, ldbat, stBAt, sBAt, RSQ, ldrsq, stRSQ, sRSQ,
                                    QN, ldq, sQ, F, ldf, stF, sF, LN, ldl, sL, info, batch,
                                    stream=0) -> int:
    return lib.mb_riccati_strided_batched_noalloc(nx, nu, N, BAt, ldbat, stBAt, sBAt, RSQ, ldrsq,
                                                  stRSQ, sRSQ, QN, ldq, sQ, F, ldf, stF, sF, LN,
                                                  ldl, sL, info, batch, stream)


def riccati_workspace_size(nx, nu, batch):
    """(status, bytes) of mb_riccati_workspace_size."""
    out = ctypes.c_size_t(0)
    st = lib.mb_riccati_workspace_size(nx, nu, batch, ctypes.byref(out))
    return st, out.value


def version() -> int:
    return lib.mb_version()


def ceiling_fp64(kind, blocks, iters, out, stream=0):
    """(status, flops) of one launch of mb_ceiling_fp64 (kind 0 MFMA, 1 FMA)."""
    fl = ctypes.c_double(0.0)
    st = lib.mb_ceiling_fp64(kind, blocks, iters, out, ctypes.byref(fl), stream)
    return st, fl.value


def ceiling_hbm(kind, src, dst, n, blocks, out, stream=0):
    """(status, bytes) of one launch of mb_ceiling_hbm (kind 0 read, 1 copy,
    2 three reads per write)."""
    by = ctypes.c_double(0.0)
    st = lib.mb_ceiling_hbm(kind, src, dst, n, blocks, out, ctypes.byref(by), stream)
    return st, by.value


def problems_array(problems):
    """ctypes array of Problem from a sequence of Problem or of dicts."""
    arr = (Problem * len(problems))()
    for i, p in enumerate(problems):
        if isinstance(p, Problem):
            arr[i] = p
            continue
        q = arr[i]
        q.op = int(p.get("op", OP_DGEMM))
        q.transa = _ch(p.get("transa", "N"))
        q.transb = _ch(p.get("transb", "N"))
        q.uplo = _ch(p.get("uplo", "L"))
        for f in ("m", "n", "k", "lda", "ldb", "ldc"):
            setattr(q, f, int(p.get(f, 0)))
        q.alpha = float(p.get("alpha", 1.0))
        q.beta = float(p.get("beta", 0.0))
        for f in ("A", "B", "C", "info"):
            setattr(q, f, p.get(f) or None)
    return arr


def plan_create(problems, tile_two_min=None, potrf_waves=None):
    """(status, handle or None, bad_index) for a ctypes Problem array; the
    keyword arguments are the tuning overrides of mb_plan_create_ex."""
    h = ctypes.c_void_p()
    bad = ctypes.c_int64(-1)
    n = len(problems)
    arr = ctypes.cast(problems, ctypes.c_void_p) if n else None
    if tile_two_min is None and potrf_waves is None:
        st = lib.mb_plan_create(arr, n, ctypes.byref(h), ctypes.byref(bad))
    else:
        opt = PlanOptions(-1 if tile_two_min is None else int(tile_two_min),
                          -1 if potrf_waves is None else int(potrf_waves))
        st = lib.mb_plan_create_ex(arr, n, ctypes.cast(ctypes.pointer(opt), ctypes.c_void_p),
                                   ctypes.byref(h), ctypes.byref(bad))
    return st, (h.value if st == MB_OK else None), bad.value


def plan_execute(plan, stream=0, mode=None) -> int:
    if mode is None:
        return lib.mb_plan_execute(plan, stream)
    return lib.mb_plan_execute_mode(plan, int(mode), stream)


def plan_stats(plan) -> dict:
    out = (ctypes.c_int64 * len(PLAN_STATS))()
    st = lib.mb_plan_stats(plan, out, len(PLAN_STATS))
    if st != MB_OK:
        raise MbError("mb_plan_stats", st)
    return dict(zip(PLAN_STATS, list(out)))


def plan_destroy(plan) -> int:
    return lib.mb_plan_destroy(plan)
