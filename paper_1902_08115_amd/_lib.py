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
VARIANT_AUTO, VARIANT_DIRECT, VARIANT_PACKED = 0, 1, 2

# every symbol the header declares, in declaration order
EXPORTS = (
    "mb_dgemm", "mb_dgemm_strided_batched", "mb_dgemm_batched",
    "mb_dgemm_strided_batched_ex", "mb_dgemm_batched_ex", "mb_dgemm_strided_batched_config",
    "mb_dgemm_config_count", "mb_dgemm_config_name", "mb_dgemm_config_max_mn", "mb_dgemm_select",
    "mb_dgemm_kernel_name", "mb_dpotrf", "mb_dpotrf_strided_batched", "mb_dpotrf_batched",
    "mb_dpotrf_kernel_name",
    "mb_status_string", "mb_version",
)


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


def version() -> int:
    return lib.mb_version()
