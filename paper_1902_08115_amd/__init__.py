"""mi355blas: batched small-matrix FP64 dgemm and lower dpotrf for MI355X (gfx950).

The compute path is the HIP shared library ``lib/libmi355blas.so`` (C ABI in
``include/mi355blas.h``); ``blas`` wraps it for torch tensors and ``_lib`` for
raw device pointers.  Importing ``blas`` or ``_lib`` fails if the library is
not built -- there is no CPU fallback.
"""
__all__ = ["blas", "inputs"]
