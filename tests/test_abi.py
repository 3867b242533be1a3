"""C ABI of libmi355blas.so on the host (no GPU needed): every symbol the
header declares is exported, illegal arguments return -(position) without
launching anything, quick returns succeed, status strings and the size switch
query behave."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mi355blas.h")


@pytest.fixture(scope="module")
def L():
    from paper_1902_08115_amd import _lib
    return _lib


def test_header_symbols_exported(L):
    decl = set(re.findall(r"^\s*(?:int|const char \*)\s*(mb_\w+)\s*\(", open(HEADER).read(), re.M))
    assert decl, "no declarations parsed"
    assert decl == set(L.EXPORTS), decl ^ set(L.EXPORTS)
    for name in decl:
        assert hasattr(L.lib, name), name


def test_version_and_status(L):
    assert L.version() >= 100
    assert L.status_string(0) == "success"
    assert "HIP" in L.status_string(L.MB_ERR_HIP)
    assert "unsupported" in L.status_string(L.MB_ERR_UNSUPPORTED)


P = 0x1000  # a non-null placeholder address: illegal calls never dereference it


def test_dgemm_argument_errors(L):
    g = lambda *a: L.dgemm(*a)  # noqa: E731
    ok = ("N", "N", 4, 4, 4, 1.0, P, 4, P, 4, 1.0, P, 4)
    assert g("X", *ok[1:]) == -1
    assert g("N", "q", *ok[2:]) == -2
    assert g("N", "N", -1, *ok[3:]) == -3
    assert g("N", "N", 4, -1, *ok[4:]) == -4
    assert g("N", "N", 4, 4, -1, *ok[5:]) == -5
    assert g("N", "N", 4, 4, 4, 1.0, P, 3, P, 4, 1.0, P, 4) == -8       # lda < m
    assert g("T", "N", 4, 4, 6, 1.0, P, 4, P, 6, 1.0, P, 4) == -8       # lda < k for 'T'
    assert g("N", "N", 4, 4, 6, 1.0, P, 4, P, 5, 1.0, P, 4) == -10      # ldb < k
    assert g("N", "t", 4, 5, 6, 1.0, P, 4, P, 4, 1.0, P, 4) == -10      # ldb < n for 'T'
    assert g("N", "N", 4, 4, 4, 1.0, P, 4, P, 4, 1.0, P, 3) == -13      # ldc < m
    assert g("N", "N", 0, 4, 4, 1.0, P, 0, P, 4, 1.0, P, 1) == -8       # lda >= 1 even if m == 0
    assert g("N", "N", 4, 4, 4, 1.0, None, 4, P, 4, 1.0, P, 4) == -7    # null A with work
    assert g("N", "N", 4, 4, 4, 1.0, P, 4, None, 4, 1.0, P, 4) == -9
    assert g("N", "N", 4, 4, 4, 1.0, P, 4, P, 4, 1.0, None, 4) == -12


def test_dgemm_quick_returns_without_gpu(L):
    # nothing is launched for these, so they succeed on a host without a GPU
    assert L.dgemm("N", "N", 0, 4, 4, 1.0, None, 1, None, 4, 1.0, None, 1) == 0
    assert L.dgemm("N", "N", 4, 0, 4, 1.0, None, 4, None, 4, 1.0, None, 4) == 0
    assert L.dgemm("N", "N", 4, 4, 4, 0.0, None, 4, None, 4, 1.0, P, 4) == 0
    assert L.dgemm("n", "c", 4, 4, 0, 2.0, None, 4, None, 4, 1.0, P, 4) == 0
    assert L.dgemm_strided_batched("T", "T", 4, 4, 4, 1.0, None, 4, 16, None, 4, 16, 1.0, None, 4,
                                   16, 0) == 0


def test_dgemm_strided_argument_errors(L):
    f = L.dgemm_strided_batched
    base = dict(ta="N", tb="N", m=4, n=4, k=4, al=1.0, A=P, lda=4, sA=16, B=P, ldb=4, sB=16,
                be=1.0, C=P, ldc=4, sC=16, batch=2)

    def call(**kw):
        a = {**base, **kw}
        return f(a["ta"], a["tb"], a["m"], a["n"], a["k"], a["al"], a["A"], a["lda"], a["sA"],
                 a["B"], a["ldb"], a["sB"], a["be"], a["C"], a["ldc"], a["sC"], a["batch"])
    assert call(ta="x") == -1 and call(tb="x") == -2
    assert call(m=-2) == -3 and call(n=-2) == -4 and call(k=-2) == -5
    assert call(lda=3) == -8 and call(ldb=3) == -11 and call(ldc=3) == -15
    assert call(sA=-1) == -9 and call(sB=-1) == -12 and call(sC=-1) == -16
    assert call(batch=-1) == -17
    assert call(sC=15) == -16  # instances of C would overlap
    assert call(A=None) == -7 and call(B=None) == -10 and call(C=None) == -14
    g = L.lib.mb_dgemm_strided_batched_ex
    assert g(b"N", b"N", 4, 4, 4, 1.0, P, 4, 16, P, 4, 16, 1.0, P, 4, 16, 2, 7, None) == -18


def test_dgemm_pointer_array_argument_errors(L):
    f = L.dgemm_batched
    assert f("N", "N", 4, 4, 4, 1.0, P, 4, P, 4, 1.0, P, 4, -1) == -14
    assert f("N", "N", 4, 4, 4, 1.0, P, 3, P, 4, 1.0, P, 4, 2) == -8
    assert f("N", "N", 4, 4, 4, 1.0, P, 4, P, 3, 1.0, P, 4, 2) == -10
    assert f("N", "N", 4, 4, 4, 1.0, P, 4, P, 4, 1.0, P, 2, 2) == -13
    assert f("N", "N", 4, 4, 4, 1.0, None, 4, P, 4, 1.0, P, 4, 2) == -7
    assert f("N", "N", 4, 4, 4, 1.0, P, 4, None, 4, 1.0, P, 4, 2) == -9
    assert f("N", "N", 4, 4, 4, 1.0, P, 4, P, 4, 1.0, None, 4, 2) == -12
    g = L.lib.mb_dgemm_batched_ex
    assert g(b"N", b"N", 4, 4, 4, 1.0, P, 4, P, 4, 1.0, P, 4, 2, -1, None) == -15


def test_dpotrf_argument_errors(L):
    assert L.dpotrf("X", 4, P, 4, P) == -1
    assert L.dpotrf("U", 4, P, 4, P) == L.MB_ERR_UNSUPPORTED
    assert L.dpotrf("L", -1, P, 4, P) == -2
    assert L.dpotrf("L", 4, P, 3, P) == -4
    assert L.dpotrf("L", 4, None, 4, P) == -3
    assert L.dpotrf("L", 4, P, 4, None) == -5
    assert L.dpotrf("l", 305, P, 305, P) == L.MB_ERR_UNSUPPORTED
    f = L.dpotrf_strided_batched
    assert f("L", 4, P, 4, -1, P, 2) == -5
    assert f("L", 4, P, 4, 15, P, 2) == -5  # overlapping instances
    assert f("L", 4, P, 4, 16, P, -1) == -7
    assert f("L", 4, P, 4, 16, None, 2) == -6
    assert f("L", 4, P, 4, 16, P, 0) == 0   # batch == 0: quick return
    g = L.dpotrf_batched
    assert g("L", 4, P, 4, P, -1) == -6
    assert g("L", 4, None, 4, P, 2) == -3
    assert g("L", 4, P, 4, None, 2) == -5
    assert g("L", 4, P, 2, P, 2) == -4


def test_size_switch_query(L):
    assert L.dgemm_select("N", "N", 4, 4, 4) == L.VARIANT_DIRECT
    assert L.dgemm_select("t", "c", 300, 300, 300) == L.VARIANT_PACKED
    assert L.dgemm_select("x", "N", 4, 4, 4) == -1
    # the choice depends on the shape only
    for ta in "NT":
        for tb in "NT":
            assert L.dgemm_select(ta, tb, 128, 128, 128) == L.VARIANT_PACKED


def test_kernel_name_queries(L):
    assert L.dgemm_kernel_name("N", "N", 4, 4, 4) == "gemm_direct"
    assert L.dgemm_kernel_name("N", "N", 4, 4, 4, L.VARIANT_PACKED).startswith("gemm_packed")
    assert L.dgemm_kernel_name("T", "T", 256, 256, 256).startswith("gemm_packed")
    assert L.dgemm_kernel_name("N", "N", 4, 4, 0) == "gemm_scale"
    assert L.dgemm_kernel_name("x", "N", 4, 4, 4) == "illegal"
    assert L.dpotrf_kernel_name(256) == "potrf_nt16"
    assert L.dpotrf_kernel_name(400) == "unsupported"


def test_config_menu_queries(L):
    count = L.dgemm_config_count()
    assert count >= 1
    names = [L.dgemm_config_name(c) for c in range(count)]
    assert len(set(names)) == count and all(n.startswith("gemm_packed_") for n in names)
    assert L.dgemm_config_name(count) == "illegal" and L.dgemm_config_max_mn(count) == -1
    for c in range(count):
        lim = L.dgemm_config_max_mn(c)
        assert lim >= 16
        if lim < 2 ** 31 - 1:  # a one-wave shape refuses larger instances (host check only)
            assert L.dgemm_strided_batched_config("N", "N", lim + 1, 1, 1, 1.0, P, lim + 1, 0, P,
                                                  1, 0, 0.0, P, lim + 1, 0, 1, c) == \
                L.MB_ERR_UNSUPPORTED
    assert L.dgemm_strided_batched_config("N", "N", 4, 4, 4, 1.0, P, 4, 16, P, 4, 16, 1.0, P, 4,
                                          16, 1, count) == -18


def test_plan_argument_errors(L):
    """Plan creation validates everything on the host before touching the
    device: argument positions, then the first failing problem by index."""
    import ctypes
    h = ctypes.c_void_p()
    bad = ctypes.c_int64(-1)
    assert L.lib.mb_plan_create(None, 1, ctypes.byref(h), ctypes.byref(bad)) == -1
    arr = L.problems_array([dict(op=0, m=4, n=4, k=4, lda=4, ldb=4, ldc=4, A=P, B=P, C=P)])
    assert L.lib.mb_plan_create(ctypes.cast(arr, ctypes.c_void_p), -1, ctypes.byref(h),
                                ctypes.byref(bad)) == -2
    assert L.lib.mb_plan_create(ctypes.cast(arr, ctypes.c_void_p), 1, None, None) == -3
    good = dict(op=0, m=4, n=4, k=4, lda=4, ldb=4, ldc=4, A=P, B=P, C=P)
    pot = dict(op=1, uplo="L", n=8, ldc=8, C=P, info=P)
    cases = [
        (dict(good, op=7), L.MB_ERR_INVALID_PROBLEM),
        (dict(good, transa="x"), L.MB_ERR_INVALID_PROBLEM),
        (dict(good, m=-1), L.MB_ERR_INVALID_PROBLEM),
        (dict(good, lda=3), L.MB_ERR_INVALID_PROBLEM),
        (dict(good, transb="T", n=6, ldb=5), L.MB_ERR_INVALID_PROBLEM),
        (dict(good, ldc=3), L.MB_ERR_INVALID_PROBLEM),
        (dict(good, A=None), L.MB_ERR_INVALID_PROBLEM),
        (dict(good, C=None), L.MB_ERR_INVALID_PROBLEM),
        (dict(good, m=70000, n=70000, lda=70000, ldc=70000), L.MB_ERR_UNSUPPORTED),  # > 4 GiB
        (dict(pot, uplo="U"), L.MB_ERR_UNSUPPORTED),
        (dict(pot, uplo="q"), L.MB_ERR_INVALID_PROBLEM),
        (dict(pot, n=305, ldc=305), L.MB_ERR_UNSUPPORTED),
        (dict(pot, ldc=7), L.MB_ERR_INVALID_PROBLEM),
        (dict(pot, info=None), L.MB_ERR_INVALID_PROBLEM),
        (dict(pot, C=None), L.MB_ERR_INVALID_PROBLEM),
    ]
    for prob, want in cases:
        arr = L.problems_array([good, pot, prob])
        st, handle, idx = L.plan_create(arr)
        assert (st, idx, handle) == (want, 2, None), (prob, st, idx)
    assert L.lib.mb_plan_execute(None, None) == -1
    assert L.lib.mb_plan_execute_mode(None, 0, None) == -1
    assert L.lib.mb_plan_stats(None, None, 0) == -1
    assert L.lib.mb_plan_destroy(None) == 0
    assert "plan problem" in L.status_string(L.MB_ERR_INVALID_PROBLEM)


def test_backward_argument_errors(L):
    f = L.dpotrf_l_backward_strided_batched
    ok = dict(n=8, L=P, ldl=8, sL=64, Lb=P, ldlb=8, sLb=64, Ab=P, ldab=8, sAb=64, batch=2)

    def call(**kw):
        a = {**ok, **kw}
        return f(a["n"], a["L"], a["ldl"], a["sL"], a["Lb"], a["ldlb"], a["sLb"], a["Ab"],
                 a["ldab"], a["sAb"], a["batch"])
    assert call(n=-1) == -1 and call(ldl=7) == -3 and call(sL=-1) == -4
    assert call(ldlb=7) == -6 and call(sLb=-1) == -7 and call(ldab=7) == -9
    assert call(sAb=63) == -10 and call(batch=-1) == -11
    assert call(L=None) == -2 and call(Lb=None) == -5 and call(Ab=None) == -8
    assert call(n=305, ldl=305, ldlb=305, ldab=305, sL=305 * 305, sLb=305 * 305,
                sAb=305 * 305) == L.MB_ERR_UNSUPPORTED
    assert call(n=0, L=None, Lb=None, Ab=None) == 0 and call(batch=0) == 0
    g = L.dpotrf_l_backward_batched
    assert g(-1, P, 8, P, 8, P, 8, 1) == -1 and g(8, P, 7, P, 8, P, 8, 1) == -3
    assert g(8, P, 8, P, 7, P, 8, 1) == -5 and g(8, P, 8, P, 8, P, 7, 1) == -7
    assert g(8, P, 8, P, 8, P, 8, -1) == -8 and g(8, None, 8, P, 8, P, 8, 1) == -2
    d = L.dgemm_backward_strided_batched
    base = ["N", "N", 4, 5, 6, 1.0, P, 4, 24, P, 6, 30, P, 4, 20, P, 4, 24, P, 6, 30, 2]

    def dcall(i, v):
        a = list(base)
        a[i] = v
        return d(*a)
    assert dcall(0, "x") == -1 and dcall(1, "x") == -2 and dcall(2, -1) == -3
    assert dcall(3, -1) == -4 and dcall(4, -1) == -5 and dcall(7, 3) == -8
    assert dcall(8, -1) == -9 and dcall(10, 5) == -11 and dcall(11, -1) == -12
    assert dcall(13, 3) == -14 and dcall(14, -1) == -15 and dcall(16, 3) == -17
    assert dcall(17, 23) == -18 and dcall(19, 5) == -20 and dcall(20, 29) == -21
    assert dcall(21, -1) == -22 and dcall(12, None) == -13 and dcall(9, None) == -10
    assert dcall(21, 0) == 0
    s = L.dlaset_strided_batched
    assert s("x", 4, 4, 0.0, 0.0, P, 4, 16, 1) == -1 and s("U", -1, 4, 0.0, 0.0, P, 4, 16, 1) == -2
    assert s("U", 4, -1, 0.0, 0.0, P, 4, 16, 1) == -3 and s("U", 4, 4, 0.0, 0.0, P, 3, 16, 1) == -7
    assert s("U", 4, 4, 0.0, 0.0, P, 4, 15, 2) == -8 and s("U", 4, 4, 0.0, 0.0, P, 4, 16, -1) == -9
    assert s("U", 4, 4, 0.0, 0.0, None, 4, 16, 1) == -6 and s("L", 0, 4, 0.0, 0.0, None, 1, 0, 1) == 0
    t = L.dlaset_batched
    assert t("q", 4, 4, 0.0, 0.0, P, 4, 1) == -1 and t("A", 4, 4, 0.0, 0.0, None, 4, 1) == -6
    assert t("A", 4, 4, 0.0, 0.0, P, 4, -1) == -8


def test_plan_options_errors(L):
    import ctypes
    h = ctypes.c_void_p()
    bad = ctypes.c_int64(-1)
    arr = L.problems_array([dict(op=7)])
    opt = L.PlanOptions(16, 5)
    vp = lambda x: ctypes.cast(x, ctypes.c_void_p)  # noqa: E731
    assert L.lib.mb_plan_create_ex(vp(arr), 1, vp(ctypes.pointer(opt)), ctypes.byref(h),
                                   ctypes.byref(bad)) == -3
    assert L.lib.mb_plan_create_ex(vp(arr), 1, None, None, None) == -4
    st, hd, idx = L.plan_create(arr, tile_two_min=32, potrf_waves=2)
    assert (st, hd, idx) == (L.MB_ERR_INVALID_PROBLEM, None, 0)


def test_variant_range_and_skinny_dispatch(L):
    """Forced families 0..3 are accepted, 4 is not (position 18 of the _ex
    call); the shape-aware dispatch names a kernel for thin, flat and small
    results without a GPU."""
    base = ("N", "N", 4, 4, 4, 1.0, P, 4, 16, P, 4, 16, 1.0, P, 4, 16, 0)
    assert L.dgemm_strided_batched(*base, 0, L.VARIANT_REGTILE) == 0  # batch 0: quick return
    assert L.dgemm_strided_batched(*base, 0, 4) == -18
    for (m, n, k) in ((4, 300, 300), (300, 4, 300), (4, 4, 300), (300, 300, 300)):
        name = L.dgemm_kernel_name("T", "N", m, n, k)
        assert name.startswith("gemm_"), name
    assert L.dgemm_kernel_name("N", "N", 4, 300, 300, L.VARIANT_REGTILE) == "gemm_regtile_t12"
    assert L.dgemm_kernel_name("N", "N", 300, 4, 300, L.VARIANT_REGTILE) == "gemm_regtile_t21"
    assert L.dgemm_select("N", "N", 4, 300, 300) in (1, 2, 3)


def test_riccati_argument_errors(L):
    """Each illegal argument of mb_riccati_strided_batched returns its
    position before anything is queried or launched; batch 0 returns MB_OK."""
    nx, nu, N, b = 8, 4, 3, 2
    m = nx + nu
    sf = m * m
    ok = dict(nx=nx, nu=nu, N=N, BAt=P, ldbat=m, stBAt=m * nx, sBAt=N * m * nx, RSQ=P, ldrsq=m,
              stRSQ=sf, sRSQ=N * sf, QN=P, ldq=nx, sQ=nx * nx, F=P, ldf=m, stF=sf, sF=N * sf,
              LN=P, ldl=nx, sL=nx * nx, info=P, work=P, work_bytes=1 << 20, batch=b, stream=None)
    order = list(ok)

    def call(**kw):
        a = dict(ok)
        a.update(kw)
        return L.riccati_strided_batched(*[a[k] for k in order])

    bad = [("nx", -1, -1), ("nu", -1, -2), ("N", -1, -3), ("ldbat", m - 1, -5), ("stBAt", -1, -6),
           ("sBAt", -1, -7), ("ldrsq", m - 1, -9), ("stRSQ", -1, -10), ("sRSQ", -1, -11),
           ("ldq", nx - 1, -13), ("sQ", -1, -14), ("ldf", m - 1, -16), ("stF", sf - 1, -17),
           ("sF", N * sf - 1, -18), ("ldl", nx - 1, -20), ("sL", nx * nx - 1, -21),
           ("batch", -1, -25), ("BAt", None, -4), ("RSQ", None, -8), ("QN", None, -12),
           ("F", None, -15), ("LN", None, -19), ("info", None, -22), ("work", None, -23),
           ("work_bytes", 2047, -24)]
    for key, val, want in bad:
        assert call(**{key: val}) == want, (key, val)
    assert call(batch=0) == 0
    assert call(nx=300, nu=5, ldbat=305, ldrsq=305, ldq=300, ldf=305, ldl=300, stF=305 * 305,
                sF=N * 305 * 305, sL=300 * 300) == L.MB_ERR_UNSUPPORTED
    # input strides may be 0 (time-invariant stages, shared inputs)
    assert call(stBAt=0, sBAt=0, stRSQ=0, sRSQ=0, sQ=0, batch=0) == 0
    st, _ = L.riccati_workspace_size(-1, 0, 1)
    assert st == -1
    assert L.riccati_workspace_size(4, -1, 1)[0] == -2
    assert L.riccati_workspace_size(4, 1, -1)[0] == -3
    assert L.lib.mb_riccati_workspace_size(4, 1, 1, None) == -4
    assert L.riccati_workspace_size(300, 5, 1)[0] == L.MB_ERR_UNSUPPORTED


def test_riccati_noalloc_argument_errors(L):
    """The allocation-free Riccati entry point validates like the workspace
    one (without work / work_bytes: batch is argument 23) before it touches
    the device scratch; batch 0 and nx + nu > 304 return before it too."""
    nx, nu, N, b = 8, 4, 3, 2
    m = nx + nu
    sf = m * m
    ok = dict(nx=nx, nu=nu, N=N, BAt=P, ldbat=m, stBAt=m * nx, sBAt=N * m * nx, RSQ=P, ldrsq=m,
              stRSQ=sf, sRSQ=N * sf, QN=P, ldq=nx, sQ=nx * nx, F=P, ldf=m, stF=sf, sF=N * sf,
              LN=P, ldl=nx, sL=nx * nx, info=P, batch=b, stream=None)
    order = list(ok)

    def call(**kw):
        a = dict(ok)
        a.update(kw)
        return L.riccati_strided_batched_noalloc(*[a[k] for k in order])

    bad = [("nx", -1, -1), ("nu", -1, -2), ("N", -1, -3), ("ldbat", m - 1, -5), ("stBAt", -1, -6),
           ("sBAt", -1, -7), ("ldrsq", m - 1, -9), ("stRSQ", -1, -10), ("sRSQ", -1, -11),
           ("ldq", nx - 1, -13), ("sQ", -1, -14), ("ldf", m - 1, -16), ("stF", sf - 1, -17),
           ("sF", N * sf - 1, -18), ("ldl", nx - 1, -20), ("sL", nx * nx - 1, -21),
           ("batch", -1, -23), ("BAt", None, -4), ("RSQ", None, -8), ("QN", None, -12),
           ("F", None, -15), ("LN", None, -19), ("info", None, -22)]
    for key, val, want in bad:
        assert call(**{key: val}) == want, (key, val)
    assert call(batch=0) == 0
    assert call(nx=300, nu=5, ldbat=305, ldrsq=305, ldq=300, ldf=305, ldl=300, stF=305 * 305,
                sF=N * 305 * 305, sL=300 * 300) == L.MB_ERR_UNSUPPORTED
    assert "scratch" in L.status_string(L.MB_ERR_SCRATCH)


def test_trmm_syrk_argument_errors(L):
    """Illegal arguments of the batched dtrmm_rlnn and dsyrk_ln return their
    positions; quick returns succeed without a GPU."""
    t = lambda *a: L.dtrmm_rlnn_strided_batched(*a)  # noqa: E731
    ok = [5, 4, 1.0, P, 4, 16, P, 5, 20, 2, None]
    for pos, val in ((0, -1), (1, -1), (4, 3), (5, -1), (7, 4), (8, 19), (9, -1)):
        a = list(ok)
        a[pos] = val
        assert t(*a) == -(pos + 1), (pos, val)
    for pos in (3, 6):
        a = list(ok)
        a[pos] = None
        assert t(*a) == -(pos + 1)
    assert t(0, 4, 1.0, None, 4, 0, None, 1, 0, 3, None) == 0
    assert t(5, 4, 1.0, P, 4, 16, P, 5, 20, 0, None) == 0
    s = lambda *a: L.dsyrk_ln_strided_batched(*a)  # noqa: E731
    ok = [6, 3, 1.0, P, 6, 18, 0.5, P, 6, 36, 2, None]
    for pos, val in ((0, -1), (1, -1), (4, 5), (5, -1), (8, 5), (9, 35), (10, -1)):
        a = list(ok)
        a[pos] = val
        assert s(*a) == -(pos + 1), (pos, val)
    for pos in (3, 7):
        a = list(ok)
        a[pos] = None
        assert s(*a) == -(pos + 1)
    assert s(6, 3, 0.0, None, 6, 18, 1.0, None, 6, 36, 2, None) == 0   # alpha 0, beta 1
    assert s(6, 0, 1.0, None, 6, 18, 1.0, None, 6, 36, 2, None) == 0   # k 0, beta 1
    assert s(0, 3, 1.0, None, 1, 0, 0.0, None, 1, 0, 2, None) == 0


def test_fortran_style_aliases_arguments(L):
    """mb_dgemm_ / mb_dpotrf_: a NULL scalar pointer is an illegal value of
    that argument; other checks and quick returns are those of the plain calls."""
    ok = ["N", "N", 4, 4, 4, 1.0, P, 4, P, 4, 1.0, P, 4]
    for pos in (0, 1, 2, 3, 4, 5, 7, 9, 10, 12):
        a = list(ok)
        a[pos] = None
        assert L.dgemm_fortran(*a) == -(pos + 1), pos
    a = list(ok)
    a[2] = -1
    assert L.dgemm_fortran(*a) == -3
    a = list(ok)
    a[0] = "X"
    assert L.dgemm_fortran(*a) == -1
    assert L.dgemm_fortran("N", "N", 0, 4, 4, 1.0, None, 1, None, 4, 1.0, None, 1) == 0
    assert L.dpotrf_fortran(None, 4, P, 4, P) == -1
    assert L.dpotrf_fortran("L", None, P, 4, P) == -2
    assert L.dpotrf_fortran("L", 4, P, None, P) == -4
    assert L.dpotrf_fortran("L", -1, P, 4, P) == -2
    assert L.dpotrf_fortran("L", 4, P, 3, P) == -4
    assert L.dpotrf_fortran("U", 4, P, 4, P) == L.MB_ERR_UNSUPPORTED


def test_ceiling_probe_argument_errors(L):
    """mb_ceiling_fp64 validates every argument (its position) before launching."""
    import ctypes
    fl = ctypes.c_double(0.0)
    buf = ctypes.c_void_p(16)  # never dereferenced: every call below fails its checks first
    assert L.lib.mb_ceiling_fp64(2, 1, 1, buf, ctypes.byref(fl), None) == -1
    assert L.lib.mb_ceiling_fp64(0, 0, 1, buf, ctypes.byref(fl), None) == -2
    assert L.lib.mb_ceiling_fp64(1, 1, 0, buf, ctypes.byref(fl), None) == -3
    assert L.lib.mb_ceiling_fp64(0, 1, 1, None, ctypes.byref(fl), None) == -4
    assert L.lib.mb_ceiling_fp64(0, 1, 1, buf, None, None) == -5


def test_hbm_ceiling_probe_argument_errors(L):
    """mb_ceiling_hbm validates every argument (its position) before launching."""
    import ctypes
    by = ctypes.c_double(0.0)
    pb = ctypes.byref(by)
    buf = ctypes.c_void_p(16)  # never dereferenced: every call below fails its checks first
    assert L.lib.mb_ceiling_hbm(3, buf, buf, 2, 1, buf, pb, None) == -1
    assert L.lib.mb_ceiling_hbm(0, None, buf, 2, 1, buf, pb, None) == -2
    assert L.lib.mb_ceiling_hbm(1, buf, None, 2, 1, buf, pb, None) == -3
    assert L.lib.mb_ceiling_hbm(2, buf, None, 2, 1, buf, pb, None) == -3
    assert L.lib.mb_ceiling_hbm(1, buf, buf, 0, 1, buf, pb, None) == -4
    assert L.lib.mb_ceiling_hbm(1, buf, buf, 3, 1, buf, pb, None) == -4
    assert L.lib.mb_ceiling_hbm(1, buf, buf, 2, 0, buf, pb, None) == -5
    assert L.lib.mb_ceiling_hbm(0, buf, None, 2, 1, None, pb, None) == -6
    assert L.lib.mb_ceiling_hbm(0, buf, None, 2, 1, buf, None, None) == -7


def test_tuned_tables_parse_and_tiny_dispatch(L):
    """The committed dispatch tables parse back (the autotuner keeps their
    choices within its noise margin) and re-emit byte for byte; results of at
    most 4 x 4 take the tiny table's choice, 16 x 16 the m, n <= 16 table's."""
    from paper_1902_08115_amd import autotune
    path = os.path.join(ROOT, "paper_1902_08115_amd", "csrc", "gemm_tuned.h")
    sq, sk = autotune.committed_tables(path)
    assert sq is not None and len(sk) == 4
    assert autotune.header(sq, sk) == open(path).read()
    for t in autotune.TRANS:
        for k in (1, 4, 8, 12, 16, 24, 300):
            e = autotune.class_index(k)
            assert L.dgemm_select(t[0], t[1], 4, 4, k) == sk[3][t][e][0], (t, k)
            assert L.dgemm_select(t[0], t[1], 3, 2, k) == sk[3][t][e][0], (t, k)
            assert L.dgemm_select(t[0], t[1], 16, 16, k) == sk[0][t][e][0], (t, k)
            assert L.dgemm_select(t[0], t[1], 16, 5, k) == sk[0][t][e][0], (t, k)
