"""GPU parity of the batched dgemm path against the CPU oracle, through the C ABI.

Element-by-element at sizes the oracle finishes quickly (several tiles plus
ragged tails, every trans case, both kernel families), bit-exact on integer
data, and sampled at the full benchmark batch sizes in the launch
configuration the benchmark times."""
import itertools

import numpy as np
import pytest

from paper_1902_08115_amd import inputs
from tests.gpu_util import (GEMM_TOL, dev, gemm_dims, gemm_errors, host, oracle_gemm_batch, say,
                            torch_mods)

pytestmark = pytest.mark.gpu

TRANS = ["NN", "NT", "TN", "TT"]
VARIANTS = {"direct": 1, "packed": 2, "auto": 0, "regtile": 3}


def _make(g, ta, tb, m, n, k, batch, pad=0, gap=0, integer=False):
    (ar, ac), (br, bc) = gemm_dims(ta, tb, m, n, k)
    A = inputs.colmajor(g, batch, ar, ac + gap, max(1, ar + pad), integer=integer, low=-4, high=4) \
        if integer else inputs.colmajor(g, batch, ar, ac + gap, max(1, ar + pad))
    B = inputs.colmajor(g, batch, br, bc + gap, max(1, br + pad), integer=integer, low=-4, high=4) \
        if integer else inputs.colmajor(g, batch, br, bc + gap, max(1, br + pad))
    C = inputs.colmajor(g, batch, m, n + gap, max(1, m + pad), integer=integer, low=-4, high=4) \
        if integer else inputs.colmajor(g, batch, m, n + gap, max(1, m + pad))
    return A, B, C


def _run_strided(ta, tb, m, n, k, alpha, A, B, beta, C, batch, variant):
    torch, _lib, _ = torch_mods()
    dA, dB, dC = dev(A), dev(B), dev(C)
    st = _lib.dgemm_strided_batched(
        ta, tb, m, n, k, alpha, dA.data_ptr(), A.shape[2], A.shape[1] * A.shape[2],
        dB.data_ptr(), B.shape[2], B.shape[1] * B.shape[2], beta, dC.data_ptr(), C.shape[2],
        C.shape[1] * C.shape[2], batch, torch.cuda.current_stream().cuda_stream, variant)
    assert st == 0, st
    return host(dC).reshape(C.shape)


def test_single_call_32():
    """One plain dgemm NN, m=n=k=32, alpha=beta=1, U[-1,1) entries."""
    torch, _lib, _ = torch_mods()
    g = inputs.rng(inputs.seed_for(0, 0))
    A, B, C = _make(g, "N", "N", 32, 32, 32, 1)
    dA, dB, dC = dev(A), dev(B), dev(C)
    say("single dgemm NN 32")
    st = _lib.dgemm("N", "N", 32, 32, 32, 1.0, dA.data_ptr(), 32, dB.data_ptr(), 32, 1.0,
                    dC.data_ptr(), 32, torch.cuda.current_stream().cuda_stream)
    assert st == 0
    Cg = host(dC).reshape(C.shape)
    Cr = oracle_gemm_batch("N", "N", 32, 32, 32, 1.0, A, 32, B, 32, 1.0, C, 32, 1)
    e1, e2 = gemm_errors(Cg, Cr, A, B, C, "N", "N", 32, 32, 32, 1.0, 1.0)
    assert e1 <= GEMM_TOL and e2 <= GEMM_TOL, (e1, e2)


EXACT_SHAPES = [(1, 1, 1), (4, 4, 4), (5, 7, 3), (8, 8, 8), (13, 9, 21), (16, 16, 16),
                (17, 33, 19), (32, 32, 32), (31, 48, 70), (64, 64, 64), (65, 97, 33),
                (130, 70, 129)]


@pytest.mark.parametrize("variant", ["direct", "packed", "auto", "regtile"])
@pytest.mark.parametrize("trans", TRANS)
def test_integer_exact(trans, variant):
    """Integer entries in [-4, 4]: every partial sum is exact, so the GPU result
    must equal the oracle bit for bit; NaN sentinels in ld padding and in the
    gaps between instances must survive."""
    ta, tb = trans
    g = inputs.rng(7000 + TRANS.index(trans))
    for (m, n, k), (alpha, beta) in zip(EXACT_SHAPES, itertools.cycle(
            [(1.0, 1.0), (-0.5, 2.0), (2.0, 0.0), (1.0, -1.0)])):
        pad, gap, batch = (m + n) % 3, 1, 3
        A, B, C = _make(g, ta, tb, m, n, k, batch, pad=pad, gap=gap, integer=True)
        if beta == 0.0:
            C[:, :, :m] = np.nan  # beta == 0 must not read C
        say(f"dgemm exact {trans} {variant} m={m} n={n} k={k} alpha={alpha} beta={beta}")
        Cg = _run_strided(ta, tb, m, n, k, alpha, A, B, beta, C, batch, VARIANTS[variant])
        Cr = oracle_gemm_batch(ta, tb, m, n, k, alpha, A, A.shape[2], B, B.shape[2], beta, C,
                               C.shape[2], batch)
        assert np.array_equal(Cg, Cr, equal_nan=True), f"m={m} n={n} k={k}"


@pytest.mark.parametrize("variant", ["direct", "packed", "regtile"])
@pytest.mark.parametrize("trans", TRANS)
def test_random_sweep_sizes(trans, variant):
    """U[-1,1) data at every sweep size (small batch): both error gates."""
    ta, tb = trans
    for si, n in enumerate(inputs.GEMM_SWEEP_SIZES):
        g = inputs.rng(inputs.seed_for(1, si))
        batch = 3
        A, B, C = _make(g, ta, tb, n, n, n, batch)
        say(f"dgemm random {trans} {variant} n={n}")
        Cg = _run_strided(ta, tb, n, n, n, 1.0, A, B, 1.0, C, batch, VARIANTS[variant])
        Cr = oracle_gemm_batch(ta, tb, n, n, n, 1.0, A, n, B, n, 1.0, C, n, batch)
        e1, e2 = gemm_errors(Cg, Cr, A, B, C, ta, tb, n, n, n, 1.0, 1.0)
        assert e1 <= GEMM_TOL and e2 <= GEMM_TOL, (n, e1, e2)


@pytest.mark.parametrize("trans", TRANS)
def test_batched_equals_single_calls(trans):
    """A strided batch equals a loop of plain calls, bit for bit."""
    torch, _lib, _ = torch_mods()
    ta, tb = trans
    g = inputs.rng(7100)
    for (m, n, k) in [(4, 4, 4), (24, 20, 28), (96, 96, 96)]:
        batch = 5
        A, B, C = _make(g, ta, tb, m, n, k, batch, pad=1)
        say(f"dgemm batch-vs-single {trans} {m}x{n}x{k}")
        Cb = _run_strided(ta, tb, m, n, k, 0.75, A, B, -1.5, C, batch, 0)
        dA, dB, dC = dev(A), dev(B), dev(C)
        sA, sB, sC = (X.shape[1] * X.shape[2] for X in (A, B, C))
        s = torch.cuda.current_stream().cuda_stream
        for b in range(batch):
            st = _lib.dgemm(ta, tb, m, n, k, 0.75, dA.data_ptr() + 8 * b * sA, A.shape[2],
                            dB.data_ptr() + 8 * b * sB, B.shape[2], -1.5,
                            dC.data_ptr() + 8 * b * sC, C.shape[2], s)
            assert st == 0
        Cs = host(dC).reshape(C.shape)
        assert np.array_equal(Cb, Cs, equal_nan=True)


@pytest.mark.parametrize("variant", ["direct", "packed", "auto", "regtile"])
def test_pointer_array_equals_strided(variant):
    torch, _lib, _ = torch_mods()
    g = inputs.rng(7200)
    for trans, (m, n, k) in zip(TRANS, [(6, 5, 7), (33, 17, 40), (64, 64, 64), (100, 80, 90)]):
        ta, tb = trans
        batch = 4
        A, B, C = _make(g, ta, tb, m, n, k, batch, pad=2, gap=1)
        say(f"dgemm pointer-array {trans} {variant} {m}x{n}x{k}")
        Cs = _run_strided(ta, tb, m, n, k, 1.25, A, B, 0.5, C, batch, VARIANTS[variant])
        dA, dB, dC = dev(A), dev(B), dev(C)
        ptr = [torch.tensor([d.data_ptr() + 8 * b * X.shape[1] * X.shape[2] for b in range(batch)],
                            dtype=torch.int64, device="cuda") for d, X in ((dA, A), (dB, B), (dC, C))]
        st = _lib.dgemm_batched(ta, tb, m, n, k, 1.25, ptr[0].data_ptr(), A.shape[2],
                                ptr[1].data_ptr(), B.shape[2], 0.5, ptr[2].data_ptr(), C.shape[2],
                                batch, torch.cuda.current_stream().cuda_stream, VARIANTS[variant])
        assert st == 0
        Cp = host(dC).reshape(C.shape)
        assert np.array_equal(Cs, Cp, equal_nan=True)


def test_special_scalars_and_quick_returns():
    torch, _lib, _ = torch_mods()
    g = inputs.rng(7300)
    m, n, k, batch = 9, 7, 5, 2
    A, B, C = _make(g, "N", "N", m, n, k, batch, pad=1)
    s = torch.cuda.current_stream().cuda_stream
    An = np.full_like(A, np.nan)
    # alpha == 0: A, B not read, C <= beta*C
    say("dgemm alpha=0 beta=2")
    Cg = _run_strided("N", "N", m, n, k, 0.0, An, An, 2.0, C, batch, 0)
    exp = C.copy()
    exp[:, :, :m] *= 2.0
    assert np.array_equal(Cg, exp, equal_nan=True)
    # alpha == 0, beta == 0: zeros, C not read
    Cn = C.copy()
    Cn[:, :, :m] = np.nan
    say("dgemm alpha=0 beta=0")
    Cg = _run_strided("N", "N", m, n, k, 0.0, An, An, 0.0, Cn, batch, 0)
    exp = Cn.copy()
    exp[:, :, :m] = 0.0
    assert np.array_equal(Cg, exp, equal_nan=True)
    # k == 0 with beta = -1: C <= -C
    say("dgemm k=0")
    Cg = _run_strided("N", "N", m, n, 0, 1.0, An, An, -1.0, C, batch, 0)
    exp = C.copy()
    exp[:, :, :m] *= -1.0
    assert np.array_equal(Cg, exp, equal_nan=True)
    # quick returns leave C bit-identical (NaN included) and launch nothing
    dC = dev(Cn)
    for args in [(0, n, k, 1.0, 1.0), (m, 0, k, 1.0, 1.0), (m, n, k, 0.0, 1.0), (m, n, 0, 1.0, 1.0)]:
        mm, nn, kk, al, be = args
        st = _lib.dgemm_strided_batched("N", "N", mm, nn, kk, al, 0, max(1, mm), 0, 0, max(1, kk),
                                        0, be, dC.data_ptr(), max(1, m + 1), 0, 1, s)
        assert st == 0
    st = _lib.dgemm_strided_batched("N", "N", m, n, k, 1.0, 0, m + 1, 0, 0, k + 1, 0, 1.0,
                                    dC.data_ptr(), m + 1, 0, 0, s)  # batch == 0
    assert st == 0
    assert np.array_equal(host(dC).reshape(Cn.shape), Cn, equal_nan=True)


def test_deterministic():
    """Two runs of the same call give bit-identical results (no atomics)."""
    g = inputs.rng(7400)
    for (n, v) in [(8, 1), (64, 2), (200, 2)]:
        A, B, C = _make(g, "T", "N", n, n, n, 4)
        say(f"dgemm determinism n={n}")
        c1 = _run_strided("T", "N", n, n, n, 1.0, A, B, 1.0, C, 4, v)
        c2 = _run_strided("T", "N", n, n, n, 1.0, A, B, 1.0, C, 4, v)
        assert np.array_equal(c1, c2)


@pytest.mark.parametrize("trans", TRANS)
def test_full_batch_sampled(trans):
    """Full benchmark batches (A+B+C ~ 1 GiB per size, inputs generated in
    device memory), auto variant as the benchmark runs it; sampled instances
    against the oracle."""
    torch, _lib, blas = torch_mods()
    import oracle
    ta, tb = trans
    s = torch.cuda.current_stream().cuda_stream
    for si, n in enumerate(inputs.GEMM_SWEEP_SIZES):
        batch = inputs.gemm_sweep_batch(n)
        seed = inputs.seed_for(1, si) + 100 * TRANS.index(trans)
        A = inputs.torch_colmajor(batch, n, n, seed=seed)
        B = inputs.torch_colmajor(batch, n, n, seed=seed + 1)
        C = inputs.torch_colmajor(batch, n, n, seed=seed + 2)
        rs = np.random.Generator(np.random.PCG64(seed))
        idx = sorted({0, batch - 1, *rs.integers(0, batch, size=6).tolist()})
        sel = torch.tensor(idx, device="cuda")
        A0 = A[sel].contiguous().cpu().numpy()  # (s, n, n) row-major copies of the matrices
        B0 = B[sel].contiguous().cpu().numpy()
        C0 = C[sel].contiguous().cpu().numpy()
        say(f"dgemm full batch {trans} n={n} batch={batch}")
        st = _lib.dgemm_strided_batched(ta, tb, n, n, n, 1.0, A.data_ptr(), n, n * n,
                                        B.data_ptr(), n, n * n, 1.0, C.data_ptr(), n, n * n,
                                        batch, s)
        assert st == 0
        Cg = C[sel].contiguous().cpu().numpy()
        for j in range(len(idx)):
            Af = np.asfortranarray(A0[j])
            Bf = np.asfortranarray(B0[j])
            Cr = np.asfortranarray(C0[j].copy())
            oracle.dgemm(ta, tb, 1.0, Af, Bf, 1.0, Cr)
            err = np.linalg.norm(Cg[j] - Cr) / np.linalg.norm(Cr)
            scale = np.linalg.norm(Af) * np.linalg.norm(Bf) + np.linalg.norm(C0[j])
            assert err <= GEMM_TOL, (n, idx[j], err)
            assert np.linalg.norm(Cg[j] - Cr) / scale <= GEMM_TOL
        del A, B, C
        torch.cuda.empty_cache()


def test_every_packed_config_exact():
    """Every configuration of the packed kernel menu (the autotuner's search
    space), every trans case, ragged shapes spanning several tiles and panels:
    bit-exact on integer data; 8-byte-load path via odd leading dimensions."""
    torch, _lib, _ = torch_mods()
    s = torch.cuda.current_stream().cuda_stream
    g = inputs.rng(7500)
    for cfg in range(_lib.dgemm_config_count()):
        name = _lib.dgemm_config_name(cfg)
        lim = min(300, _lib.dgemm_config_max_mn(cfg))
        # k = 53: an odd number of full panels before the last one (both panel depths)
        shapes = [(min(lim, 13), min(lim, 9), 37), (lim, lim, 16), (min(lim, 150), min(lim, 70), 45),
                  (min(lim, 40), min(lim, 33), 53)]
        for trans in TRANS:
            ta, tb = trans
            for (m, n, k), pad in zip(shapes, (0, 1, 0, 1)):
                batch = 2
                A, B, C = _make(g, ta, tb, m, n, k, batch, pad=pad, gap=1, integer=True)
                dA, dB, dC = dev(A), dev(B), dev(C)
                say(f"dgemm config {name} {trans} {m}x{n}x{k} pad={pad}")
                st = _lib.dgemm_strided_batched_config(
                    ta, tb, m, n, k, 1.0, dA.data_ptr(), A.shape[2], A.shape[1] * A.shape[2],
                    dB.data_ptr(), B.shape[2], B.shape[1] * B.shape[2], -0.5, dC.data_ptr(),
                    C.shape[2], C.shape[1] * C.shape[2], batch, cfg, s)
                assert st == 0, (name, st)
                Cg = host(dC).reshape(C.shape)
                Cr = oracle_gemm_batch(ta, tb, m, n, k, 1.0, A, A.shape[2], B, B.shape[2], -0.5,
                                       C, C.shape[2], batch)
                assert np.array_equal(Cg, Cr, equal_nan=True), (name, trans, m, n, k)
    # a WAVE configuration refuses an instance larger than its tile
    assert _lib.dgemm_strided_batched_config("N", "N", 17, 17, 4, 1.0, 16, 17, 289, 16, 4, 68,
                                             0.0, 16, 17, 289, 1, 0, s) == _lib.MB_ERR_UNSUPPORTED


@pytest.mark.parametrize("trans", ["NN", "TT"])
def test_packed_huge_leading_dimension(trans):
    """A leading dimension above 2^21 is beyond the packed kernel's 32-bit
    buffer offsets: the launcher falls back to 64-bit addressing.  A alone
    has the huge stride (about 1.2 GB on the device); bit-exact on integer
    data against the oracle on the compact operands."""
    torch, _lib, _ = torch_mods()
    s = torch.cuda.current_stream().cuda_stream
    ta, tb = trans
    m, n, k = 70, 37, 45
    g = inputs.rng(7600 + TRANS.index(trans))
    A, B, C = _make(g, ta, tb, m, n, k, 1, integer=True)
    ar, ac = A.shape[2], A.shape[1]
    lda = (1 << 21) + 8
    big = torch.full((ac, lda), float("nan"), dtype=torch.float64, device="cuda")
    big[:, :ar] = torch.from_numpy(A[0]).cuda()
    dB, dC = dev(B), dev(C)
    say(f"dgemm huge lda={lda} {trans} {m}x{n}x{k}")
    st = _lib.dgemm_strided_batched_config(ta, tb, m, n, k, 1.0, big.data_ptr(), lda, ac * lda,
                                           dB.data_ptr(), B.shape[2], B.shape[1] * B.shape[2],
                                           -0.5, dC.data_ptr(), C.shape[2],
                                           C.shape[1] * C.shape[2], 1, 5, s)
    assert st == 0, st
    Cg = host(dC).reshape(C.shape)
    Cr = oracle_gemm_batch(ta, tb, m, n, k, 1.0, A, ar, B, B.shape[2], -0.5, C, C.shape[2], 1)
    assert np.array_equal(Cg, Cr, equal_nan=True)
    del big
    torch.cuda.empty_cache()


@pytest.mark.parametrize("huge", ["A", "B"])
@pytest.mark.parametrize("config", [5, 15])
def test_packed_record_count_at_largest_buffer_ld(huge, config):
    """An operand whose rows are contiguous ('N' A, 'T' B) bounds k by the
    record count of its panel's buffer resource, (k - kb) ld 8 bytes, capped
    just under 2 GiB.  At ld = 2^21 (the largest on the buffer path) and
    k = 200 the full panels take the capped count and the last, partial panel
    the exact one; the columns past k hold NaN.  Bit-exact on integer data."""
    torch, _lib, _ = torch_mods()
    s = torch.cuda.current_stream().cuda_stream
    ta, tb = ("N", "N") if huge == "A" else ("T", "T")
    m, n, k = 70, 37, 200
    g = inputs.rng(7700 + config + (0 if huge == "A" else 1))
    A, B, C = _make(g, ta, tb, m, n, k, 1, integer=True)
    ld = 1 << 21
    X = A if huge == "A" else B
    rows, cols = X.shape[2], X.shape[1]
    big = torch.full((cols + 1, ld), float("nan"), dtype=torch.float64, device="cuda")
    big[:cols, :rows] = torch.from_numpy(X[0]).cuda()
    dA = big if huge == "A" else dev(A)
    dB = big if huge == "B" else dev(B)
    lda = ld if huge == "A" else A.shape[2]
    ldb = ld if huge == "B" else B.shape[2]
    dC = dev(C)
    say(f"dgemm record count ld={ld} huge {huge} {ta}{tb} {m}x{n}x{k} config {config}")
    st = _lib.dgemm_strided_batched_config(ta, tb, m, n, k, 1.0, dA.data_ptr(), lda,
                                           A.shape[1] * lda, dB.data_ptr(), ldb,
                                           B.shape[1] * ldb, -0.5, dC.data_ptr(), C.shape[2],
                                           C.shape[1] * C.shape[2], 1, config, s)
    assert st == 0, st
    Cg = host(dC).reshape(C.shape)
    Cr = oracle_gemm_batch(ta, tb, m, n, k, 1.0, A, A.shape[2], B, B.shape[2], -0.5, C,
                           C.shape[2], 1)
    assert np.array_equal(Cg, Cr, equal_nan=True)
    del big
    torch.cuda.empty_cache()


SKINNY = [(4, 4, 1), (4, 4, 2), (4, 4, 3), (4, 4, 17), (4, 4, 300), (1, 300, 5), (4, 300, 300),
          (4, 37, 200), (16, 17, 33), (300, 4, 300), (97, 4, 15), (17, 16, 9), (3, 5, 300),
          (16, 16, 257), (33, 2, 64), (2, 3, 8), (4, 4, 12)]


@pytest.mark.parametrize("variant", ["auto", "regtile"])
@pytest.mark.parametrize("trans", TRANS)
def test_skinny_shapes(trans, variant):
    """Thin, flat and small results with long and short k (the paper's skinny
    sweeps, App. C, plus ragged edges): bit-exact on integer data, NaN ld
    padding untouched, both through the shape-aware dispatch and forced onto
    the register-tile kernels."""
    ta, tb = trans
    g = inputs.rng(7700 + TRANS.index(trans))
    for (m, n, k), (alpha, beta) in zip(SKINNY, itertools.cycle([(1.0, 1.0), (-2.0, 0.5),
                                                                  (1.0, 0.0)])):
        A, B, C = _make(g, ta, tb, m, n, k, 3, pad=1, gap=1, integer=True)
        if beta == 0.0:
            C[:, :, :m] = np.nan
        say(f"dgemm skinny {trans} {variant} m={m} n={n} k={k} "
            f"[{_lib_name(ta, tb, m, n, k)}]")
        Cg = _run_strided(ta, tb, m, n, k, alpha, A, B, beta, C, 3, VARIANTS[variant])
        Cr = oracle_gemm_batch(ta, tb, m, n, k, alpha, A, A.shape[2], B, B.shape[2], beta, C,
                               C.shape[2], 3)
        assert np.array_equal(Cg, Cr, equal_nan=True), f"m={m} n={n} k={k}"


def _lib_name(ta, tb, m, n, k):
    from paper_1902_08115_amd import _lib
    return _lib.dgemm_kernel_name(ta, tb, m, n, k)


def test_fortran_alias_matches_plain():
    """mb_dgemm_ (scalars by pointer, null stream) matches mb_dgemm bit for bit
    in every trans case."""
    torch, _lib, _ = torch_mods()
    g = inputs.rng(9100)
    m, n, k = 23, 17, 29
    for ta in "NT":
        for tb in "NT":
            (ar, ac), (br, bc) = gemm_dims(ta, tb, m, n, k)
            A = inputs.colmajor(g, 1, ar, ac)
            B = inputs.colmajor(g, 1, br, bc)
            C = inputs.colmajor(g, 1, m, n)
            say(f"dgemm fortran alias {ta}{tb}")
            dA, dB = dev(A), dev(B)
            c1, c2 = dev(C), dev(C)
            assert _lib.dgemm(ta, tb, m, n, k, 0.5, dA.data_ptr(), ar, dB.data_ptr(), br, -1.5,
                              c1.data_ptr(), m, 0) == 0
            assert _lib.dgemm_fortran(ta, tb, m, n, k, 0.5, dA.data_ptr(), ar, dB.data_ptr(), br,
                                      -1.5, c2.data_ptr(), m) == 0
            torch.cuda.synchronize()
            assert torch.equal(c1, c2), (ta, tb)
