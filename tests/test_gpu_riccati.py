"""GPU parity of the batched factorized Riccati recursion (Sec. 5.2) against
the CPU oracle, through the C ABI.

Gates: info bit-exact; every stage factor F_n and the terminal factor within
RIC_TOL (normwise: max abs difference over max abs entry of the oracle's
factor); the stage backward error -- F_n F_n^T against RSQ_n + C C^T with
C = BAt_n Lc_{n+1} formed from the GPU's own previous factor -- within
RIC_TOL; strictly upper triangles untouched.  FP64 throughout; the two sides
sum in different orders, and the expected differences are ~1e-15."""
import numpy as np
import pytest

import oracle
from paper_1902_08115_amd import inputs
from tests.gpu_util import say, torch_mods

pytestmark = pytest.mark.gpu

RIC_TOL = 1e-12
SENTINEL = 7.25


def _gen(nx, nu, N, batch, seed):
    return inputs.torch_riccati(nx, nu, N, batch, seed, device="cuda")


def _outputs(torch, batch, N, m, nx):
    F = torch.full((batch, N, m, m), SENTINEL, dtype=torch.float64, device="cuda").transpose(2, 3)
    LN = torch.full((batch, nx, nx), SENTINEL, dtype=torch.float64, device="cuda").transpose(1, 2)
    info = torch.full((batch, N + 1), -7, dtype=torch.int32, device="cuda")
    return F, LN, info


def _np(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)) if a.size else 0.0


def _check_problem(BAt, RSQ, QN, nu, F, LN, info, tag):
    """One problem (host arrays in math layout) against the oracle."""
    N, m, nx = BAt.shape
    Fo, LNo, info_o = oracle.riccati(BAt, RSQ, QN, nu)
    assert np.array_equal(info, info_o), (tag, info, info_o)
    lo_x, lo_m = np.tril_indices(nx), np.tril_indices(m)
    up_x, up_m = np.triu_indices(nx, 1), np.triu_indices(m, 1)
    assert _rel(LN[lo_x], LNo[lo_x]) <= RIC_TOL, (tag, "LN", _rel(LN[lo_x], LNo[lo_x]))
    assert np.all(LN[up_x] == SENTINEL), (tag, "LN upper written")
    Lc = np.tril(LN)
    for n in range(N - 1, -1, -1):
        Fn = F[n]
        e = _rel(Fn[lo_m], Fo[n][lo_m])
        assert e <= RIC_TOL, (tag, n, e)
        assert np.all(Fn[up_m] == SENTINEL), (tag, n, "upper written")
        C = BAt[n] @ Lc
        M = np.tril(RSQ[n]) + np.tril(RSQ[n], -1).T + C @ C.T
        Ln = np.tril(Fn)
        res = _rel(Ln @ Ln.T, M)
        assert res <= RIC_TOL, (tag, n, "residual", res)
        Lc = Ln[nu:, nu:]


def _run(nx, nu, N, BAt, RSQ, QN, F, LN, info, work=None):
    torch, _lib, blas = torch_mods()
    return blas.riccati(BAt, RSQ, QN, nu, F=F, LN=LN, info=info, work=work)


@pytest.mark.parametrize("nx,nu,N,batch", [
    (8, 4, 10, 7), (24, 12, 10, 5), (40, 20, 4, 3), (64, 32, 3, 2),
    (1, 1, 4, 9), (5, 0, 3, 4), (17, 9, 5, 3), (3, 2, 1, 6), (6, 3, 0, 5), (16, 16, 2, 3),
    (33, 15, 2, 2), (0, 4, 3, 3), (70, 10, 2, 2), (50, 60, 2, 2),
])
def test_riccati_vs_oracle(nx, nu, N, batch):
    """Every stage of every problem, shapes spanning several 16 x 16 tiles with
    ragged edges, nu = 0, nx = 0, N = 0 and N = 1; every kernel of the
    recursion (one tile up to m = 16, registers up to m = 96 and nx = 64, the
    workspace kernel beyond: (70, 10) and (50, 60))."""
    torch, _lib, blas = torch_mods()
    m = nx + nu
    say(f"riccati nx={nx} nu={nu} N={N} batch={batch}")
    BAt, RSQ, QN = _gen(nx, nu, N, batch, inputs.seed_for(40, 100 * nx + nu))
    F, LN, info = _outputs(torch, batch, N, m, nx)
    _run(nx, nu, N, BAt, RSQ, QN, F, LN, info)
    Fh, LNh, infoh = _np(F), _np(LN), _np(info)
    Bh, Rh, Qh = _np(BAt), _np(RSQ), _np(QN)
    assert np.all(infoh == 0), infoh
    for b in range(batch):
        _check_problem(Bh[b], Rh[b], Qh[b], nu, Fh[b], LNh[b], infoh[b], f"b={b}")


@pytest.mark.parametrize("nx,nu", [(20, 7), (40, 20), (64, 32)])
def test_riccati_info_and_skipped_stages(nx, nu):
    """A stage that is not positive definite at column j: info = j + 1 there
    (bit-exact against the oracle), -1 and untouched output for the stages
    after it in the recursion, the columns before j still factor values; a
    non-SPD Q_N stops the whole recursion.  One shape per kernel family."""
    torch, _lib, blas = torch_mods()
    N, batch = 6, 5
    m = nx + nu
    say(f"riccati info nx={nx} nu={nu} N={N}")
    BAt, RSQ, QN = _gen(nx, nu, N, batch, inputs.seed_for(41, nx))
    cases = {0: (3, 0), 1: (0, m - 5), 2: (5, 17), 4: (2, 16)}
    for b, (stage, j) in cases.items():
        d = torch.arange(1.0, m + 1, dtype=torch.float64, device="cuda")
        d[j] = -1.0
        RSQ[b, stage] = torch.diag(d)
        BAt[b, stage, j, :] = 0.0
    QN[3, 4, 4] = -2.0
    F, LN, info = _outputs(torch, batch, N, m, nx)
    _run(nx, nu, N, BAt, RSQ, QN, F, LN, info)
    Fh, LNh, infoh = _np(F), _np(LN), _np(info)
    Bh, Rh, Qh = _np(BAt), _np(RSQ), _np(QN)
    for b in range(batch):
        Fo, LNo, info_o = oracle.riccati(Bh[b], Rh[b], Qh[b], nu)
        assert np.array_equal(infoh[b], info_o), (b, infoh[b], info_o)
        fail = [n for n in range(N + 1) if info_o[n] > 0]
        if b == 3:
            assert info_o.tolist() == [-1] * N + [5]
            assert np.all(Fh[b] == SENTINEL)
            continue
        assert len(fail) == 1
        s = fail[0]
        for n in range(s):
            assert np.all(Fh[b][n] == SENTINEL), (b, n)
        col = info_o[s] - 1
        for n in range(s, N):
            cols = col if n == s else m
            for c in range(cols):
                got, ref = Fh[b][n][c:, c], Fo[n][c:, c]
                assert _rel(got, ref) <= RIC_TOL or np.max(np.abs(got - ref)) <= 1e-13, (b, n, c)


@pytest.mark.parametrize("nx,nu", inputs.RICCATI_SHAPES)
def test_riccati_full_size_sampled(nx, nu):
    """The paper's four shapes at the benchmark's batch and launch
    configuration (full-occupancy workspace): every info zero, sampled
    problems (first, last and spread) against the oracle."""
    torch, _lib, blas = torch_mods()
    N, batch = inputs.RICCATI_N, inputs.RICCATI_BATCH[(nx, nu)]
    m = nx + nu
    say(f"riccati full nx={nx} nu={nu} N={N} batch={batch}")
    BAt, RSQ, QN = _gen(nx, nu, N, batch, inputs.seed_for(42, nx))
    F, LN, info = _outputs(torch, batch, N, m, nx)
    work = blas.riccati_workspace(nx, nu, batch)
    _run(nx, nu, N, BAt, RSQ, QN, F, LN, info, work=work)
    infoh = _np(info)
    assert np.all(infoh == 0)
    rng = inputs.rng(inputs.seed_for(42, 1000 + nx))
    sample = sorted(set([0, batch - 1] + rng.integers(0, batch, size=10).tolist()))
    for b in sample:
        _check_problem(_np(BAt[b]), _np(RSQ[b]), _np(QN[b]), nu, _np(F[b]), _np(LN[b]), infoh[b],
                       f"b={b}")
    del BAt, RSQ, QN, F, LN, work
    torch.cuda.empty_cache()


def test_riccati_workspace_inplace_and_broadcast():
    """Results do not depend on how many waves share the batch (one slot,
    three slots, full workspace: bit-identical); F may overwrite RSQ in place
    (bit-identical); time-invariant stages (stage stride 0) and inputs shared
    by all problems (problem stride 0) match the oracle."""
    torch, _lib, blas = torch_mods()
    nx, nu, N, batch = 24, 12, 5, 11
    m = nx + nu
    say(f"riccati workspace/in-place nx={nx} nu={nu} N={N} batch={batch}")
    BAt, RSQ, QN = _gen(nx, nu, N, batch, inputs.seed_for(43))
    slot = 2 * 1024 * ((m + 15) // 16) * ((nx + 15) // 16)
    outs = []
    for nslots in (1, 3, None):
        F, LN, info = _outputs(torch, batch, N, m, nx)
        work = (torch.empty(nslots * slot // 8, dtype=torch.float64, device="cuda")
                if nslots else None)
        _run(nx, nu, N, BAt, RSQ, QN, F, LN, info, work=work)
        outs.append((_np(F), _np(LN), _np(info)))
    for F, LN, info in outs[1:]:
        assert np.array_equal(F, outs[0][0]) and np.array_equal(LN, outs[0][1])
        assert np.array_equal(info, outs[0][2]) and np.all(info == 0)
    # in place: F = RSQ (upper triangles keep RSQ's values)
    R2 = RSQ.clone()
    F, LN, info = _outputs(torch, batch, N, m, nx)
    blas.riccati(BAt, R2, QN, nu, F=R2, LN=LN, info=info)
    R2h = _np(R2)
    lo = np.tril_indices(m)
    for b in range(batch):
        for n in range(N):
            assert np.array_equal(R2h[b, n][lo], outs[0][0][b, n][lo])
    # broadcast: one problem's stage 0 repeated over stages and problems
    Bb = BAt[0:1, 0:1].expand(batch, N, m, nx)
    Rb = RSQ[0:1, 0:1].expand(batch, N, m, m)
    Qb = QN[0:1].expand(batch, nx, nx)
    F, LN, info = _outputs(torch, batch, N, m, nx)
    blas.riccati(Bb, Rb, Qb, nu, F=F, LN=LN, info=info)
    Bh = np.repeat(_np(BAt[0, 0])[None], N, axis=0)
    Rh = np.repeat(_np(RSQ[0, 0])[None], N, axis=0)
    Fh, LNh, infoh = _np(F), _np(LN), _np(info)
    for b in (0, batch - 1):
        _check_problem(Bh, Rh, _np(QN[0]), nu, Fh[b], LNh[b], infoh[b], f"broadcast b={b}")


@pytest.mark.parametrize("m,n,alpha", [(12, 8, 1.0), (36, 24, -0.5), (96, 64, 1.0), (1, 1, 2.0),
                                       (17, 33, 1.0), (40, 5, 0.0), (0, 4, 1.0)])
def test_dtrmm_rlnn_vs_oracle(m, n, alpha):
    """Batched dtrmm_rlnn against the oracle: A's upper triangle (NaN) is
    never read, B's ld padding rows (NaN) never written, result within
    RIC_TOL normwise."""
    torch, _lib, blas = torch_mods()
    batch, lda, ldb = 5, n + 3, m + 2
    say(f"dtrmm_rlnn m={m} n={n} alpha={alpha}")
    g = inputs.rng(inputs.seed_for(44, m * 100 + n))
    A = g.uniform(-1, 1, size=(batch, max(n, 1), lda))
    B = g.uniform(-1, 1, size=(batch, max(n, 1), ldb))
    for b in range(batch):
        for j in range(n):
            A[b, j, :j] = np.nan          # strictly upper part of column j
            A[b, j, n:] = np.nan
        B[b, :, m:] = np.nan
    dA = torch.from_numpy(A.copy()).cuda()
    dB = torch.from_numpy(B.copy()).cuda()
    st = _lib.dtrmm_rlnn_strided_batched(m, n, alpha, dA.data_ptr(), lda, A[0].size, dB.data_ptr(),
                                         ldb, B[0].size, batch,
                                         torch.cuda.current_stream().cuda_stream)
    assert st == 0
    got = _np(dB)
    for b in range(batch):
        Bo = np.asfortranarray(B[b].T[:m, :n])
        Ao = np.asfortranarray(A[b].T[:n, :n])
        oracle.dtrmm_rlnn(alpha, Ao, Bo)
        g_b = got[b].T
        assert np.all(np.isnan(g_b[m:, :n])), "padding written"
        assert _rel(g_b[:m, :n], Bo) <= RIC_TOL or np.max(np.abs(g_b[:m, :n] - Bo)) == 0.0


@pytest.mark.parametrize("n,k,alpha,beta", [(12, 8, 1.0, 1.0), (36, 24, -1.0, 0.5),
                                            (96, 64, 1.0, 1.0), (33, 17, 2.0, 0.0),
                                            (5, 0, 1.0, 2.0), (20, 3, 0.0, -1.0), (1, 1, 1.0, 1.0)])
def test_dsyrk_ln_vs_oracle(n, k, alpha, beta):
    """Batched dsyrk_ln against the oracle: strictly upper triangle (NaN)
    untouched, beta == 0 does not read C, lower triangle within RIC_TOL."""
    torch, _lib, blas = torch_mods()
    batch, lda, ldc = 4, n + 1, n + 2
    say(f"dsyrk_ln n={n} k={k} alpha={alpha} beta={beta}")
    g = inputs.rng(inputs.seed_for(45, n * 100 + k))
    A = g.uniform(-1, 1, size=(batch, max(k, 1), lda))
    C = g.uniform(-1, 1, size=(batch, max(n, 1), ldc))
    for b in range(batch):
        for j in range(n):
            C[b, j, :j] = np.nan
            if beta == 0.0:
                C[b, j, j:n] = np.nan
    dA = torch.from_numpy(A.copy()).cuda()
    dC = torch.from_numpy(C.copy()).cuda()
    st = _lib.dsyrk_ln_strided_batched(n, k, alpha, dA.data_ptr(), lda, A[0].size, beta,
                                       dC.data_ptr(), ldc, C[0].size, batch,
                                       torch.cuda.current_stream().cuda_stream)
    assert st == 0
    got = _np(dC)
    lo, up = np.tril_indices(n), np.triu_indices(n, 1)
    for b in range(batch):
        Co = np.asfortranarray(C[b].T[:n, :n])
        oracle.dsyrk_ln(alpha, np.asfortranarray(A[b].T[:n, :k]), beta, Co)
        g_b = got[b].T[:n, :n]
        assert np.all(np.isnan(g_b[up])), "upper triangle written"
        assert _rel(g_b[lo], Co[lo]) <= RIC_TOL or np.max(np.abs(g_b[lo] - Co[lo])) == 0.0
