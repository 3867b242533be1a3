"""GPU parity of the backward path: the Cholesky adjoint kernel, the dgemm
adjoints and dlaset against the CPU oracle through the C ABI; the autograd
Functions against central finite differences (h = 1e-6, 50 directions) and
the oracle gradient on the 8192 x n=64 workload; the mixed-order batch (n in
16..192) through fused plans."""
import numpy as np
import pytest

import oracle
from paper_1902_08115_amd import inputs
from tests.gpu_util import GEMM_TOL, dev, host, say, torch_mods

pytestmark = pytest.mark.gpu

GRAD_TOL = 1e-9  # oracle-gradient gate (relative Frobenius)
FD_TOL = 1e-6    # |FD - <grad, dir>| <= FD_TOL * |FD|


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _factor_host(A, n, ld):
    """Oracle factor of every instance of a (batch, n, ld) SPD buffer, with
    the strict upper triangle replaced by NaN (it must never be read)."""
    L = np.ascontiguousarray(A).copy()
    info = oracle.dpotrf_l_strided_batched(n, L.ravel(), ld, n * ld, L.shape[0])
    assert (info == 0).all()
    iu = np.triu_indices(n, 1)
    L[:, iu[1], iu[0]] = np.nan
    return L


def _spread(blocks, ld, stride):
    """Flat buffer holding instance b's (n, ld) column-major block at b*stride,
    NaN in the gaps between instances."""
    batch, n = blocks.shape[0], blocks.shape[1]
    flat = np.full((batch - 1) * stride + n * ld, np.nan)
    for b in range(batch):
        flat[b * stride:b * stride + n * ld] = blocks[b].ravel()
    return flat


@pytest.mark.parametrize("n", [1, 2, 5, 15, 16, 17, 31, 33, 47, 64, 100, 129, 160, 192, 256, 304])
def test_cholesky_adjoint_vs_oracle(n):
    """Abar for random lower Lbar at orders spanning ragged tiles, one tile,
    many tiles and the 304 limit: within 1e-9 of the oracle adjoint (expected
    ~1e-14), exactly symmetric, the strict upper parts of L and Lbar (NaN)
    never read, the leading-dimension padding of Abar and the gaps between
    its instances untouched.  L, Lbar and Abar each have their own leading
    dimension and instance stride, with NaN between instances, so an ld or
    stride taken from the wrong operand reads NaN or writes out of place."""
    torch, _lib, _ = torch_mods()
    g = inputs.rng(inputs.seed_for(4, n))
    batch = 6 if n <= 64 else 3
    ldl, ldlb, ldab = n + 3, n + 1, n + 6
    sl, slb, sab = n * ldl + 5, n * ldlb + 17, n * ldab + 2
    A = inputs.spd_batch(g, batch, n, ld=ldl)
    L = _factor_host(A, n, ldl)
    Lb = inputs.colmajor(g, batch, n, n, ldlb)
    iu = np.triu_indices(n, 1)
    Lb[:, iu[1], iu[0]] = np.nan
    Lh = np.where(np.isnan(L), 0.0, L)
    Lbh = np.where(np.isnan(Lb), 0.0, Lb)
    ref = _spread(np.full((batch, n, ldab), np.nan), ldab, sab)
    oracle.dpotrf_l_adjoint_strided_batched(n, _spread(Lh, ldl, sl), ldl, sl,
                                            _spread(Lbh, ldlb, slb), ldlb, slb, ref, ldab, sab,
                                            batch)
    say(f"cholesky adjoint n={n} batch={batch}")
    dL, dLb = dev(_spread(L, ldl, sl)), dev(_spread(Lb, ldlb, slb))
    dAb = dev(_spread(np.full((batch, n, ldab), np.nan), ldab, sab))
    st = _lib.dpotrf_l_backward_strided_batched(n, dL.data_ptr(), ldl, sl, dLb.data_ptr(), ldlb,
                                                slb, dAb.data_ptr(), ldab, sab, batch,
                                                torch.cuda.current_stream().cuda_stream)
    assert st == 0, st
    G = host(dAb)
    for b in range(batch):
        blk = G[b * sab:b * sab + n * ldab].reshape(n, ldab)
        rblk = ref[b * sab:b * sab + n * ldab].reshape(n, ldab)
        g2, r2 = blk.T[:n], rblk.T[:n]
        assert np.isfinite(g2).all(), b
        assert rel(g2, r2) <= GRAD_TOL, (b, rel(g2, r2))
        assert np.array_equal(g2, g2.T), b
        assert np.isnan(blk.T[n:]).all(), "padding touched"
        if b + 1 < batch:
            assert np.isnan(G[b * sab + n * ldab:(b + 1) * sab]).all(), "gap touched"


def test_cholesky_adjoint_pointer_array_and_zero_sizes():
    """The pointer-array form equals the strided form bit for bit; n = 0 and
    batch = 0 launch nothing."""
    torch, _lib, blas = torch_mods()
    g = inputs.rng(inputs.seed_for(4, 900))
    n, batch = 40, 5
    A = inputs.spd_batch(g, batch, n)
    L = _factor_host(A, n, n)
    Lb = inputs.colmajor(g, batch, n, n)
    dL, dLb = dev(L), dev(Lb)
    out1 = dev(np.zeros((batch, n, n)))
    out2 = dev(np.zeros((batch, n, n)))
    sh = torch.cuda.current_stream().cuda_stream
    say("cholesky adjoint pointer array")
    assert _lib.dpotrf_l_backward_strided_batched(n, dL.data_ptr(), n, n * n, dLb.data_ptr(), n,
                                                  n * n, out1.data_ptr(), n, n * n, batch, sh) == 0
    idx = torch.arange(batch, dtype=torch.int64, device="cuda") * (8 * n * n)
    pa, pb, pc = idx + dL.data_ptr(), idx + dLb.data_ptr(), idx + out2.data_ptr()
    assert _lib.dpotrf_l_backward_batched(n, pa.data_ptr(), n, pb.data_ptr(), n, pc.data_ptr(),
                                          n, batch, sh) == 0
    assert np.array_equal(host(out1), host(out2))
    assert _lib.dpotrf_l_backward_strided_batched(0, None, 1, 0, None, 1, 0, None, 1, 0, 3,
                                                  sh) == 0
    assert _lib.dpotrf_l_backward_strided_batched(8, None, 8, 64, None, 8, 64, None, 8, 64, 0,
                                                  sh) == 0


@pytest.mark.parametrize("trans", inputs.TRANS_CASES)
def test_dgemm_backward_vs_definition(trans):
    """dA and dB of C = alpha op(A) op(B) for every trans case equal their
    definitions evaluated by the oracle dgemm (1e-12), and a NULL output is
    skipped."""
    torch, _lib, _ = torch_mods()
    ta, tb = trans
    g = inputs.rng(inputs.seed_for(4, 1000 + "NT".index(ta) * 2 + "NT".index(tb)))
    m, n, k, batch, alpha = 37, 29, 45, 4, -1.75
    (ar, ac), (br, bc) = ((m, k) if ta == "N" else (k, m)), ((k, n) if tb == "N" else (n, k))
    A = inputs.colmajor(g, batch, ar, ac, ar + 1)
    B = inputs.colmajor(g, batch, br, bc, br + 2)
    dC = inputs.colmajor(g, batch, m, n, m + 3)
    sh = torch.cuda.current_stream().cuda_stream
    dA_d = dev(np.full((batch, ac, ar + 4), np.nan))
    dB_d = dev(np.full((batch, bc, br + 1), np.nan))
    dA_in, dB_in, dC_in = dev(A), dev(B), dev(dC)
    say(f"dgemm backward {trans}")
    st = _lib.dgemm_backward_strided_batched(
        ta, tb, m, n, k, alpha, dA_in.data_ptr(), ar + 1, ac * (ar + 1), dB_in.data_ptr(), br + 2,
        bc * (br + 2), dC_in.data_ptr(), m + 3, n * (m + 3), dA_d.data_ptr(), ar + 4,
        ac * (ar + 4), dB_d.data_ptr(), br + 1, bc * (br + 1), batch, sh)
    assert st == 0, st
    GA = host(dA_d).reshape(batch, ac, ar + 4)
    GB = host(dB_d).reshape(batch, bc, br + 1)
    for b in range(batch):
        a, bm, c = A[b].ravel(), B[b].ravel(), dC[b].ravel()
        ra = np.zeros(ac * (ar + 4))
        rb = np.zeros(bc * (br + 1))
        if ta == "N":
            oracle.dgemm_raw("N", "T" if tb == "N" else "N", m, k, n, alpha, c, m + 3, bm, br + 2,
                             0.0, ra, ar + 4)
        else:
            oracle.dgemm_raw(tb, "T", k, m, n, alpha, bm, br + 2, c, m + 3, 0.0, ra, ar + 4)
        if tb == "N":
            oracle.dgemm_raw("T" if ta == "N" else "N", "N", k, n, m, alpha, a, ar + 1, c, m + 3,
                             0.0, rb, br + 1)
        else:
            oracle.dgemm_raw("T", ta, n, k, m, alpha, c, m + 3, a, ar + 1, 0.0, rb, br + 1)
        ga, rra = GA[b].T[:ar], ra.reshape(ac, ar + 4).T[:ar]
        gb, rrb = GB[b].T[:br], rb.reshape(bc, br + 1).T[:br]
        assert rel(ga, rra) <= GEMM_TOL and rel(gb, rrb) <= GEMM_TOL, b
        assert np.isnan(GA[b].T[ar:]).all() and np.isnan(GB[b].T[br:]).all()
    # dB skipped: dB untouched
    dB_d.fill_(7.0)
    st = _lib.dgemm_backward_strided_batched(
        ta, tb, m, n, k, alpha, dA_in.data_ptr(), ar + 1, ac * (ar + 1), dB_in.data_ptr(), br + 2,
        bc * (br + 2), dC_in.data_ptr(), m + 3, n * (m + 3), dA_d.data_ptr(), ar + 4,
        ac * (ar + 4), None, br + 1, bc * (br + 1), batch, sh)
    assert st == 0 and (host(dB_d) == 7.0).all()


@pytest.mark.parametrize("uplo", ["U", "L", "A"])
def test_dlaset(uplo):
    torch, _lib, _ = torch_mods()
    m, n, ld, batch = 23, 17, 25, 3
    X = inputs.colmajor(inputs.rng(5), batch, m, n, ld)
    d = dev(X)
    say(f"dlaset {uplo}")
    assert _lib.dlaset_strided_batched(uplo, m, n, 2.5, -1.0, d.data_ptr(), ld, n * ld, batch,
                                       torch.cuda.current_stream().cuda_stream) == 0
    G = host(d).reshape(batch, n, ld)
    i, j = np.meshgrid(np.arange(m), np.arange(n), indexing="ij")
    sel = (i < j) if uplo == "U" else ((i > j) if uplo == "L" else (i != j))
    for b in range(batch):
        ref = X[b].T[:m].copy()
        ref[sel] = 2.5
        ref[i == j] = -1.0
        assert np.array_equal(G[b].T[:m], ref)
        assert np.isnan(G[b].T[m:]).all()


def _loss_grads(torch, ag, A, B, W):
    A = A.detach().requires_grad_(True)
    B = B.detach().requires_grad_(True)
    C = ag.cholesky_product(A, B)
    loss = (C * W).sum()
    loss.backward()
    return C.detach(), A.grad.detach(), B.grad.detach()


def test_autograd_fd_and_oracle_gradient_n64_batch8192():
    """The differentiation workload: 8192 SPD instances of order 64, B 64 x 32,
    loss <W, chol(A) B>.  Central differences with h = 1e-6 along 50 random
    directions (symmetric dA, dB uniform [-1, 1)) match <Abar, dA> + <Bbar, dB>
    to 1e-6 relative, and 24 sampled instances match the oracle gradient to
    1e-9."""
    torch, _lib, blas = torch_mods()
    from paper_1902_08115_amd import autograd as ag
    batch, n, nb = inputs.BACKWARD_BATCH, inputs.BACKWARD_N, inputs.BACKWARD_NB
    A = inputs.torch_spd(batch, n, seed=inputs.seed_for(4, 1))
    B = inputs.torch_colmajor(batch, n, nb, seed=inputs.seed_for(4, 2))
    W = inputs.torch_colmajor(batch, n, nb, seed=inputs.seed_for(4, 3))
    say("autograd n=64 batch=8192 forward/backward")
    C, Ab, Bb = _loss_grads(torch, ag, A, B, W)
    torch.cuda.synchronize()
    h = inputs.FD_STEP

    def f(Ax, Bx):
        with torch.no_grad():
            return float((ag.cholesky_product(Ax, Bx) * W).sum())

    worst = 0.0
    for d in range(inputs.FD_DIRECTIONS):
        dA = inputs.torch_symmetric(batch, n, seed=inputs.seed_for(4, 100 + d))
        dB = inputs.torch_colmajor(batch, n, nb, seed=inputs.seed_for(4, 200 + d))
        fd = (f(A + h * dA, B + h * dB) - f(A - h * dA, B - h * dB)) / (2 * h)
        an = float((Ab * dA).sum() + (Bb * dB).sum())
        err = abs(fd - an) / (abs(fd) + 1e-300)
        worst = max(worst, err)
        assert err <= FD_TOL, (d, fd, an, err)
    say(f"fd worst relative error {worst:.2e}")
    # oracle gradient on sampled instances
    g = inputs.rng(inputs.seed_for(4, 4))
    for b in sorted(g.choice(batch, 24, replace=False)):
        a = np.asfortranarray(A[b].cpu().numpy())
        bm = np.asfortranarray(B[b].cpu().numpy())
        w = np.asfortranarray(W[b].cpu().numpy())
        L = a.copy(order="F")
        assert oracle.dpotrf_l(L) == 0
        L = np.asfortranarray(np.tril(L))
        Cref = np.zeros((n, nb), order="F")
        oracle.dgemm("N", "N", 1.0, L, bm, 0.0, Cref)
        Lbar = np.zeros((n, n), order="F")
        oracle.dgemm("N", "T", 1.0, w, bm, 0.0, Lbar)
        Bbar = np.zeros((n, nb), order="F")
        oracle.dgemm("T", "N", 1.0, L, w, 0.0, Bbar)
        Abar = oracle.dpotrf_l_adjoint(L, Lbar)
        assert rel(C[b].cpu().numpy(), Cref) <= GEMM_TOL, b
        assert rel(Ab[b].cpu().numpy(), Abar) <= GRAD_TOL, (b, rel(Ab[b].cpu().numpy(), Abar))
        assert rel(Bb[b].cpu().numpy(), Bbar) <= GRAD_TOL, b


def test_cholesky_raises_on_non_spd():
    torch, _lib, blas = torch_mods()
    from paper_1902_08115_amd import autograd as ag
    A = inputs.torch_spd(4, 20, seed=7).clone()
    A[2, 5, 5] = -1.0
    say("autograd non-SPD")
    with pytest.raises(torch.linalg.LinAlgError, match="instance 2"):
        ag.cholesky(A)


def test_mixed_orders_fused_plans():
    """The mixed batch (2048 instances, n = floor(exp(U[ln 16, ln 193)))),
    forward and backward as fused plans behind a torch.autograd.Function:
    64 sampled instances match the oracle forward and gradient (1e-9), and
    central differences (h = 1e-6) along 50 random directions (dA symmetric
    per instance, dB uniform) match the directional derivative of
    <Cbar, C> that autograd's gradients give; a backward whose forward was
    overwritten raises."""
    torch, _lib, blas = torch_mods()
    from paper_1902_08115_amd.mixed import MixedCholeskyProduct
    ns = inputs.backward_mixed_sizes(inputs.seed_for(4, 10))
    nb = inputs.BACKWARD_NB
    mp = MixedCholeskyProduct(ns, nb)
    g = inputs.rng(inputs.seed_for(4, 11))
    # inputs: SPD A per instance, B and the cotangent W uniform [-1, 1)
    A0 = torch.zeros_like(mp.buf["A"])
    for n in np.unique(ns):
        idx = np.nonzero(ns == n)[0]
        S = inputs.torch_spd(len(idx), int(n), seed=inputs.seed_for(4, 20000 + int(n)))
        for j, b in enumerate(idx):
            o = int(mp.off_sq[b])
            A0[o:o + int(n) * int(n)].view(int(n), int(n)).t().copy_(S[j])
    B0 = torch.empty_like(mp.buf["B"]).uniform_(
        -1.0, 1.0, generator=torch.Generator(device="cuda").manual_seed(12))
    W = torch.empty_like(mp.buf["C"]).uniform_(
        -1.0, 1.0, generator=torch.Generator(device="cuda").manual_seed(13))
    say(f"mixed plans through autograd: {len(ns)} instances, n {ns.min()}..{ns.max()}")
    A = A0.clone().requires_grad_(True)
    B = B0.clone().requires_grad_(True)
    C = mp(A, B)
    (C * W).sum().backward()
    torch.cuda.synchronize()
    assert int(mp.info.abs().sum()) == 0
    Abar, Bbar = A.grad.detach().clone(), B.grad.detach().clone()
    Cg = C.detach().clone()
    for b in sorted(g.choice(len(ns), 64, replace=False)):
        n = int(ns[b])
        o, r = int(mp.off_sq[b]), int(mp.off_rect[b])
        a = A0[o:o + n * n].view(n, n).t().cpu().numpy().copy(order="F")
        bm = B0[r:r + n * nb].view(nb, n).t().cpu().numpy().copy(order="F")
        w = W[r:r + n * nb].view(nb, n).t().cpu().numpy().copy(order="F")
        L = a.copy(order="F")
        assert oracle.dpotrf_l(L) == 0
        L = np.asfortranarray(np.tril(L))
        Cref = np.zeros((n, nb), order="F")
        oracle.dgemm("N", "N", 1.0, L, bm, 0.0, Cref)
        Lbar = np.zeros((n, n), order="F")
        oracle.dgemm("N", "T", 1.0, w, bm, 0.0, Lbar)
        Bref = np.zeros((n, nb), order="F")
        oracle.dgemm("T", "N", 1.0, L, w, 0.0, Bref)
        Aref = oracle.dpotrf_l_adjoint(L, Lbar)
        assert rel(Cg[r:r + n * nb].view(nb, n).t().cpu().numpy(), Cref) <= GEMM_TOL, b
        assert rel(Abar[o:o + n * n].view(n, n).t().cpu().numpy(), Aref) <= GRAD_TOL, b
        assert rel(Bbar[r:r + n * nb].view(nb, n).t().cpu().numpy(), Bref) <= GRAD_TOL, b
    # a second forward overwrites the factors the first graph's backward needs
    C1 = mp(A, B)
    C2 = mp(A, B)
    with pytest.raises(RuntimeError, match="overwrote"):
        (C1 * W).sum().backward()
    del C2
    # central differences of <W, C> over the whole batch, 50 directions
    t = mp.symmetrize_index()
    h = inputs.FD_STEP
    with torch.no_grad():
        def f(Ax, Bx):
            return float((mp(Ax, Bx) * W).sum())

        for d in range(inputs.FD_DIRECTIONS):
            gen = torch.Generator(device="cuda").manual_seed(300 + d)
            dA = torch.empty_like(A0).uniform_(-1.0, 1.0, generator=gen)
            dA = 0.5 * (dA + dA[t])  # symmetric per instance
            dB = torch.empty_like(B0).uniform_(-1.0, 1.0, generator=gen)
            fp = f(A0 + h * dA, B0 + h * dB)
            fm = f(A0 - h * dA, B0 - h * dB)
            fd = (fp - fm) / (2 * h)
            an = float((Abar * dA).sum() + (Bbar * dB).sum())
            assert abs(fd - an) <= FD_TOL * abs(fd), (d, fd, an)
    mp.close()
