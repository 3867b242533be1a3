"""GPU parity of the fused uneven batch (one persistent kernel over mixed
dgemm / dpotrf problems, through the plan entry points of the C ABI) against
the CPU oracle, problem by problem; every execution mode of a plan; repeated
executions; special scalars, quick returns, ragged and padded operands; the
full 100,000-problem batch on sampled problems plus every info word."""
import numpy as np
import pytest

import oracle
from paper_1902_08115_amd import inputs
from tests.gpu_util import GEMM_TOL, POTRF_TOL, say, torch_mods

pytestmark = pytest.mark.gpu

MODES = ("fused_graph", "fused", "grouped", "grouped_graph")


def problem_dicts(spec, base, info_base, idx=None):
    """mb_problem dicts for ``spec`` laid out in an arena at device address base."""
    idx = range(spec["count"]) if idx is None else idx
    out = []
    for i in idx:
        if spec["op"][i] == 0:
            out.append(dict(op=0, transa="NT"[spec["ta"][i]], transb="NT"[spec["tb"][i]],
                            m=spec["m"][i], n=spec["n"][i], k=spec["k"][i],
                            lda=spec["lda"][i], ldb=spec["ldb"][i], ldc=spec["ldc"][i],
                            alpha=spec["alpha"], beta=spec["beta"],
                            A=base + 8 * int(spec["off_a"][i]), B=base + 8 * int(spec["off_b"][i]),
                            C=base + 8 * int(spec["off_c"][i])))
        else:
            out.append(dict(op=1, uplo="L", n=spec["n"][i], ldc=spec["ldc"][i],
                            C=base + 8 * int(spec["off_c"][i]), info=info_base + 4 * int(i)))
    return out


def oracle_problem(spec, i, X0):
    """Oracle result of problem i on a host copy of its operands: the new
    C (or factored matrix) as a flat array, and info (dpotrf)."""
    oc = int(spec["off_c"][i])
    if spec["op"][i] == 0:
        m, n, k = (int(spec[f][i]) for f in ("m", "n", "k"))
        ldc = int(spec["ldc"][i])
        C = X0[oc:oc + ldc * n].copy()
        oracle.dgemm_raw("NT"[spec["ta"][i]], "NT"[spec["tb"][i]], m, n, k, spec["alpha"],
                         X0[int(spec["off_a"][i]):], int(spec["lda"][i]),
                         X0[int(spec["off_b"][i]):], int(spec["ldb"][i]), spec["beta"], C, ldc)
        return C, 0
    n = int(spec["n"][i])
    L = X0[oc:oc + n * n].copy()
    info = oracle.dpotrf_l_raw(n, L, n)
    return L, info


def check_problem(spec, i, X0, Xg, info_g):
    """Assert problem i of the GPU result against the oracle."""
    oc = int(spec["off_c"][i])
    ref, info_r = oracle_problem(spec, i, X0)
    if spec["op"][i] == 0:
        m, n = int(spec["m"][i]), int(spec["n"][i])
        ldc = int(spec["ldc"][i])
        g = Xg[oc:oc + ldc * n].reshape(n, ldc).T[:m]
        r = ref.reshape(n, ldc).T[:m]
        err = np.linalg.norm(g - r) / max(np.linalg.norm(r), 1e-300)
        assert err <= GEMM_TOL, (i, err)
        return
    n = int(spec["n"][i])
    assert int(info_g[i]) == info_r, (i, int(info_g[i]), info_r)
    f = int(spec["fail_col"][i])
    assert info_r == (f + 1 if f >= 0 else 0), (i, info_r, f)
    A0 = X0[oc:oc + n * n].reshape(n, n).T
    G = Xg[oc:oc + n * n].reshape(n, n).T
    R = ref.reshape(n, n).T
    iu = np.triu_indices(n, 1)
    assert np.array_equal(G[iu], A0[iu]), (i, "upper triangle touched")
    cols = n if info_r == 0 else info_r - 1
    if cols == 0:
        return
    low = np.tril(np.ones((n, n), dtype=bool))[:, :cols]
    d = np.linalg.norm((G[:, :cols] - R[:, :cols])[low]) / np.linalg.norm(R[:, :cols][low])
    assert d <= POTRF_TOL, (i, d)
    if info_r == 0:
        S = np.tril(A0) + np.tril(A0, -1).T
        Lg = np.tril(G).astype(np.longdouble)
        res = np.sqrt(((S - Lg @ Lg.T) ** 2).sum()) / np.sqrt((S.astype(np.longdouble) ** 2).sum())
        assert float(res) <= POTRF_TOL, (i, float(res))


def _run_modes(spec, X0, modes=MODES):
    """Run the plan of ``spec`` in each mode on a fresh device copy of X0;
    return {mode: (host arena, info)}."""
    torch, _lib, blas = torch_mods()
    out = {}
    for mode in modes:
        X = torch.from_numpy(X0).cuda()
        info = torch.full((max(spec["count"], 1),), -7, dtype=torch.int32, device="cuda")
        with blas.Plan(problem_dicts(spec, X.data_ptr(), info.data_ptr())) as plan:
            say(f"fused plan mode={mode} problems={spec['count']} stats={plan.stats()}")
            plan.execute(getattr(blas.Plan, mode.upper()))
            torch.cuda.synchronize()
            out[mode] = (X.cpu().numpy(), info.cpu().numpy())
    return out


# largest dpotrf order the plain launches factor with kernels of their own
# (whole rows in lanes up to 32, the factor in registers up to 112 and at
# 128); above it they run the same code as the fused kernel
SMALL_MAX_N = 128


@pytest.mark.parametrize("seed", [0, 1])
def test_uneven_batch_every_mode(seed):
    """400 mixed problems (sizes 4..160, 70% dgemm, 10% of the dpotrf
    non-SPD): every execution mode equals the oracle problem by problem;
    the graph and direct launches of one code path agree bit for bit;
    dpotrf info agrees across all modes, and dpotrf factors agree bit for bit
    across all modes for orders above 128 (smaller orders take kernels of their
    own in the grouped path -- whole rows in lanes, or the factor in
    registers -- whose evaluation order differs from the fused kernel's; both
    were checked against the oracle above)."""
    spec = inputs.uneven_spec(400, inputs.seed_for(3, seed), non_spd_frac=0.1)
    X0 = inputs.uneven_host(spec, inputs.seed_for(3, 100 + seed))
    res = _run_modes(spec, X0)
    for mode, (Xg, info) in res.items():
        say(f"checking mode {mode}")
        for i in range(spec["count"]):
            check_problem(spec, i, X0, Xg, info)
    assert np.array_equal(res["fused_graph"][0], res["fused"][0])
    assert np.array_equal(res["grouped"][0], res["grouped_graph"][0])
    pot = np.nonzero(spec["op"] == 1)[0]
    for i in pot:
        o, n = int(spec["off_c"][i]), int(spec["n"][i])
        if n > SMALL_MAX_N:
            assert np.array_equal(res["fused"][0][o:o + n * n], res["grouped"][0][o:o + n * n]), i
    assert np.array_equal(res["fused"][1][pot], res["grouped"][1][pot])


def test_uneven_ragged_sizes_beyond_the_workload():
    """Sizes 1..300 (past the 160 of the workload, tiles of every raggedness,
    dpotrf up to the 304 limit), all four trans cases."""
    spec = inputs.uneven_spec(160, inputs.seed_for(3, 7), lo=1, hi=300, p_gemm=0.6,
                              non_spd_frac=0.2)
    X0 = inputs.uneven_host(spec, inputs.seed_for(3, 107))
    Xg, info = _run_modes(spec, X0, ("fused_graph",))["fused_graph"]
    for i in range(spec["count"]):
        check_problem(spec, i, X0, Xg, info)


def test_special_problems():
    """Hand-made problems: alpha = 0 with NaN operands, beta = 0 with NaN in C,
    k = 0, quick returns (m = 0, n = 0, alpha = 0 and beta = 1), padded
    leading dimensions whose padding must survive, dpotrf of order 0 and 1,
    beside ordinary problems in the same plan."""
    torch, _lib, blas = torch_mods()
    g = inputs.rng(inputs.seed_for(3, 50))
    nan = np.nan
    cases = []  # (dict without pointers, A, B, C host arrays (flat), kind)

    def gemm(ta, tb, m, n, k, alpha, beta, lda=None, ldb=None, ldc=None, a_fill=None,
             c_fill=None):
        ar, ac = (m, k) if ta == "N" else (k, m)
        br, bc = (k, n) if tb == "N" else (n, k)
        lda = max(1, ar) if lda is None else lda
        ldb = max(1, br) if ldb is None else ldb
        ldc = max(1, m) if ldc is None else ldc
        A = inputs.colmajor(g, 1, ar, ac, lda)[0].ravel()
        B = inputs.colmajor(g, 1, br, bc, ldb)[0].ravel()
        C = inputs.colmajor(g, 1, m, n, ldc)[0].ravel()
        if a_fill is not None:
            A[:] = a_fill
            B[:] = a_fill
        if c_fill is not None:
            C[:] = c_fill
        cases.append((dict(op=0, transa=ta, transb=tb, m=m, n=n, k=k, lda=lda, ldb=ldb, ldc=ldc,
                           alpha=alpha, beta=beta), A, B, C))

    gemm("N", "N", 20, 20, 20, 0.0, 2.0, a_fill=nan)        # alpha = 0: A, B never read
    gemm("T", "N", 33, 17, 9, 1.5, 0.0, c_fill=nan)         # beta = 0: NaN in C ignored
    gemm("N", "T", 40, 35, 0, 3.0, -0.5)                    # k = 0: C = beta C
    gemm("N", "N", 0, 5, 5, 1.0, 1.0)                       # m = 0: nothing
    gemm("T", "T", 5, 0, 5, 1.0, 1.0)                       # n = 0: nothing
    gemm("N", "N", 6, 6, 6, 0.0, 1.0, a_fill=nan)           # quick return
    gemm("T", "T", 37, 29, 50, -1.25, 0.75, lda=61, ldb=33, ldc=45)  # padded ld (NaN padding)
    gemm("N", "T", 1, 1, 1, 2.0, 1.0)
    gemm("T", "N", 161, 3, 200, 1.0, 1.0)
    pots = []
    for n, fail in ((0, -1), (1, -1), (19, -1), (48, 30), (160, -1), (304, -1)):
        A = inputs.spd_batch(g, 1, n, ld=n + 2, upper_value=nan)[0].ravel() if n else \
            np.zeros(1)
        if fail >= 0:
            A[fail + fail * (n + 2)] = -1.0
        pots.append((n, fail, A))

    # one arena: every array back to back
    arrays = [a for c in cases for a in c[1:]] + [p[2] for p in pots]
    offs = np.cumsum([0] + [len(a) for a in arrays])
    X0 = np.concatenate(arrays)
    X = torch.from_numpy(X0).cuda()
    info = torch.full((len(pots),), -7, dtype=torch.int32, device="cuda")
    base = X.data_ptr()
    probs = []
    for ci, c in enumerate(cases):
        d = dict(c[0])
        d.update(A=base + 8 * int(offs[3 * ci]), B=base + 8 * int(offs[3 * ci + 1]),
                 C=base + 8 * int(offs[3 * ci + 2]))
        probs.append(d)
    for pi, (n, fail, A) in enumerate(pots):
        probs.append(dict(op=1, uplo="L", n=n, ldc=max(1, n + 2 if n else 1),
                          C=base + 8 * int(offs[3 * len(cases) + pi]), info=info.data_ptr() + 4 * pi))
    say(f"fused special problems: {len(probs)}")
    with blas.Plan(probs) as plan:
        st = plan.stats()
        assert st["idle"] == 3, st  # m = 0, n = 0 and the alpha = 0, beta = 1 quick return
        plan.execute()
        torch.cuda.synchronize()
    Xg = X.cpu().numpy()
    ig = info.cpu().numpy()
    for ci, (d, A, B, C) in enumerate(cases):
        o = int(offs[3 * ci + 2])
        Cr = C.copy()
        oracle.dgemm_raw(d["transa"], d["transb"], d["m"], d["n"], d["k"], d["alpha"], A,
                         d["lda"], B, d["ldb"], d["beta"], Cr, d["ldc"])
        Cg = Xg[o:o + len(C)]
        m, n, ldc = d["m"], d["n"], d["ldc"]
        if m and n:
            g2 = Cg.reshape(n, ldc).T
            r2 = Cr.reshape(n, ldc).T
            assert not np.isnan(g2[:m]).any() or np.isnan(r2[:m]).any(), ci
            err = np.linalg.norm(g2[:m] - r2[:m]) / max(np.linalg.norm(r2[:m]), 1e-300)
            assert err <= GEMM_TOL, (ci, err)
            pad_g, pad_0 = g2[m:], C.reshape(n, ldc).T[m:]
            assert np.array_equal(np.isnan(pad_g), np.isnan(pad_0)), (ci, "ld padding touched")
        else:
            assert np.array_equal(Cg, C, equal_nan=True), ci
        if d["alpha"] == 0.0 and d["beta"] == 1.0:
            assert np.array_equal(Cg, C, equal_nan=True), ci
    for pi, (n, fail, A) in enumerate(pots):
        Lr = A.copy()
        info_r = oracle.dpotrf_l_raw(n, Lr, max(1, n + 2)) if n else 0
        assert ig[pi] == info_r == (fail + 1 if fail >= 0 else 0), (n, ig[pi], info_r)
        if n == 0:
            continue
        o = int(offs[3 * len(cases) + pi])
        G = Xg[o:o + len(A)].reshape(n, n + 2).T
        R = Lr.reshape(n, n + 2).T
        cols = n if info_r == 0 else info_r - 1
        low = np.tril(np.ones((n, n), dtype=bool))[:, :cols]
        if cols:
            d = np.linalg.norm((G[:n, :cols] - R[:n, :cols])[low]) / np.linalg.norm(
                R[:n, :cols][low])
            assert d <= POTRF_TOL, (n, d)
        iu = np.triu_indices(n, 1)
        assert np.isnan(G[:n][iu]).all() and np.isnan(G[n:]).all(), (n, "upper/padding touched")


def test_repeated_execution_and_two_plans():
    """Executions reset the queue counters: the same plan run twice on
    restored inputs, with another plan executed in between, gives identical
    results (the second plan smaller than the first)."""
    torch, _lib, blas = torch_mods()
    spec1 = inputs.uneven_spec(300, inputs.seed_for(3, 20), non_spd_frac=0.1)
    spec2 = inputs.uneven_spec(50, inputs.seed_for(3, 21))
    X01 = inputs.uneven_host(spec1, inputs.seed_for(3, 120))
    X02 = inputs.uneven_host(spec2, inputs.seed_for(3, 121))
    X1 = torch.from_numpy(X01).cuda()
    X2 = torch.from_numpy(X02).cuda()
    i1 = torch.zeros(spec1["count"], dtype=torch.int32, device="cuda")
    i2 = torch.zeros(spec2["count"], dtype=torch.int32, device="cuda")
    p1 = blas.Plan(problem_dicts(spec1, X1.data_ptr(), i1.data_ptr()))
    p2 = blas.Plan(problem_dicts(spec2, X2.data_ptr(), i2.data_ptr()))
    say("fused repeated execution")
    p1.execute()
    p2.execute()
    torch.cuda.synchronize()
    first = X1.cpu().numpy(), i1.cpu().numpy()
    X1.copy_(torch.from_numpy(X01))
    i1.zero_()
    p2.execute()
    p1.execute()
    p1.close()
    p2.close()
    torch.cuda.synchronize()
    assert np.array_equal(X1.cpu().numpy(), first[0]) and np.array_equal(i1.cpu().numpy(), first[1])
    for i in range(spec1["count"]):
        check_problem(spec1, i, X01, first[0], first[1])


def test_full_uneven_batch_sampled():
    """The full batch: 100,000 problems (sizes 4..160 log-uniform, 70% dgemm,
    1% of the dpotrf non-SPD), fused graph execution.  Every dpotrf info word
    equals its construction (0, or the failing column + 1), and 600 sampled
    problems equal the oracle."""
    torch, _lib, blas = torch_mods()
    spec = inputs.uneven_spec(inputs.UNEVEN_COUNT, inputs.seed_for(3, 0), non_spd_frac=0.01)
    say(f"fused full batch: arena {spec['total'] * 8 / 2**30:.2f} GiB")
    X = inputs.uneven_device(spec, inputs.seed_for(3, 200))
    info = torch.full((spec["count"],), -7, dtype=torch.int32, device="cuda")
    g = inputs.rng(inputs.seed_for(3, 300))
    sample = np.sort(g.choice(spec["count"], 600, replace=False))

    def grab(i):
        lo = int(min(spec["off_a"][i], spec["off_b"][i], spec["off_c"][i]))
        hi = int(spec["off_c"][i] + spec["ldc"][i] * spec["n"][i])
        return lo, X[lo:hi].cpu().numpy()

    before = {int(i): grab(i) for i in sample}
    with blas.Plan(problem_dicts(spec, X.data_ptr(), info.data_ptr())) as plan:
        say(f"stats {plan.stats()}")
        plan.execute()
        torch.cuda.synchronize()
    ig = info.cpu().numpy()
    pot = spec["op"] == 1
    exp = np.where(spec["fail_col"] >= 0, spec["fail_col"] + 1, 0)
    assert np.array_equal(ig[pot], exp[pot])
    assert (ig[~pot] == -7).all()
    for i in sample:
        lo, X0 = before[int(i)]
        lo2, Xg = grab(i)
        # shift the spec offsets to the local window
        loc = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in spec.items()}
        for f in ("off_a", "off_b", "off_c"):
            loc[f] = spec[f] - lo
        check_problem(loc, int(i), X0, Xg, ig)
