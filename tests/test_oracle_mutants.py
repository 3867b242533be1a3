"""Plant plausible mistakes in a copy of the oracle and check that the pins
catch every one of them (CPU only; the oracle source itself is not modified).

Each mutant is a textual edit of oracle.c -- a dropped term, a wrong sign or
index, a transposed operand, a wrong pivot test -- compiled into a temporary
shared library and run against the same pins that the real oracle passes."""
import os

import pytest

import oracle
from tests.oracle_pins import ALL_PINS

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTANTS = [
    ("dgemm_transposed_A", "op_elem(transa, A, lda, i, p)", "op_elem(transa, A, lda, p, i)"),
    ("dgemm_lowercase_n", "return t == 'N' || t == 'n';", "return t == 'N';"),
    ("dgemm_dropped_beta", "*cij = alpha * s + beta * (*cij);", "*cij = alpha * s;"),
    ("dgemm_wrong_sign", "s += op_elem(transa", "s -= op_elem(transa"),
    ("dgemm_dropped_last_term", "for (int p = 0; p < k; ++p)\n                s +=",
     "for (int p = 0; p < k - 1; ++p)\n                s +="),
    ("dgemm_beta0_reads_C", "if (beta == 0.0)\n                *cij = alpha * s;\n            else\n", ""),
    ("dgemm_alpha0_reads_AB", "            if (alpha == 0.0 || k == 0) {\n",
     "            if (k == 0) {\n"),
    ("dgemm_batched_skips_first", "for (int b = 0; b < batch; ++b)\n        oracle_dgemm(",
     "for (int b = 1; b < batch; ++b)\n        oracle_dgemm("),
    ("potrf_pivot_test", "if (!(d > 0.0))", "if (d < 0.0)"),
    ("potrf_info_off_by_one", "return j + 1;", "return j;"),
    ("potrf_diag_sign", "d -= ljp * ljp;", "d += ljp * ljp;"),
    ("potrf_multiply_not_divide", "A[(size_t)i + (size_t)j * (size_t)lda] = s / ljj;",
     "A[(size_t)i + (size_t)j * (size_t)lda] = s * ljj;"),
    ("potrf_dropped_update_term", "for (int p = 0; p < j; ++p)\n                s -=",
     "for (int p = 0; p < j - 1; ++p)\n                s -="),
    ("potrf_reads_upper",
     "s -= A[(size_t)i + (size_t)p * (size_t)lda] * A[(size_t)j + (size_t)p * (size_t)lda];",
     "s -= A[(size_t)i + (size_t)p * (size_t)lda] * A[(size_t)p + (size_t)j * (size_t)lda];"),
    ("potrf_skips_first_subdiag_row", "for (int i = j + 1; i < n; ++i)", "for (int i = j + 2; i < n; ++i)"),
    ("potrf_batched_skips_first", "for (int b = 0; b < batch; ++b)\n        info[b]",
     "for (int b = 1; b < batch; ++b)\n        info[b]"),
    ("adjoint_no_half_diagonal", "                if (i == j)\n                    v *= 0.5;\n", ""),
    ("adjoint_not_symmetrized", "0.5 * (Px(i, j) + Px(j, i))", "Px(i, j)"),
    ("adjoint_dropped_diag_product", "for (int p = i; p < n; ++p)\n                    v +=",
     "for (int p = i + 1; p < n; ++p)\n                    v +="),
    ("adjoint_transposed_L", "v -= Lx(p, i) * Px(p, j);", "v -= Lx(i, p) * Px(p, j);"),
    ("adjoint_second_solve_sign", "v -= Px(r, p) * Lx(p, c);", "v += Px(r, p) * Lx(p, c);"),
    ("adjoint_batched_swapped_strides", "Lbar + (ptrdiff_t)b * strideLb, ldlb,",
     "Lbar + (ptrdiff_t)b * strideL, ldlb,"),
    ("adjoint_batched_swapped_ld", "Lbar + (ptrdiff_t)b * strideLb, ldlb,",
     "Lbar + (ptrdiff_t)b * strideLb, ldl,"),
    ("adjoint_batched_skips_first", "        bad |= oracle_dpotrf_l_adjoint(n, L + (ptrdiff_t)b",
     "        if (b > 0) bad |= oracle_dpotrf_l_adjoint(n, L + (ptrdiff_t)b"),
    ("trmm_reads_upper", "* A[(size_t)p + (size_t)j * (size_t)lda];\n            B[",
     "* A[(size_t)j + (size_t)p * (size_t)lda];\n            B["),
    ("trmm_dropped_diagonal", "for (int p = j; p < n; ++p)\n                s += B",
     "for (int p = j + 1; p < n; ++p)\n                s += B"),
    ("trmm_no_alpha", "B[(size_t)i + (size_t)j * (size_t)ldb] = alpha * s;",
     "B[(size_t)i + (size_t)j * (size_t)ldb] = s;"),
    ("syrk_writes_upper", "for (int i = j; i < n; ++i) {\n            double *c =",
     "for (int i = 0; i < n; ++i) {\n            double *c ="),
    ("syrk_transposed_factor", "acc += A[(size_t)i + (size_t)p * (size_t)lda] * A[(size_t)j + (size_t)p * (size_t)lda];",
     "acc += A[(size_t)i + (size_t)p * (size_t)lda] * A[(size_t)p + (size_t)j * (size_t)lda];"),
    ("riccati_wrong_factor_block", "Lc = Fn + (size_t)nu + (size_t)nu * (size_t)ldf;", "Lc = Fn;"),
    ("riccati_no_syrk", "oracle_dsyrk_ln(m, nx, 1.0, C, m, 1.0, Fn, ldf);", ""),
    ("riccati_forward_order", "for (int n = N - 1; n >= 0; --n) {", "for (int n = 0; n < N; ++n) {"),
    ("riccati_no_trmm", "oracle_dtrmm_rlnn(m, nx, 1.0, Lc, ldlc, C, m);", ""),
    ("riccati_unreached_zero", "        info[n] = -1;\n    for (int j", "        info[n] = 0;\n    for (int j"),
    ("riccati_continues_after_failure", "        if (info[n] != 0)\n            break;\n", ""),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(name, old, new, tmp_path):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation target for {name} not found exactly once"
    mpath = tmp_path / f"oracle_{name}.c"
    mpath.write_text(src.replace(old, new))
    so = oracle.build(src=str(mpath), out=str(tmp_path / f"lib_{name}.so"))
    lib = oracle.load(so)
    caught = []
    for pin in ALL_PINS:
        try:
            pin(lib)
        except AssertionError:
            caught.append(pin.__name__)
            break
    assert caught, f"mutant {name} passed every pin"
