"""Strength of the oracle's pins: plant a plausible mistake in a copy of
oracle.c (CPU only), build it, and check that the pins catch it.  Each
mutation runs the named pin tests in a child process against the broken
library and expects them to fail."""

import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

# (name, exact text to replace, replacement, pin tests that must fail)
MUTATIONS = [
    ("ilu0_transposed_operand",
     "blk_mul(bs, val + pj * bb, inv, Lij);", "blk_mul(bs, inv, val + pj * bb, Lij);",
     ["test_bilu0_matches_A_on_pattern"]),
    ("ilu0_skips_update",
     "for (int e = 0; e < bb; ++e) val[pk * bb + e] -= tmp[e];", "for (int e = 0; e < bb; ++e) val[pk * bb + e] -= 0.5 * tmp[e];",
     ["test_bilu0_matches_A_on_pattern", "test_bilu0_scalar_laplacian_pivots"]),
    ("ildu0_right_scaling",
     "blk_mul(bs, inv, val + pk * bb, tmp);\n            memcpy(val + pk * bb, tmp, sizeof(double) * bb);",
     "blk_mul(bs, val + pk * bb, inv, tmp);\n            memcpy(val + pk * bb, tmp, sizeof(double) * bb);",
     ["test_ildu0_reproduces_lu"]),
    ("apply_backward_sign",
     "if (col[p] > I) blk_matvec_sub(bs, f + p * bb, z + (int64_t)col[p] * bs, z + I * bs);",
     "if (col[p] > I) blk_matvec(bs, f + p * bb, z + (int64_t)col[p] * bs, z + I * bs);",
     ["test_apply_inverts_factors"]),
    ("levels_off_by_one",
     "if (col[j] < I && lev[col[j]] + 1 > l) l = lev[col[j]] + 1;",
     "if (col[j] < I && lev[col[j]] + 2 > l) l = lev[col[j]] + 2;",
     ["test_levels_structured_closed_form", "test_levels_brute_force_random_dag"]),
    ("drop_wrong_window",
     "if (col[j] / S == I / S) {", "if (col[j] / S <= I / S) {",
     ["test_drop_count_closed_form", "test_drop_keeps_diagonal_windows"]),
    ("bicgstab_beta_without_alpha_over_omega",
     "double beta = (rho_new / rho) * (alpha / omega);", "double beta = (rho_new / rho);",
     ["test_bicgstab_cross_check_scipy"]),
    ("reorder_columns_unmapped",
     "ocol[m] = old2new[col[j]];", "ocol[m] = col[j];",
     ["test_reorder_is_symmetric_permutation"]),
    ("mlp_backward_wrong_mask",
     "g2[k] = h2[k] > 0.0 ? s : 0.0;", "g2[k] = s;",
     ["test_mlp_forward_backward_against_torch", "test_loss_gradient_central_differences"]),
    ("lic_dC_transposed",
     "dC[f * 9 + a * 3 + b] += A[(int64_t)q * 3 * n + (int64_t)fI[f] * 3 + a] *\n"
     "                                             R[(int64_t)q * 3 * n + (int64_t)fJ[f] * 3 + b];",
     "dC[f * 9 + a * 3 + b] += A[(int64_t)q * 3 * n + (int64_t)fI[f] * 3 + b] *\n"
     "                                             R[(int64_t)q * 3 * n + (int64_t)fJ[f] * 3 + a];",
     ["test_loss_gradient_central_differences", "test_least_squares_bound"]),
    ("adjoint_block_not_transposed",
     "for (int d = 0; d < bs; ++d) s += f[p * bb + d * bs + c] * a[K * bs + d];",
     "for (int d = 0; d < bs; ++d) s += f[p * bb + c * bs + d] * a[K * bs + d];",
     ["test_apply_transpose_adjoint", "test_least_squares_bound"]),
    ("features_diagonal_blocks_swapped",
     "x[e] = Aii[e] / sigma;", "x[e] = Ajj[e] / sigma;",
     ["test_features_hand_worked"]),
    ("features_reverse_coupling",
     "*Aij = val + (int64_t)fq[f] * 9,", "*Aij = val + find_col(ptr, col, fJ[f], fI[f]) * 9,",
     ["test_features_hand_worked"]),
    ("features_coupling_transposed",
     "x[9 + e] = Aij[e] / sigma;", "x[9 + e] = Aij[(e % 3) * 3 + e / 3] / sigma;",
     ["test_features_hand_worked"]),
    ("features_sigma_over_nine",
     "sqrt(fabs(ti) * fabs(tj)) / 3.0;", "sqrt(fabs(ti) * fabs(tj)) / 9.0;",
     ["test_features_hand_worked"]),
]

LIC_PINS = ("test_mlp_forward_backward_against_torch", "test_loss_gradient_central_differences",
            "test_least_squares_bound", "test_features_hand_worked")


@pytest.mark.parametrize("name,old,new,pins", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_mutation_is_caught(name, old, new, pins, tmp_path):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site not unique/found: {name}"
    mutated = tmp_path / "oracle_mut.c"
    mutated.write_text(src.replace(old, new))
    lib = tmp_path / "liboracle_mut.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", str(lib), str(mutated), "-lm"])
    env = dict(os.environ, ORACLE_LIB=str(lib))
    tests = []
    for pin in pins:
        mod = "tests/test_oracle_lic.py" if pin in LIC_PINS else "tests/test_oracle.py"
        tests.append(f"{mod}::{pin}")
    for t in tests:
        r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", t],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
        assert r.returncode != 0, f"{name}: pin {t} did not catch the mutation"
