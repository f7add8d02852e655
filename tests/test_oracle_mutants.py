"""Planted mistakes in a copy of the oracle must fail the pins.

Each mutant is oracle.c with one plausible slip (a dropped term, a wrong
sign, a wrong index, a transposed operand), compiled on the CPU into a
temporary library. The pin battery below (a subset of test_oracle_pins)
must reject every one of them, and accept the unmodified source.
"""
import os
import subprocess

import numpy as np
import pytest

import oracle as orc
import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(orc.__file__), "oracle.c")

MUTANTS = {
    "E_transposed_O": ("gemm(n, BLK(Dinv, k, n), BLK(O, k, n), T);",
                       "gemm_nt(n, BLK(Dinv, k, n), BLK(O, k, n), T);"),
    "Hd_dropped_term": ("if (k > 0) {\n      gemm_tn(n, BLK(E, k - 1, n)",
                        "if (0) {\n      gemm_tn(n, BLK(E, k - 1, n)"),
    "Hl_wrong_index": ("gemm(n, BLK(O, k, n), BLK(E, k + 1, n), U);",
                       "gemm(n, BLK(O, k, n), BLK(E, k, n), U);"),
    "G_wrong_sign": ("gemvt_acc(n, -1.0, BLK(E, k - 1, n)",
                     "gemvt_acc(n, 1.0, BLK(E, k - 1, n)"),
    "stair_parity": ("return (k % 2) == 1;  /* paper's even rows */",
                     "return (k % 2) == 0;  /* paper's even rows */"),
    "spmv_lower_not_transposed": (
        "if (k > 0) gemvt_acc(n, 1.0, BLK(O, k - 1, n), VEC(x, k - 1, n), yk);",
        "if (k > 0) gemv_acc(n, 1.0, BLK(O, k - 1, n), VEC(x, k - 1, n), yk);"),
    "schur_sign": ("S[i * n + j] = Dn[i * n + j] - t;",
                   "S[i * n + j] = Dn[i * n + j] + t;"),
    "pcg_beta_inverted": ("double beta = rho1 / rho;",
                          "double beta = rho / rho1;"),
    "alpha_index": ("z[e] += pc->alpha[i] * pc->y[e];",
                    "z[e] += pc->alpha[i - 1] * pc->y[e];"),
    "adjoint_dO_transposed": ("-(lk[i] * x1[j] + xk[i] * l1[j]);",
                              "-(lk[i] * x1[j] + l1[i] * xk[j]);"),
    "split_H_weight": ("y[i] = c->a * (c->t1[i] + c->t2[i]) + c->b * c->t3[i];\n}\n\n/* Exported",
                       "y[i] = c->a * (c->t1[i] + c->t2[i]) - c->b * c->t3[i];\n}\n\n/* Exported"),
}


def battery():
    """Run the pins; return the names of those that fail."""
    checks = {
        "btchol": lambda: pins.test_block_cholesky_matches_dense_solve(7, 3),
        "spmv": pins.test_spmv_matches_dense,
        "closed_form": lambda: pins.test_closed_form_Gopt_Hopt_match_definitions(5, 3),
        "split": lambda: pins.test_splitting_form_matches_definition(0.25, 0.5),
        "precond": lambda: pins.test_precond_matches_dense_polynomial(
            3, orc.PC_OPT),
        "footnote": lambda: pins.test_footnote_identity_opt_m_equals_jacobi_2m(2),
        "finite_termination": lambda: pins.test_distinct_eigs_and_finite_termination(6, 3),
        "pcg": pins.test_pcg_solution_and_monotone_in_m,
        "adjoint": pins.test_adjoint_matches_dense_gradient,
        "adjoint_fd": pins.test_adjoint_matches_finite_differences,
    }
    failed = []
    for name, fn in checks.items():
        try:
            fn()
        except Exception:  # noqa: BLE001 - any failure counts as caught
            failed.append(name)
    return failed


def _build(text, tmp_path, tag):
    src = tmp_path / f"{tag}.c"
    lib = tmp_path / f"lib{tag}.so"
    src.write_text(text)
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o",
                           str(lib), str(src), "-lm"])
    return str(lib)


def test_unmodified_oracle_passes_battery(oracle_lib, tmp_path):
    path = _build(open(SRC).read(), tmp_path, "orig")
    with orc.use_library(path):
        assert battery() == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, oracle_lib, tmp_path):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation site for {name} not unique"
    path = _build(text.replace(old, new), tmp_path, name)
    with orc.use_library(path):
        failed = battery()
    assert failed, f"mutant {name} passed every pin"
