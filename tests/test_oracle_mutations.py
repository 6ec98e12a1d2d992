"""Plants plausible mistakes in copies of the oracle's C source (on the CPU)
and checks that the pin suite in test_oracle_pins.py rejects every one of
them: a dropped block, a wrong sign, the factor -i instead of i, a missing
1/2, a transposed block, the reversed digit order of the string index, the
printed n-1 loop bound, the wrong Y matrix, a zero test that ignores the
imaginary part or NaN, and transposed reads in the definition and synthesis,
plus mistakes in the multithreaded form of Algorithm 2 (loop bound, a
dropped row range).
"""
import os

import pytest

from oracle import oracle as O
import test_oracle_pins as P

MUTANTS = {
    "dropped_block_in_Omega0": ("re = (a11[0] + a22[0]) * 0.5; im = (a11[1] + a22[1]) * 0.5;",
                                "re = (a11[0]) * 0.5; im = (a11[1]) * 0.5;"),
    "sign_of_Omega3": ("re = (a11[0] - a22[0]) * 0.5; im = (a11[1] - a22[1]) * 0.5;",
                       "re = (a22[0] - a11[0]) * 0.5; im = (a22[1] - a11[1]) * 0.5;"),
    "minus_i_in_Omega2": ("re = -di * 0.5;\n          im = dr * 0.5;",
                          "re = di * 0.5;\n          im = -dr * 0.5;"),
    "missing_half_in_Omega1": ("re = (a12[0] + a21[0]) * 0.5; im = (a12[1] + a21[1]) * 0.5;",
                               "re = (a12[0] + a21[0]); im = (a12[1] + a21[1]);"),
    "wrong_quadrant_for_A12": ("const double* a12 = M + 2 * (r * dim + c + h);",
                               "const double* a12 = M + 2 * ((r + h) * dim + c + h);"),
    "reversed_digit_order": ("tpd_rec(ctx, C, m - 1, prefix * 4 + (uint64_t)t);",
                             "tpd_rec(ctx, C, m - 1, prefix + ((uint64_t)t << (2 * (depth - 1))));"),
    "printed_loop_bound_n_minus_1": ("for (int i = 1; i <= n; ++i) {\n    const int m = n - i + 1; /* parent",
                                     "for (int i = 1; i < n; ++i) {\n    const int m = n - i + 1; /* parent"),
    "multithreaded_form_loop_bound_n_minus_1": (
        "for (int i = 1; i <= n; ++i) {\n    const int m = n - i + 1;\n    const uint64_t psize",
        "for (int i = 1; i < n; ++i) {\n    const int m = n - i + 1;\n    const uint64_t psize"),
    "multithreaded_form_drops_last_row_range": ("const uint64_t r0 = h * part / split, r1 = h * (part + 1) / split;",
                                                "const uint64_t r0 = h * part / split, r1 = h * part / split + "
                                                "(h / split > 1 ? h / split - 1 : 1);"),
    "wrong_sign_of_Y": ("/* Y */ {{-1, 3}, {1, -1}},", "/* Y */ {{-1, 1}, {3, -1}},"),
    "zero_test_ignores_imag": ("if (re != 0.0 || im != 0.0 || re != re || im != im) nonzero = 1;",
                               "if (re != 0.0 || re != re) nonzero = 1;"),
    "zero_test_ignores_nan": ("if (re != 0.0 || im != 0.0 || re != re || im != im) nonzero = 1;",
                              "if (fabs(re) > 0.0 || fabs(im) > 0.0) nonzero = 1;"),
    "transposed_read_in_definition": ("const double* a = A + 2 * ((i ^ x) * dim + i); /* A[i^x][i] */",
                                      "const double* a = A + 2 * (i * dim + (i ^ x));"),
    "transposed_write_in_synthesis": ("double* a = A + 2 * (i * dim + (i ^ x)); /* sigma^t[i][i^x] */",
                                      "double* a = A + 2 * ((i ^ x) * dim + i);"),
    "xy_mask_uses_Z": ("if (t == 1 || t == 2) x |= (uint64_t)1 << (n - k);",
                       "if (t == 1 || t == 3) x |= (uint64_t)1 << (n - k);"),
    "dense_definition_transposed": ("const double* a = A + 2 * (j * dim + i); /* A[j][i] */",
                                    "const double* a = A + 2 * (i * dim + j);"),
}


def pin_checks(golden_dir):
    return [
        lambda: P.test_one_qubit_worked_examples(golden_dir),
        lambda: P.test_tfim_n3_golden(golden_dir),
        P.test_index_convention_order_pins,
        lambda: P.test_definition_matches_numpy_kron(2),
        P.test_dense_and_sparse_definitions_agree_n4,
        P.test_xy_mask_and_diagonal_form,
        lambda: P.test_integer_inputs_bit_exact(4),
        lambda: P.test_gaussian_recursion_vs_brute_force(5),
        P.test_partial_tpd_matches_full,
        lambda: P.test_tfim_closed_form(4),
        P.test_parseval_and_reconstruction,
        P.test_hermitian_weights_exactly_real,
        P.test_zero_and_nan_semantics,
        P.test_tensor_factorisation,
        P.test_purely_imaginary_cmw_is_live,
        lambda: P.test_multithreaded_algorithm_2_is_the_serial_one(3),
    ]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_planted_mistake(name, tmp_path, golden_dir):
    old, new = MUTANTS[name]
    src = O.source_text()
    assert src.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    lib = O.compile_variant(src.replace(old, new), os.path.join(str(tmp_path), name + ".so"))
    failures = 0
    with O.use_library(lib):
        for check in pin_checks(golden_dir):
            try:
                check()
            except (AssertionError, RuntimeError):
                failures += 1
    assert failures > 0, f"no pin rejects the planted mistake '{name}'"


def test_unmutated_oracle_passes_all_checks(golden_dir):
    for check in pin_checks(golden_dir):
        check()
