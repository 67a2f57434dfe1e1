"""Planted mistakes in the C oracle must each fail at least one pin.

Each mutant is a one-line textual change to a temporary copy of
oracle/lift_oracle.c (a dropped term, a wrong sign, a wrong index or stride,
a transposed operand, a wrong decoder constant), compiled with gcc on the CPU
and swapped in for the real library while a fast subset of the pins in
test_oracle_blas.py runs.  The real oracle is untouched.
"""
import ctypes
import os
import subprocess

import pytest

import oracle
from tests import test_oracle_blackscholes as bs
from tests import test_oracle_md as md
from tests import test_oracle_blas as pins

SRC = open(os.path.join(os.path.dirname(oracle.__file__), "lift_oracle.c")).read()

MUTANTS = {
    "reduce_drops_last_term": ("for (int64_t i = 0; i < n; ++i)\n        acc = f(acc, in[i], env);",
                               "for (int64_t i = 0; i < n - 1; ++i)\n        acc = f(acc, in[i], env);"),
    "reduce_wrong_start": ("double acc = z;", "double acc = z + 1.0;"),
    "abs_wrong_sign": ("return (x < 0) ? -x : x; }", "return (x < 0) ? x : x; }"),
    "dot_adds_instead_of_mult": ("return dot_common(n, xt, x, yt, y, fn_mult, result);",
                                 "return dot_common(n, xt, x, yt, y, fn_add, result);"),
    "scal_adds": ("return *(const double *)env * x; }", "return *(const double *)env + x; }"),
    "gemv_row_stride_n": ("(size_t)i * (size_t)lda * esz, 1, row)", "(size_t)i * (size_t)n * esz, 1, row)"),
    "gemv_transposed": ("widen(n, at, (const char *)A + (size_t)i * (size_t)lda * esz, 1, row);",
                        "widen(n, at, (const char *)A + (size_t)i * esz, lda, row);"),
    "gemv_beta_uses_alpha": ("map1(m, wy, by, fn_mult_bound, &b);", "map1(m, wy, by, fn_mult_bound, &alpha);"),
    "gemv_drops_alpha": ("map1(1, one, scaled, fn_mult_bound, &a);", "scaled[0] = one[0];"),
    "f16_wrong_bias": ("e - 25);", "e - 24);"),
    "f16_subnormal_scale": ("ldexp((double)m, -24)", "ldexp((double)m, -25)"),
    "bf16_wrong_shift": ("(uint32_t)h << 16", "(uint32_t)h << 15"),
    "zip_swaps_pairs": ("out[i].a = a[i];\n        out[i].b = b[i];", "out[i].a = a[i];\n        out[i].b = a[i];"),
    "split_join_drops_last_chunk": ("for (int64_t i = 0; i < p; ++i)\n            acc = fn_add(acc, c[i].partial, NULL);",
                                    "for (int64_t i = 0; i + 1 < p; ++i)\n            acc = fn_add(acc, c[i].partial, NULL);"),
    "split_join_byte_offsets": ("c[i].x = (const char *)x + (size_t)lo * elem_size(xt);",
                                "c[i].x = (const char *)x + (size_t)lo;"),
    "split_join_chunk_too_short": ("int64_t k = n > 0 ? (n + p - 1) / p : 0;", "int64_t k = n > 0 ? n / p : 0;"),
    "bs_d2_adds_spread": ("return d1 - q->v * sqrt(q->T);", "return d1 + q->v * sqrt(q->T);"),
    "bs_drops_half_variance": ("(q->r + 0.5 * q->v * q->v) * q->T)", "(q->r) * q->T)"),
    "bs_put_wrong_tail": ("* cnd(-d2) - s * cnd(-d1);", "* cnd(d2) - s * cnd(-d1);"),
    "bs_call_undiscounted": ("return s * cnd(d1) - q->K * exp(-q->r * q->T) * cnd(d2);",
                             "return s * cnd(d1) - q->K * cnd(d2);"),
    "bs_cnd_wrong_scale": ("0.5 * erfc(-x / sqrt(2.0))", "0.5 * erfc(-x / 2.0)"),
    "md_force_sign_x": ("double dx = (double)p[0] - q[0]", "double dx = (double)q[0] - p[0]"),
    "md_drops_repulsion_factor": ("* s6 * 2.0 * s6;", "* s6 * s6;"),
    "md_cutoff_compares_squared_distance": ("sqrt(d0 * d0 + d1 * d1 + d2 * d2) < t;", "d0 * d0 + d1 * d1 + d2 * d2 < t;"),
    "md_cutoff_not_strict": ("sqrt(d0 * d0 + d1 * d1 + d2 * d2) < t;", "sqrt(d0 * d0 + d1 * d1 + d2 * d2) <= t;"),
    "md_cutoff_rounded_like_binary32": (
        "return sqrt(d0 * d0 + d1 * d1 + d2 * d2) < t;",
        "volatile float fx = (float)d0, fy = (float)d1, fz = (float)d2, xx = fx * fx, yy = fy * fy, zz = fz * fz;"
        " volatile float r2 = (xx + yy) + zz; return r2 < (float)(t * t);"),
    "md_ignores_cutoff": ("if (md_within(p, q, m->t)) {", "if (1) {"),
    "md_sigma_not_squared": ("md_params m = {24.0 * epsilon, sigma * sigma,", "md_params m = {24.0 * epsilon, sigma,"),
}

FAST_PINS = [
    pins.test_decode_f16_all_patterns,
    pins.test_decode_bf16_all_patterns,
    pins.test_scal_rounds_like_one_float32_multiply,
    pins.test_scal_identity_and_mul3,
    pins.test_asum_closed_forms,
    pins.test_asum_brute_force_rational_small,
    pins.test_dot_orthogonal_closed_forms,
    pins.test_dot_hadamard_rows,
    pins.test_dot_brute_force_rational_small_mixed_storage,
    pins.test_gemv_identity_matrix,
    pins.test_gemv_alpha_zero_and_beta_zero,
    pins.test_gemv_brute_force_rational_nonsquare_with_lda,
    pins.test_gemv_absmass_definition,
    pins.test_split_join_integer_exact_every_split,
    pins.test_split_join_16bit_storage_and_scal_map,
    bs.test_put_call_parity_and_homogeneity,
    bs.test_at_the_forward_call_equals_put,
    bs.test_matches_numerical_integration_all_cases,
    md.test_gradient_all_cases,
    md.test_zero_force_at_potential_minimum,
    md.test_newton_third_law_on_symmetric_lists,
    md.test_cutoff_and_empty_slots,
    md.test_cutoff_is_the_exact_distance,
]


@pytest.fixture(scope="module")
def builddir(tmp_path_factory):
    return tmp_path_factory.mktemp("mutants")


def _build(src: str, path: str):
    c = path + ".c"
    with open(c, "w") as f:
        f.write(src)
    subprocess.run(["gcc", "-O1", "-std=c99", "-ffp-contract=off", "-pthread", "-fPIC", "-shared", "-o", path, c, "-lm"],
                   check=True)


def test_mutations_apply_cleanly():
    for name, (old, new) in MUTANTS.items():
        assert SRC.count(old) == 1, name


def test_unmutated_copy_passes_fast_pins(builddir):
    path = str(builddir / "base.so")
    _build(SRC, path)
    saved = oracle._lib
    try:
        oracle._lib = oracle._configure(ctypes.CDLL(path))
        for pin in FAST_PINS:
            pin()
    finally:
        oracle._lib = saved


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, builddir):
    old, new = MUTANTS[name]
    path = str(builddir / f"{name}.so")
    _build(SRC.replace(old, new), path)
    saved = oracle._lib
    caught = []
    try:
        oracle._lib = oracle._configure(ctypes.CDLL(path))
        for pin in FAST_PINS:
            try:
                pin()
            except (AssertionError, RuntimeError, ValueError):
                caught.append(pin.__name__)
    finally:
        oracle._lib = saved
    assert caught, f"mutant {name} survived every pin"
