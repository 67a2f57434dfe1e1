"""Pins for the pattern semantics (Tables 1 and 2) and the rewrite rules.

Every rule of Fig. 3 (algorithmic) and Fig. 4 (OpenCL-specific) is an
equality between two evaluable expressions; on integer-valued data the
equalities hold exactly, so these tests compare with ``==``.  The asum
derivation of Fig. 8, the three low-level asum expressions of Fig. 9 and the
vector-scaling example of Fig. 2 are evaluated with the parameters the paper
prints (tests/golden/paper_parameters.json).
"""
import json
import os
import random

import pytest

from oracle import patterns as P

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_parameters.json")))


def ints(n, seed, lo=-50, hi=50):
    r = random.Random(seed)
    return [r.randint(lo, hi) for _ in range(n)]


def floats(n, seed):
    r = random.Random(seed)
    return [r.uniform(-1, 1) for _ in range(n)]


# ---------------------------------------------------------------- Table 1 types


def test_split_join_shapes():
    x = list(range(24))
    s = P.split(6)(x)
    assert len(s) == 4 and all(len(c) == 6 for c in s)           # T[m] -> T[m/n][n]
    assert s[1] == [6, 7, 8, 9, 10, 11]
    assert P.join()(s) == x                                       # T[m][n] -> T[m*n]
    with pytest.raises(ValueError):
        P.split(5)(x)                                             # n must divide m


def test_reduce_returns_length_one_and_empty_is_z():
    assert P.reduce_(P.add, 0)([3, 4, 5]) == [12]
    assert P.reduce_(P.add, 0)([]) == [0]                        # reduce([]) = [z]
    # sequential left fold: order of application is visible with a
    # non-commutative f
    assert P.reduce_(lambda a, b: a * 10 + b, 0)([1, 2, 3]) == [123]


def test_zip_requires_equal_lengths():
    assert P.zip_([1, 2], [3, 4]) == [(1, 3), (2, 4)]
    with pytest.raises(ValueError):
        P.zip_([1], [1, 2])


def test_iterate_definition():
    f = lambda xs: [v + 1 for v in xs]
    assert P.iterate(0, f)([5]) == [5]                           # f^0 = id
    assert P.iterate(3, f)([5]) == [8]
    assert P.iterate(4, f)([1]) == P.compose(P.iterate(3, f), f)([1])   # f^(n+1) = f^n o f


def test_as_vector_as_scalar_shapes():
    x = list(range(16))
    v = P.as_vector(4)(x)
    assert len(v) == 4 and v[2] == P.Vec((8, 9, 10, 11))          # T[m] -> T4[m/4]
    nested = P.split(8)(x)
    vn = P.as_vector(4)(nested)                                   # innermost dimension only
    assert len(vn) == 2 and len(vn[0]) == 2
    with pytest.raises(ValueError):
        P.as_vector(3)(x)


# ---------------------------------------------------------------- reorder-stride


@pytest.mark.parametrize("size,s", [(12, 3), (16, 4), (262144 // 64, 64), (8, 1), (8, 8)])
def test_reorder_stride_formula_and_bijection(size, s):
    x = list(range(size))
    out = P.reorder_stride(s)(x)
    n = size // s
    assert out == [x[i // n + s * (i % n)] for i in range(size)]
    assert sorted(out) == x                                       # a permutation
    # after split^n, chunk t holds t, t+s, t+2s, ... (coalesced lanes)
    for t, chunk in enumerate(P.split(n)(out)):
        assert chunk == [t + s * k for k in range(n)]


def test_reorder_stride_rejects_bad_stride():
    with pytest.raises(ValueError):
        P.reorder_stride(5)(list(range(12)))


# ---------------------------------------------------------------- Fig. 3 algorithmic rules


def test_rule_iterate_decomposition():
    halve = P.compose(P.join(), P.map_(P.reduce_(P.add, 0)), P.split(2))
    x = ints(256, 1)
    for m, n in [(0, 3), (2, 3), (5, 1), (4, 4)]:
        assert P.iterate(m + n, halve)(x) == P.compose(P.iterate(m, halve), P.iterate(n, halve))(x)


def test_rule_reorder_commutativity():
    r = random.Random(2)
    x = ints(40, 3)
    perm = list(range(40))
    r.shuffle(perm)
    f = lambda v: 3 * v - 7
    assert P.compose(P.map_(f), P.reorder(perm))(x) == P.compose(P.reorder(perm), P.map_(f))(x)


@pytest.mark.parametrize("n", [1, 2, 5, 10, 60])
def test_rule_split_join(n):
    x = ints(60, 4)
    f = lambda v: v * v - v
    assert P.map_(f)(x) == P.compose(P.join(), P.map_(P.map_(f)), P.split(n))(x)


def test_rule_reduction_all_part_red_forms():
    x = ints(96, 5)
    red = P.reduce_(P.add, 0)
    base = red(x)
    r = random.Random(6)
    perm = list(range(96))
    r.shuffle(perm)
    part = P.part_red_reduce(P.add, 0)
    forms = [
        part,                                                     # -> reduce (m = 1)
        P.part_red_reorder(part, perm),                           # -> part-red o reorder
        P.part_red_split(part, 8),                                # -> join o map(part-red) o split^8
        P.part_red_iterate(P.part_red_split(part, 2), 3),         # -> iterate^3(part-red)
        P.part_red_split(P.part_red_split(part, 4), 24),          # nested split
    ]
    for form in forms:
        assert P.compose(red, form)(x) == base                     # reduce = reduce o part-red
    # the split form is a genuine partial reduction (1 <= m < n)
    assert len(P.part_red_split(part, 8)(x)) == 12


def test_rule_reduction_holds_only_with_identity_z():
    # part-red chunks each start at z; with z not the identity of f the
    # split form changes the result -- the reading that z must be f's identity.
    x = [1, 2, 3, 4]
    red = P.reduce_(P.add, 10)
    assert P.compose(red, P.part_red_split(P.part_red_reduce(P.add, 10), 2))(x) != red(x)


def test_rule_simplification():
    x = ints(48, 7)
    assert P.compose(P.join(), P.split(6))(x) == x                # join o split^n = id
    xs = P.split(6)(x)
    assert P.compose(P.split(6), P.join())(xs) == xs              # split^n o join = id
    assert P.compose(P.as_scalar(), P.as_vector(4))(x) == x       # asScalar o asVector = id
    v = P.as_vector(4)(x)
    assert P.compose(P.as_vector(4), P.as_scalar())(v) == v       # asVector o asScalar = id


def test_rule_fusion():
    x = ints(33, 8)
    f = lambda v: v + 5
    g = lambda v: -2 * v
    assert P.compose(P.map_(f), P.map_(g))(x) == P.map_(P.compose(f, g))(x)
    fused = P.reduce_seq(lambda acc, v: P.add(acc, g(v)), 0)
    assert P.compose(P.reduce_seq(P.add, 0), P.map_seq(g))(x) == fused(x)


# ---------------------------------------------------------------- Fig. 4 lowering rules


def test_lowering_map_variants_and_reduce_seq():
    x = ints(30, 9)
    f = lambda v: v * 7
    ref = P.map_(f)(x)
    for low in (P.map_workgroup, P.map_local, P.map_global, P.map_seq):
        assert low(f)(x) == ref
    assert P.reduce_seq(P.add, 0)(x) == P.reduce_(P.add, 0)(x)


def test_lowering_reorder_to_stride_or_id():
    x = ints(64, 10)
    red = P.reduce_(P.add, 0)
    assert P.compose(red, P.reorder_stride(8))(x) == red(x)
    assert P.compose(red, P.identity)(x) == red(x)


@pytest.mark.parametrize("width", [1, 2, 4, 8])
def test_lowering_vectorization(width):
    x = ints(64, 11)
    f = lambda v: 3 * v + 1
    vec = P.compose(P.as_scalar(), P.map_(P.vect(width, f)), P.as_vector(width))
    assert vec(x) == P.map_(f)(x)


# ---------------------------------------------------------------- Fig. 8 derivation


@pytest.mark.parametrize("n", [1, 4, 16, 64])
def test_asum_derivation_integer_exact(n):
    x = ints(256, 12)
    want = sum(abs(v) for v in x)
    for k, expr in enumerate(P.asum_derivation(n), start=1):
        assert expr(x) == [want], f"eq. ({k})"


def test_asum_derivation_float_bitwise_from_eq2():
    x = floats(1024, 13)
    vals = [expr(x)[0] for expr in P.asum_derivation(32)]
    # (2)-(8) share one association (chunk folds, then a fold of the chunk
    # sums), so they agree bit for bit; (1) differs only by rounding.
    assert len(set(vals[1:])) == 1
    assert abs(vals[0] - vals[1]) <= 1024 * 2.0 ** -52 * vals[0]


# ---------------------------------------------------------------- Fig. 9 low-level asum


def test_fig9a_paper_parameters():
    p = GOLDEN["fig9a_asum_gpu_scalar"]
    lanes = p["wg_chunk"] // p["lane_chunk"]
    assert lanes == 128 and 2 ** p["iterate"] == lanes            # iterate-7 reduces 128 -> 1
    x = ints(p["wg_chunk"] * 2, 14, -8, 8)
    expr = P.asum_lowlevel_gpu_scalar(p["wg_chunk"], p["lane_chunk"])
    assert expr(x) == [sum(abs(v) for v in x)]


def test_fig9b_paper_parameters():
    p = GOLDEN["fig9b_asum_gpu_vector"]
    lanes = p["wg_chunk"] // p["vector_width"] // p["per_lane"]
    assert lanes == 256 and 2 ** p["iterate"] == lanes            # iterate-8 reduces 256 -> 1
    x = ints(p["wg_chunk"] * 5, 15, -8, 8)
    expr = P.asum_lowlevel_gpu_vector(p["wg_chunk"], p["per_lane"], p["vector_width"])
    assert expr(x) == [sum(abs(v) for v in x)]


def test_fig9c_paper_parameters():
    p = GOLDEN["fig9c_asum_cpu"]
    assert p["wg_chunk"] == p["vector_width"] * p["lane_chunk"]   # one lane per work-group
    x = ints(p["wg_chunk"] * 3, 16, -8, 8)
    expr = P.asum_lowlevel_cpu(p["wg_chunk"], p["lane_chunk"], p["vector_width"])
    assert expr(x) == [sum(abs(v) for v in x)]


def test_fig9_partials_per_workgroup():
    # count what each work-group hands to the final reduce-seq o join
    x = ints(2048 * 4, 17, -8, 8)
    wg_b = P.compose(P.as_scalar(), P.map_workgroup(
        P.compose(P.join(), P.map_local(P.reduce_seq(P.vect(4, P.abs_and_plus), P.Vec((0,) * 4))),
                  P.split(512))), P.as_vector(4), P.split(2048))
    partials = P.join()(wg_b(x))
    assert len(partials) == 4 * len(x) // 2048                    # 4 floats per work-group
    assert sum(partials) == sum(abs(v) for v in x)


@pytest.mark.parametrize("wg,lane", [(64, 8), (128, 4), (256, 256)])
def test_fig9a_scaled_parameters(wg, lane):
    x = ints(wg * 3, 18)
    assert P.asum_lowlevel_gpu_scalar(wg, lane)(x) == [sum(abs(v) for v in x)]


# ---------------------------------------------------------------- Fig. 2 vector scaling


def test_fig2_vector_scaling():
    p = GOLDEN["fig2b_vector_scaling"]
    x = ints(p["wg_chunk"] * 3, 19, -1000, 1000)
    low = P.vector_scal_lowlevel(p["wg_chunk"], p["vector_width"])
    assert low(x) == P.vector_scal_highlevel()(x) == [3 * v for v in x]


# ---------------------------------------------------------------- Fig. 5 BLAS as patterns


def test_blas_patterns_small_closed_forms():
    assert P.scal(2, [1, -2, 3]) == [2, -4, 6]
    assert P.asum([1, -2, 3, -4]) == [10]
    assert P.dot([1, 2, 3], [4, -5, 6]) == [12]
    A = [[1, 2], [3, 4], [5, 6]]
    assert P.gemv(A, [1, -1], [10, 20, 30], 2, 0.5) == [-2 + 5, -2 + 10, -2 + 15]


def test_section7_sizes_imply_four_byte_elements():
    s = GOLDEN["section7_sizes"]
    assert s["small_vector_MB"] * 2 ** 20 == s["small_vector_elems_M"] * 2 ** 20 * 4
    assert s["large_vector_MB"] * 2 ** 20 == s["large_vector_elems_M"] * 2 ** 20 * 4
    m, n = s["gemv_small"]
    assert m * n * 4 == s["gemv_small_matrix_MB"] * 2 ** 20 and n * 4 == s["gemv_small_vector_KB"] * 1024
    m, n = s["gemv_large"]
    assert m * n * 4 == s["gemv_large_matrix_MB"] * 2 ** 20
    assert s["gemv_large_vector"] * 4 == s["gemv_large_vector_KB"] * 1024
