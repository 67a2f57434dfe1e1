"""Pins for the binary64 BLAS oracle (the C code in oracle/).

Nothing here re-types the oracle's formulas: each expected value comes from a
closed form, exact integer or rational arithmetic, a correctly rounded sum
(math.fsum, Shewchuk's algorithm), an orthogonality identity, or a library
routine for the special case (numpy's float32 multiply, numpy/torch 16-bit
decoders).  A sequential binary64 fold of t_1..t_n has error at most
(n - 1) * 2^-53 * sum |t_i|; tests with floating-point data allow exactly
that bound against the correctly rounded sum.
"""
import math
import random
from fractions import Fraction

import numpy as np
import pytest
import torch

import oracle
from oracle import patterns as P

U = 2.0 ** -53


def seq_bound(terms_abs_sum, n):
    return max(n - 1, 0) * U * terms_abs_sum


# ---------------------------------------------------------------- decoders


def test_decode_f16_all_patterns():
    bits = np.arange(65536, dtype=np.uint32).astype(np.uint16)
    h = bits.view(np.float16)
    got = oracle.widen(h)
    want = h.astype(np.float64)
    nan = np.isnan(want)
    assert np.array_equal(np.isnan(got), nan)
    assert np.array_equal(got[~nan], want[~nan])
    assert np.array_equal(np.signbit(got[~nan]), np.signbit(want[~nan]))


def test_decode_bf16_all_patterns():
    bits = np.arange(65536, dtype=np.uint32).astype(np.uint16)
    got = oracle.widen(bits, dtype="bf16")
    want = torch.from_numpy(bits.view(np.int16).copy()).view(torch.bfloat16).to(torch.float64).numpy()
    nan = np.isnan(want)
    assert np.array_equal(np.isnan(got), nan)
    assert np.array_equal(got[~nan], want[~nan])
    assert np.array_equal(np.signbit(got[~nan]), np.signbit(want[~nan]))


def test_decode_f32_exact():
    r = np.random.default_rng(0)
    bits = r.integers(0, 2 ** 32, 4096, dtype=np.uint64).astype(np.uint32)
    x = bits.view(np.float32)
    got = oracle.widen(x)
    with np.errstate(all="ignore"):
        want = x.astype(np.float64)
    nan = np.isnan(want)
    assert np.array_equal(got[~nan], want[~nan]) and np.array_equal(np.isnan(got), nan)


# ---------------------------------------------------------------- scal


def test_scal_rounds_like_one_float32_multiply():
    r = np.random.default_rng(1)
    x = np.concatenate([
        r.uniform(-1, 1, 5000).astype(np.float32),
        (r.standard_normal(2000) * 1e30).astype(np.float32),
        np.array([1e-45, -1e-45, 1e-40, 0.0, -0.0, 3.4e38], dtype=np.float32),
    ])
    for alpha in (2.5, -0.1, 1.0, 3.0, np.float32(1.0 / 3.0)):
        with np.errstate(all="ignore"):
            got = oracle.scal(float(np.float32(alpha)), x).astype(np.float32)
            want = np.float32(alpha) * x                             # IEEE RNE single multiply
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


def test_scal_product_is_exact_in_binary64():
    x = np.array([0.1, -7.25, 1e-30, 3.0], dtype=np.float32)
    got = oracle.scal(2.5, x)
    for g, v in zip(got, x):
        assert Fraction(g) == Fraction(2.5) * Fraction(float(v))


def test_scal_identity_and_mul3():
    x = np.arange(-500, 500, dtype=np.float32)
    assert np.array_equal(oracle.scal(1.0, x), x.astype(np.float64))
    assert np.array_equal(oracle.scal(3.0, x), 3.0 * np.arange(-500, 500))   # Fig. 2 mul3
    assert oracle.scal(2.0, np.zeros(0, np.float32)).size == 0


# ---------------------------------------------------------------- asum


def test_asum_closed_forms():
    n = 1 << 20
    assert oracle.asum(np.full(n, 0.5, np.float32)) == 2.0 ** 19          # n |c|
    alt = np.where(np.arange(n) % 2 == 0, 0.75, -0.75).astype(np.float32)
    assert oracle.asum(alt) == 0.75 * n
    assert oracle.asum(np.zeros(0, np.float32)) == 0.0                     # reduce([]) = [0]
    assert oracle.asum(np.array([-3.0], np.float32)) == 3.0


def test_asum_integer_exact():
    g = torch.Generator().manual_seed(0)
    x = torch.randint(-8, 9, (1 << 20,), generator=g).float().numpy()
    assert oracle.asum(x) == float(sum(abs(int(v)) for v in x))


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
def test_asum_within_sequential_bound_of_fsum(dtype):
    g = torch.Generator().manual_seed(1)
    t = (torch.rand(200_000, generator=g) * 2 - 1)
    t = t.to({"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[dtype])
    if dtype == "bf16":
        x = t.view(torch.int16).numpy().view(np.uint16)
        vals = t.to(torch.float64).numpy()
    else:
        x = t.numpy()
        vals = x.astype(np.float64)
    got = oracle.asum(x, dtype=dtype if dtype == "bf16" else None)
    exact = math.fsum(abs(v) for v in vals)              # correctly rounded true sum
    assert abs(got - exact) <= seq_bound(exact, len(vals)) + U * exact


def test_asum_brute_force_rational_small():
    r = random.Random(2)
    for n in range(0, 65):
        x = np.array([r.uniform(-4, 4) for _ in range(n)], dtype=np.float32)
        exact = sum((abs(Fraction(float(v))) for v in x), Fraction(0))
        got = oracle.asum(x)
        assert abs(Fraction(got) - exact) <= Fraction(seq_bound(float(exact), n))


def test_asum_negative_zero_and_nan():
    assert oracle.asum(np.array([-0.0, -0.0], np.float32)) == 0.0
    assert math.isnan(oracle.asum(np.array([1.0, np.nan, 2.0], np.float32)))
    assert oracle.asum(np.array([-np.inf, 1.0], np.float32)) == math.inf


# ---------------------------------------------------------------- dot


def test_dot_orthogonal_closed_forms():
    n = 1 << 16
    ones = np.ones(n, np.float32)
    alt = np.where(np.arange(n) % 2 == 0, 1.0, -1.0).astype(np.float32)
    assert oracle.dot(ones, alt) == 0.0
    assert oracle.dot(alt, alt) == float(n)
    assert oracle.dot(np.zeros(0, np.float32), np.zeros(0, np.float32)) == 0.0


def _hadamard(k):
    H = np.array([[1.0]])
    for _ in range(k):
        H = np.block([[H, H], [H, -H]])
    return H.astype(np.float32)


def test_dot_hadamard_rows():
    H = _hadamard(6)                                   # 64 x 64 Sylvester matrix
    n = H.shape[0]
    for i in range(n):
        for j in range(0, n, 7):
            assert oracle.dot(np.ascontiguousarray(H[i]), np.ascontiguousarray(H[j])) == (n if i == j else 0.0)


def test_dot_integer_exact_and_symmetric():
    g = torch.Generator().manual_seed(3)
    x = torch.randint(-4, 5, (1 << 20,), generator=g).float().numpy()
    y = torch.randint(-4, 5, (1 << 20,), generator=g).float().numpy()
    want = float(sum(int(a) * int(b) for a, b in zip(x.tolist(), y.tolist())))
    assert oracle.dot(x, y) == want
    assert oracle.dot(y, x) == want


def test_dot_self_within_bound_of_fsum():
    g = torch.Generator().manual_seed(4)
    x = (torch.rand(100_000, generator=g) * 2 - 1).numpy()
    y = (torch.rand(100_000, generator=g) * 2 - 1).numpy()
    for a, b in ((x, x), (x, y)):
        prods = [float(u) * float(v) for u, v in zip(a.tolist(), b.tolist())]   # exact in binary64
        exact = math.fsum(prods)
        mass = math.fsum(abs(p) for p in prods)
        assert abs(oracle.dot(a, b) - exact) <= seq_bound(mass, len(prods)) + U * abs(exact)
        assert oracle.dot_absmass(a, b) == pytest.approx(mass, rel=1e-12)


def test_dot_brute_force_rational_small_mixed_storage():
    r = random.Random(5)
    for n in (1, 2, 3, 17, 64):
        xs = np.array([r.uniform(-2, 2) for _ in range(n)], np.float16)
        ys = np.array([r.uniform(-2, 2) for _ in range(n)], np.float32)
        exact = sum((Fraction(float(a)) * Fraction(float(b)) for a, b in zip(xs, ys)), Fraction(0))
        mass = sum(abs(float(a) * float(b)) for a, b in zip(xs, ys))
        got = oracle.dot(xs, ys)
        assert abs(Fraction(got) - exact) <= Fraction(seq_bound(mass, n))


# ---------------------------------------------------------------- gemv


def test_gemv_identity_matrix():
    n = 300
    r = np.random.default_rng(6)
    x = r.standard_normal(n).astype(np.float32)
    y = r.standard_normal(n).astype(np.float32)
    A = np.eye(n, dtype=np.float32)
    got = oracle.gemv(1.5, A, x, -0.25, y)
    want = np.float64(1.5) * x.astype(np.float64) + np.float64(-0.25) * y.astype(np.float64)
    assert np.array_equal(got, want)                     # dot with e_i is exact


def test_gemv_all_ones_is_scaled_sum():
    m, n = 7, 1000
    r = np.random.default_rng(7)
    x = r.uniform(-1, 1, n).astype(np.float32)
    y = r.uniform(-1, 1, m).astype(np.float32)
    got = oracle.gemv(2.0, np.ones((m, n), np.float32), x, 0.5, y)
    s = math.fsum(x.astype(np.float64))
    mass = math.fsum(abs(x.astype(np.float64)))
    for i in range(m):
        assert abs(got[i] - (2.0 * s + 0.5 * float(y[i]))) <= 2.0 * seq_bound(mass, n) + 4 * U * (2 * mass + 1)


def test_gemv_alpha_zero_and_beta_zero():
    r = np.random.default_rng(8)
    A = r.standard_normal((5, 9)).astype(np.float32)
    x = r.standard_normal(9).astype(np.float32)
    y = r.standard_normal(5).astype(np.float32)
    assert np.array_equal(oracle.gemv(0.0, A, x, 0.5, y), 0.5 * y.astype(np.float64))
    ynan = np.full(5, np.nan, np.float32)
    out = oracle.gemv(1.0, A, x, 0.0, ynan)              # beta == 0: y is not read
    assert np.all(np.isfinite(out))


def test_gemv_brute_force_rational_nonsquare_with_lda():
    r = random.Random(9)
    m, n, lda = 6, 5, 8
    A = np.full((m, lda), np.nan, np.float32)            # padding columns must never be read
    for i in range(m):
        for j in range(n):
            A[i, j] = r.uniform(-3, 3)
    x = np.array([r.uniform(-3, 3) for _ in range(n)], np.float32)
    y = np.array([r.uniform(-3, 3) for _ in range(m)], np.float32)
    alpha, beta = 1.25, -0.75
    got = oracle.gemv(alpha, A, x, beta, y, lda=lda)
    for i in range(m):
        d = sum((Fraction(float(A[i, j])) * Fraction(float(x[j])) for j in range(n)), Fraction(0))
        want = Fraction(alpha) * d + Fraction(beta) * Fraction(float(y[i]))
        mass = sum(abs(float(A[i, j]) * float(x[j])) for j in range(n))
        tol = abs(alpha) * seq_bound(mass, n) + 4 * U * (abs(alpha) * mass + abs(beta * float(y[i])))
        assert abs(Fraction(got[i]) - want) <= Fraction(tol)


def test_gemv_integer_exact():
    g = torch.Generator().manual_seed(10)
    m, n = 64, 512
    A = torch.randint(-8, 9, (m, n), generator=g).float().numpy()
    x = torch.randint(-8, 9, (n,), generator=g).float().numpy()
    y = torch.randint(-8, 9, (m,), generator=g).float().numpy()
    got = oracle.gemv(1.0, A, x, 0.5, y)
    Ai, xi = A.astype(np.int64), x.astype(np.int64)
    for i in range(m):
        assert got[i] == float(int((Ai[i] * xi).sum())) + 0.5 * float(y[i])


def test_gemv_empty_extents():
    y = np.arange(4, dtype=np.float32)
    out = oracle.gemv(2.0, np.zeros((4, 1), np.float32), np.zeros(0, np.float32), 0.5, y, lda=1)
    assert np.array_equal(out, 0.5 * y.astype(np.float64))   # n = 0: y' = beta y
    assert oracle.gemv(1.0, np.zeros((0, 3), np.float32), np.zeros(3, np.float32), 1.0,
                       np.zeros(0, np.float32)).size == 0


def test_gemv_absmass_definition():
    A = np.array([[1, -2], [-3, 4]], np.float32)
    x = np.array([5, -6], np.float32)
    y = np.array([-1, 2], np.float32)
    got = oracle.gemv_absmass(-2.0, A, x, -0.5, y)
    assert list(got) == [2 * (5 + 12) + 0.5, 2 * (15 + 24) + 1.0]


# ---------------------------------------------------------------- two independent oracles


def test_c_oracle_matches_pattern_evaluator_bitwise():
    r = random.Random(11)
    for n in (0, 1, 5, 33, 200):
        x = np.array([r.uniform(-1, 1) for _ in range(n)], np.float32)
        y = np.array([r.uniform(-1, 1) for _ in range(n)], np.float32)
        xf, yf = [float(v) for v in x], [float(v) for v in y]
        assert oracle.asum(x) == P.asum(xf)[0]
        assert oracle.dot(x, y) == P.dot(xf, yf)[0]
        assert list(oracle.scal(0.5, x)) == P.scal(0.5, xf)
    m, n = 4, 6
    A = np.array([[r.uniform(-1, 1) for _ in range(n)] for _ in range(m)], np.float32)
    x = np.array([r.uniform(-1, 1) for _ in range(n)], np.float32)
    y = np.array([r.uniform(-1, 1) for _ in range(m)], np.float32)
    want = P.gemv([[float(v) for v in row] for row in A], [float(v) for v in x], [float(v) for v in y], 1.5, 0.25)
    assert list(oracle.gemv(1.5, A, x, 0.25, y)) == want


def test_rejects_bad_arguments():
    with pytest.raises(ValueError):
        oracle.dot(np.zeros(3, np.float32), np.zeros(4, np.float32))
    with pytest.raises(TypeError):
        oracle.asum(np.zeros(3, np.int32))


# ---------------------------------------------------------------- split-join form (rule 3d)

PAR_THREADS = (1, 2, 3, 7, 8, 16)


def test_split_join_integer_exact_every_split():
    g = torch.Generator().manual_seed(6)
    n = (1 << 18) + 5
    x = torch.randint(-8, 9, (n,), generator=g).float().numpy()
    y = torch.randint(-4, 5, (n,), generator=g).float().numpy()
    want_a = float(sum(abs(int(v)) for v in x.tolist()))
    want_d = float(sum(int(a) * int(b) for a, b in zip(x.tolist(), y.tolist())))
    for p in PAR_THREADS:
        assert oracle.asum_par(x, p) == want_a, p
        assert oracle.dot_par(x, y, p) == want_d, p
    # fewer elements than threads, empty, single element
    for m in (0, 1, 5):
        xs, ys = np.ascontiguousarray(x[:m]), np.ascontiguousarray(y[:m])
        assert oracle.asum_par(xs, 8) == float(sum(abs(int(v)) for v in xs.tolist()))
        assert oracle.dot_par(xs, ys, 8) == float(sum(int(a) * int(b) for a, b in zip(xs.tolist(), ys.tolist())))


def test_split_join_one_chunk_is_the_sequential_form():
    g = torch.Generator().manual_seed(7)
    x = (torch.rand(100_003, generator=g) * 2 - 1).numpy()
    y = (torch.rand(100_003, generator=g) * 2 - 1).numpy()
    assert oracle.asum_par(x, 1) == oracle.asum(x)
    assert oracle.dot_par(x, y, 1) == oracle.dot(x, y)


@pytest.mark.parametrize("p", PAR_THREADS)
def test_split_join_within_bound_of_fsum(p):
    g = torch.Generator().manual_seed(8)
    t = (torch.rand(60_001, generator=g) * 2 - 1)
    x = t.numpy()
    y = (torch.rand(60_001, generator=g) * 2 - 1).numpy()
    vals = x.astype(np.float64)
    exact = math.fsum(abs(v) for v in vals)
    # each term passes through at most (chunk - 1) + (p - 1) <= n - 1 additions
    assert abs(oracle.asum_par(x, p) - exact) <= seq_bound(exact, len(vals)) + U * exact
    prods = [float(a) * float(b) for a, b in zip(x.tolist(), y.tolist())]
    ed, mass = math.fsum(prods), math.fsum(abs(q) for q in prods)
    assert abs(oracle.dot_par(x, y, p) - ed) <= seq_bound(mass, len(prods)) + U * abs(ed)


def test_split_join_16bit_storage_and_scal_map():
    g = torch.Generator().manual_seed(9)
    t = torch.randint(-8, 9, (40_000,), generator=g).to(torch.bfloat16)
    xb = t.view(torch.int16).numpy().view(np.uint16)
    want = float(sum(abs(int(v)) for v in t.float().tolist()))
    for p in (3, 8):
        assert oracle.asum_par(xb, p, dtype="bf16") == want
    xf = (torch.rand(50_001, generator=g) * 2 - 1).numpy()
    want_s = xf.astype(np.float64) * 2.5                  # exact: binary32 x 2.5 fits binary64
    for p in PAR_THREADS:
        assert np.array_equal(oracle.scal_par(2.5, xf, p), want_s), p


def test_split_join_rejects_bad_thread_counts():
    x = np.ones(4, np.float32)
    for p in (0, -1, 257):
        with pytest.raises(RuntimeError):
            oracle.asum_par(x, p)
