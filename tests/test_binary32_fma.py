"""Pins of the binary32 arithmetic used to evaluate low-level expressions:
the emulated fused multiply-add against the exact rational result rounded
once to binary32, including inputs where rounding the binary64 sum directly
(double rounding) gives the wrong binary32 value."""
import random
from fractions import Fraction

import numpy as np
import pytest

from tests import binary32 as F

def round_binary32(q: Fraction) -> float:
    """Exact rational -> binary32, nearest with ties to even (normal and
    subnormal range, no overflow)."""
    if q == 0:
        return 0.0
    sign = -1 if q < 0 else 1
    q = abs(q)
    e = q.numerator.bit_length() - q.denominator.bit_length()
    while Fraction(2) ** e > q:
        e -= 1
    while Fraction(2) ** (e + 1) <= q:
        e += 1
    e = max(e, -126)                       # subnormals share the minimum exponent
    ulp = Fraction(2) ** (e - 23)
    m = q / ulp
    f = m.numerator // m.denominator
    r = m - f
    if r > Fraction(1, 2) or (r == Fraction(1, 2) and f % 2 == 1):
        f += 1
    return sign * float(f * ulp)


def rand_f32(r: random.Random, lo=-30, hi=30) -> float:
    m = r.getrandbits(24) | (1 << 23)
    return float(np.float32(m * 2.0 ** (r.randint(lo, hi) - 23) * r.choice((-1, 1))))


def test_fma_equals_exact_single_rounding_random():
    r = random.Random(5)
    for _ in range(20_000):
        a, b = rand_f32(r), rand_f32(r)
        c = rand_f32(r, -60, 60)
        assert F.fma(a, b, c) == round_binary32(Fraction(a) * Fraction(b) + Fraction(c)), (a, b, c)


def test_fma_on_double_rounding_hazards():
    # a * b = 64 (1 - k^2 2^-46), just below 64, and c = T, a binary32 value
    # near 2^30 with an odd last significand bit (spacing 128 there).  The
    # exact sum T + 64 - k^2 2^-40 lies just below the halfway point T + 64,
    # so the correct binary32 result is T.  In binary64 (spacing 2^-22 at
    # 2^30) the sum rounds to exactly T + 64, and rounding that tie to even
    # gives T + 128: the plain binary64 evaluation is wrong on every case.
    r = random.Random(11)
    for _ in range(2000):
        k = r.randint(1, 300)
        a = float(np.float32(1 + k * 2.0 ** -23))
        b = float(np.float32(64 * (1 - k * 2.0 ** -23)))
        t = float(np.float32(2.0 ** 30 + 128 * (2 * r.randrange(1 << 22) + 1)))
        for sa, sc in ((1, 1), (-1, -1)):
            exact = round_binary32(Fraction(sa * a) * Fraction(b) + Fraction(sc * t))
            assert exact == sc * t
            assert float(np.float32(sa * a * b + sc * t)) == sc * (t + 128)    # double rounding
            assert F.fma(sa * a, b, sc * t) == exact, (k, t)


def test_fma_specials_and_signs():
    assert F.fma(2.0, 3.0, 1.0) == 7.0
    assert F.fma(-2.0, 3.0, 6.0) == 0.0 and str(F.fma(-2.0, 3.0, 6.0)) == "0.0"   # +0 under round to nearest
    assert F.fma(0.0, 5.0, -0.0) == 0.0
    t = float(np.float32(2.0 ** -149))                      # smallest subnormal
    assert F.fma(t, 0.5, 0.0) == 0.0                        # 2^-150 is a tie: to even (0)
    assert F.fma(t, 0.75, 0.0) == t                         # above the tie
    assert F.add(1.0, 2.0 ** -24) == 1.0 and F.add(1.0, 2.0 ** -23) == 1.0 + 2.0 ** -23
