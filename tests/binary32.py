"""IEEE binary32 arithmetic on Python floats, for evaluating low-level
expressions bit for bit (test infrastructure).

add(a, b): the binary32 sum, rounded to nearest even.
fma(a, b, c): a * b + c with ONE rounding to binary32 (round to nearest even),
emulated in binary64 with rounding to odd (Boldo and Melquiond, "Emulation of
FMA and correctly rounded sums: proved algorithms using rounding to odd",
IEEE Trans. Computers 57(4), 2008): for binary32 a and b the product is
exact in binary64 (at most 48 significant bits); the binary64 sum s = p + c
is rounded to nearest, its exact error e comes from TwoSum (Knuth); if e != 0
and s's last significand bit is 0, s moves one ulp towards the exact value,
which is the sum rounded to odd with 53 bits.  Rounding that to 24 bits
gives the correctly rounded result, as 53 >= 24 + 2.
"""
import math
import struct

_F32 = struct.Struct("<f")


def to_binary32(v: float) -> float:
    """Round a binary64 value to binary32 (nearest, ties to even; the C
    conversion behind struct's 'f' format), overflowing to infinity."""
    try:
        return _F32.unpack(_F32.pack(v))[0]
    except OverflowError:
        return math.copysign(math.inf, v)


def add(a, b) -> float:
    return to_binary32(float(a) + float(b))


def _last_bit(v: float) -> int:
    return struct.unpack("<Q", struct.pack("<d", v))[0] & 1


def fma(a, b, c) -> float:
    a, b, c = float(a), float(b), float(c)
    p = a * b                     # exact: two 24-bit significands
    s = p + c
    bb = s - p                    # TwoSum: p + c == s + e exactly
    e = (p - (s - bb)) + (c - bb)
    if e != 0.0 and _last_bit(s) == 0:
        s = math.nextafter(s, math.inf if e > 0 else -math.inf)
    return to_binary32(s)


def mul(a, b) -> float:
    return to_binary32(float(a) * float(b))
