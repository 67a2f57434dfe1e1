"""Executable semantics of the paper's patterns (TEST INFRASTRUCTURE ONLY).

Steuwer, Fensch, Dubach, "Patterns and Rewrite Rules for Systematic Code
Generation" (arXiv 1502.02389):

* Table 1 (Section 3.1): the high-level algorithmic patterns
  ``map, reduce, zip, split^n, join, iterate^n, reorder``;
* Table 2 (Section 3.2): the OpenCL-specific patterns
  ``map-workgroup, map-local, map-global, map-seq, reduce-seq,
  reorder-stride^s, toLocal, toGlobal, asVector^n, asScalar, vect^n``;
* Fig. 5 (Section 5.1): scal, asum, dot, gemv as compositions;
* Fig. 8 (Section 6.1): the eight-step derivation of a fused asum;
* Fig. 9 (Section 6.2): the three device-specific low-level asum expressions;
* Fig. 2 (Section 2): the vector-scaling example and its low-level form.

Arrays are Python lists; nesting carries the shape (the paper stores the
shape in the type, Section 3.1).  A primitive result is a length-1 list, as
the paper encodes every type as an array with primitives of length 1
(Section 3).  ``zip`` produces tuples; ``asVector`` produces :class:`Vec`
elements.  Every pattern is a function that returns a one-argument function
on an array, so expressions compose with :func:`compose` exactly as they are
written with the composition operator in the paper (rightmost applied first).

This module is plain Python for small inputs: it is what the rewrite-rule and
derivation tests evaluate.  The numeric BLAS oracle at full size is the C
code next to it; the two are independent implementations of the same
definitions, and tests compare them on tiny inputs.
"""
from __future__ import annotations

from functools import reduce as _functools_reduce
from typing import Callable, Sequence

# --------------------------------------------------------------------------
# composition
# --------------------------------------------------------------------------


def compose(*fs: Callable) -> Callable:
    """``compose(f, g, h)(x) == f(g(h(x)))`` -- the paper's ``f o g o h``."""

    def run(x):
        for f in reversed(fs):
            x = f(x)
        return x

    return run


def identity(x):
    return x


# --------------------------------------------------------------------------
# Table 1: algorithmic patterns
# --------------------------------------------------------------------------


def map_(f: Callable) -> Callable:
    """map(f): T[n] -> U[n], f applied to every element (outermost dim)."""
    return lambda xs: [f(x) for x in xs]


def reduce_(f: Callable, z) -> Callable:
    """reduce(f, z): T[] -> T[1].

    Evaluated as the sequential left fold (``acc = z; acc = f(acc, x_i)``),
    the only reduction the paper's code generator knows (reduce-seq,
    Table 2; reduction lowering, Fig. 4b).  ``f`` must be associative and
    commutative with ``z`` its identity for the rewrite rules to hold
    (Section 3.1); this function does not check that.
    """

    def run(xs):
        acc = z
        for x in xs:
            acc = f(acc, x)
        return [acc]

    return run


def zip_(a: Sequence, b: Sequence) -> list:
    """zip(a, b): T[n], U[n] -> <T,U>[n]; lengths must match."""
    if len(a) != len(b):
        raise ValueError(f"zip of unequal lengths {len(a)} and {len(b)}")
    return list(zip(a, b))


def split(n: int) -> Callable:
    """split^n: T[m] -> T[m/n][n].  Requires n to divide m."""
    if n <= 0:
        raise ValueError("split size must be positive")

    def run(xs):
        if len(xs) % n:
            raise ValueError(f"split^{n} of an array of length {len(xs)}")
        return [list(xs[i : i + n]) for i in range(0, len(xs), n)]

    return run


def join() -> Callable:
    """join: T[m][n] -> T[m*n] (merges the two outermost dimensions)."""
    return lambda xss: [x for xs in xss for x in xs]


def iterate(n: int, f: Callable) -> Callable:
    """iterate^n(f): f^0 = id, f^(n+1) = f^n o f."""
    if n < 0:
        raise ValueError("iterate count must be non-negative")

    def run(x):
        for _ in range(n):
            x = f(x)
        return x

    return run


def reorder(perm: Sequence[int]) -> Callable:
    """reorder: any permutation of the elements; here the given one.

    ``out[i] = in[perm[i]]``.
    """
    perm = list(perm)
    if sorted(perm) != list(range(len(perm))):
        raise ValueError("reorder needs a permutation")

    def run(xs):
        if len(xs) != len(perm):
            raise ValueError("permutation length mismatch")
        return [xs[p] for p in perm]

    return run


# --------------------------------------------------------------------------
# partial reduction (Fig. 3d) -- the four derivation forms
# --------------------------------------------------------------------------


def part_red_reduce(f, z):
    """part-red(f, z) -> reduce(f, z): the m = 1 form."""
    return reduce_(f, z)


def part_red_reorder(part, perm):
    """part-red(f, z) -> part-red(f, z) o reorder."""
    return compose(part, reorder(perm))


def part_red_split(part, n):
    """part-red(f, z) -> join o map(part-red(f, z)) o split^n.

    The one form that introduces parallelism (Section 4.1).
    """
    return compose(join(), map_(part), split(n))


def part_red_iterate(part, n):
    """part-red(f, z) -> iterate^n(part-red(f, z))."""
    return iterate(n, part)


# --------------------------------------------------------------------------
# Table 2: OpenCL-specific patterns (same semantics as their high-level
# counterparts; the name records where the work runs)
# --------------------------------------------------------------------------

map_workgroup = map_
map_local = map_
map_global = map_
map_seq = map_
reduce_seq = reduce_


def reorder_stride(s: int) -> Callable:
    """reorder-stride^s: out[i] = in[i / n + s * (i mod n)], n * s = size.

    (Section 3.2, "Reorder-stride".)  After a following split^n, chunk t
    holds the elements t, t + s, t + 2s, ... -- consecutive threads touch
    consecutive addresses.
    """

    def run(xs):
        size = len(xs)
        if s <= 0 or size % s:
            raise ValueError(f"reorder-stride^{s} of an array of length {size}")
        n = size // s
        return [xs[i // n + s * (i % n)] for i in range(size)]

    return run


def to_local(f: Callable) -> Callable:
    """toLocal(f): result of f placed in local memory -- a type cast only."""
    return f


def to_global(f: Callable) -> Callable:
    """toGlobal(f): result of f placed in global memory -- a type cast only."""
    return f


class Vec(tuple):
    """An OpenCL vector value (``int4``, ``float4``): a fixed-width tuple."""

    def __repr__(self):
        return f"Vec{tuple(self)!r}"


def as_vector(n: int) -> Callable:
    """asVector^n: T[]*[m] -> Tn[]*[m/n] on the innermost dimension."""

    def run(xs):
        if xs and isinstance(xs[0], list):
            return [run(x) for x in xs]
        if len(xs) % n:
            raise ValueError(f"asVector^{n} of an array of length {len(xs)}")
        return [Vec(xs[i : i + n]) for i in range(0, len(xs), n)]

    return run


def as_scalar() -> Callable:
    """asScalar: Tn[]*[m] -> T[]*[m*n] on the innermost dimension."""

    def run(xs):
        if xs and isinstance(xs[0], list):
            return [run(x) for x in xs]
        return [e for v in xs for e in v]

    return run


def vect(n: int, f: Callable) -> Callable:
    """vect^n(f): f applied lane-wise to width-n vector arguments."""

    def run(*args):
        for a in args:
            if not isinstance(a, Vec) or len(a) != n:
                raise TypeError(f"vect^{n} expects width-{n} vectors")
        return Vec(f(*lanes) for lanes in zip(*args))

    return run


# --------------------------------------------------------------------------
# user functions of the BLAS figure (Fig. 5)
# --------------------------------------------------------------------------


def add(x, y):
    return x + y


def mult(x, y):
    return x * y


def abs_(x):
    return -x if x < 0 else x


def abs_and_plus(acc, a):
    """The fused lambda of the asum derivation: acc + abs(a)."""
    return acc + abs_(a)


def mult_by(a):
    """mult(a): mult with its first argument bound."""
    return lambda x: mult(a, x)


# --------------------------------------------------------------------------
# Fig. 5: the BLAS programs as pattern compositions
# --------------------------------------------------------------------------


def scal(a, x):
    """scal(a, x) = map(mult(a), x)."""
    return map_(mult_by(a))(x)


def asum(x):
    """asum(x) = reduce(add, 0) o map(abs, x)."""
    return compose(reduce_(add, 0), map_(abs_))(x)


def dot(x, y):
    """dot(x, y) = reduce(add, 0) o map(mult) o zip(x, y)."""
    return compose(reduce_(add, 0), map_(lambda p: mult(*p)))(zip_(x, y))


def gemv(A, x, y, a, b):
    """gemv: z = map(scal(a) o dot(x), A); map(add) o zip(z, scal(b, y)).

    ``A`` is a list of rows.  ``dot(x)`` partially applied to a row is
    ``dot(x, row)``; ``scal(a)`` of its length-1 result is ``[a * d]``.
    Returns the new y as a list.
    """
    z = join()(map_(lambda row: scal(a, dot(x, row)))(A))
    return map_(lambda p: add(*p))(zip_(z, scal(b, y)))


# --------------------------------------------------------------------------
# Fig. 8: the asum derivation, equations (1)-(8)
# --------------------------------------------------------------------------


def asum_derivation(n: int) -> list:
    """The eight expressions of the fused-asum derivation, chunk size n.

    Each entry maps x to a length-1 list.  ``part-red(+, 0)`` is given the
    concrete m = 1 form (``reduce``), the choice eq. (7) makes explicit, so
    (2)-(8) share one association; (1) is the unsplit sequential fold.
    Eq. (8) is read with its missing closing parenthesis after ``0)``.
    """
    part = part_red_reduce(add, 0)
    return [
        # (1)
        compose(reduce_(add, 0), map_(abs_)),
        # (2) reduction rule twice
        compose(reduce_(add, 0), join(), map_(part), split(n), map_(abs_)),
        # (3) split-join on the map
        compose(reduce_(add, 0), join(), map_(part), split(n), join(),
                map_(map_(abs_)), split(n)),
        # (4) split^n o join -> id
        compose(reduce_(add, 0), join(), map_(part), map_(map_(abs_)), split(n)),
        # (5) map fusion
        compose(reduce_(add, 0), join(), map_(compose(part, map_(abs_))), split(n)),
        # (6) inner map lowered to map-seq
        compose(reduce_(add, 0), join(), map_(compose(part, map_seq(abs_))), split(n)),
        # (7) part-red -> reduce -> reduce-seq
        compose(reduce_(add, 0), join(),
                map_(compose(reduce_seq(add, 0), map_seq(abs_))), split(n)),
        # (8) reduce-seq o map-seq fusion
        compose(reduce_(add, 0), join(), map_(reduce_seq(abs_and_plus, 0)), split(n)),
    ]


# --------------------------------------------------------------------------
# Fig. 9: the device-specific low-level asum expressions
# --------------------------------------------------------------------------


def _log2_exact(v: int) -> int:
    k = v.bit_length() - 1
    if v <= 0 or (1 << k) != v:
        raise ValueError(f"{v} is not a power of two")
    return k


def asum_lowlevel_gpu_scalar(wg_chunk: int = 262144, lane_chunk: int = 2048) -> Callable:
    """Fig. 9a (tuned there for an Nvidia GPU), parametrised.

    reduce-seq o join o map-workgroup(
        join o toGlobal(map-local(map-seq(id))) o split-1
      o iterate-k(join o map-local(reduce-seq(plus, 0)) o split-2)
      o join o toLocal(map-local(reduce-seq(absAndPlus, 0))) o split-L
      o reorder-stride^s
    ) o split-W

    with W = 262144, L = 2048, s = W / L = 128 lanes and k = log2(128) = 7
    in the paper.  reorder-stride's stride, not printed, is the number of
    lane chunks (the reading that makes the lane accesses coalesced).
    """
    lanes = wg_chunk // lane_chunk
    if lanes * lane_chunk != wg_chunk:
        raise ValueError("lane chunk must divide the work-group chunk")
    k = _log2_exact(lanes)
    wg = compose(
        join(), to_global(map_local(map_seq(identity))), split(1),
        iterate(k, compose(join(), map_local(reduce_seq(add, 0)), split(2))),
        join(), to_local(map_local(reduce_seq(abs_and_plus, 0))), split(lane_chunk),
        reorder_stride(lanes),
    )
    return compose(reduce_seq(add, 0), join(), map_workgroup(wg), split(wg_chunk))


def asum_lowlevel_gpu_vector(wg_chunk: int = 2048, per_lane: int = 2, width: int = 4) -> Callable:
    """Fig. 9b (tuned there for an AMD GPU), parametrised.

    reduce-seq o join o asScalar o map-workgroup(
        join o toGlobal(map-local(map-seq(vect-4(id)))) o split-1
      o iterate-k(join o map-local(reduce-seq(vect-4(plus), vect-4(0))) o split-2)
      o join o toLocal(map-local(reduce-seq(vect-4(absAndPlus), vect-4(0))))
      o split-2 o reorder-stride^s
    ) o asVector-4 o split-2048

    Paper: 2048 floats per work-group = 512 float4, split-2 gives 256 lanes,
    iterate-8 reduces 256 -> 1 float4, so each work-group emits 4 floats.
    """
    vecs = wg_chunk // width
    lanes = vecs // per_lane
    if lanes * per_lane * width != wg_chunk:
        raise ValueError("inconsistent vector asum parameters")
    k = _log2_exact(lanes)
    zero = Vec((0,) * width)
    wg = compose(
        join(), to_global(map_local(map_seq(vect(width, identity)))), split(1),
        iterate(k, compose(join(), map_local(reduce_seq(vect(width, add), zero)), split(2))),
        join(), to_local(map_local(reduce_seq(vect(width, abs_and_plus), zero))),
        split(per_lane), reorder_stride(lanes),
    )
    return compose(reduce_seq(add, 0), join(), as_scalar(), map_workgroup(wg),
                   as_vector(width), split(wg_chunk))


def asum_lowlevel_cpu(wg_chunk: int = 32768, lane_chunk: int = 8192, width: int = 4) -> Callable:
    """Fig. 9c (tuned there for a multi-core CPU), parametrised.

    reduce-seq o join o asScalar o map-workgroup(
        join o map-local(reduce-seq(vect-4(absAndPlus), vect-4(0))) o split-8192
    ) o asVector-4 o split-32768

    32768 floats = 8192 float4 per work-group, split-8192 leaves one lane;
    no local memory, no reorder.  Each work-group emits 4 floats.
    """
    if (wg_chunk // width) % lane_chunk:
        raise ValueError("inconsistent CPU asum parameters")
    zero = Vec((0,) * width)
    wg = compose(join(), map_local(reduce_seq(vect(width, abs_and_plus), zero)),
                 split(lane_chunk))
    return compose(reduce_seq(add, 0), join(), as_scalar(), map_workgroup(wg),
                   as_vector(width), split(wg_chunk))


# --------------------------------------------------------------------------
# Fig. 2: vector scaling
# --------------------------------------------------------------------------


def mul3(x):
    return x * 3


def vector_scal_highlevel():
    """Fig. 2a: vectorScal = map(mul3)."""
    return map_(mul3)


def vector_scal_lowlevel(chunk: int = 1024, width: int = 4):
    """Fig. 2b: join o map-workgroup(asScalar o map-local(vectorize-4(mul3))
    o asVector-4) o split-1024."""
    return compose(
        join(),
        map_workgroup(compose(as_scalar(), map_local(vect(width, mul3)), as_vector(width))),
        split(chunk),
    )


def fold(f, xs, z):
    """Plain left fold helper for tests (functools.reduce with a start)."""
    return _functools_reduce(f, xs, z)
