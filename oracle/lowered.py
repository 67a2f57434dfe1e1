"""Low-level asum / dot expressions for a launch configuration (TEST INFRASTRUCTURE).

The paper lowers ``asum = reduce(+,0) . map(abs)`` to device-specific
expressions built from its OpenCL patterns (Fig. 9, Section 6.2), choosing
split factors and vector widths per device.  This module builds the same kind
of expression for one launch of the GPU library's asum -- from the launch
rules its interface documents (split rounded up to whole steps of
block * unroll vectors, one work-group per chunk, a scalar head before the
first aligned vector and a scalar tail after the last) and the reduction tree
its kernels use -- and evaluates it with the patterns of ``patterns.py``:

    reduce-seq o join o map-workgroup(
        toGlobal(...)
      o reduce-seq(plus)                       (wave totals, in wave order)
      o map-wave(iterate-6(join o map(reduce-seq(plus, 0)) o split-2))
      o split-64
      o map-local(iterate-log2(E)(join o map(reduce-seq(plus, 0)) o split-2)
                  o asScalar o reduce-seq(vect-E(absAndPlus), vect-E(0)))
      o split-(C/B) o reorder-stride^B
    ) o split-C o asVector-E                    (C vectors per work-group)

followed, when there is more than one work-group, by the final combine of
the work-group partials: lane t of one wavefront folds partials t, t+64, ...,
then the wave's butterfly (the batched form combines a problem's tile
partials over a whole work-group: lane t of B folds t, t+B, ..., then the
work-group tree).  The head and tail scalars are added to component 0 of lanes of the
first and last work-group.

``evaluate(x, shape, add)`` runs the expression with a caller-given binary
``add``: with exact integer arithmetic it must equal asum (every knob point
is a valid derivation), and with IEEE binary32 addition it predicts the
library's floating-point result bit for bit.

``evaluate_dot(x, y, shape, add, fma)`` does the same for
``dot = reduce(+,0) . map(*) . zip`` (Fig. 5): the work-group and lane
structure is the asum one, over ``zip(asVector-E x, asVector-E y)``, and the
lane step is ``reduce-seq(vect-E(multAndPlus))`` with multAndPlus(acc, a, b)
= fma(a, b, acc) (the fused form of rule 3f; reading 7 allows the
contraction); head and tail pairs enter component 0 of their lanes the same
way.  Shares no code with the GPU library.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

from . import patterns as P


@dataclass(frozen=True)
class Shape:
    """How one asum launch cuts n elements (all sizes in elements / vectors)."""

    n: int
    head: int        # scalars before the first aligned vector
    e: int           # elements per vector load (asVector width)
    nvec: int        # whole vectors after the head
    block: int       # work-group size B
    chunk: int       # vectors per work-group C (a multiple of B * unroll)
    grid: int        # work-groups G
    step: int = 0    # B * unroll vectors: with interleave, work-group b takes
    interleave: bool = False   # steps b, b + G, ... instead of one chunk
    final_lanes: int = 64      # lanes of the final combine of the G partials
    runs: bool = False         # lane t takes the t-th contiguous run of C / B
    #                            vectors (split) instead of t, t + B, ... (reorder-stride)
    seq: bool = False          # the lane partials meet in one reduce-seq in lane
    #                            order instead of the tree

    @property
    def tail(self) -> int:
        return self.n - self.head - self.nvec * self.e


def launch_shape(n: int, elem_bytes: int, vec_bytes: int, block: int, unroll: int, split: int,
                 misalign_elems: int = 0, max_workgroups: int = 8192, interleave: bool = False,
                 final_lanes: int = 64, lane_form: int = 0) -> Shape:
    """The documented launch rules for an explicit split (elements per chunk).

    ``misalign_elems``: how many elements past a vec_bytes boundary x starts.
    ``interleave``: the work-groups (as many as the split gives) take steps
    of block * unroll vectors round-robin instead of one chunk each.
    ``final_lanes``: lanes that fold the work-group partials at the end (one
    wavefront in the per-call kernels; a whole work-group in the batched
    form's per-problem combine); a block of fewer than 64 lanes folds them
    over its own lanes.
    ``lane_form``: bit 0 = the lanes meet in lane order, bit 1 = lanes on
    contiguous runs (the interface's lane forms).
    """
    if block < 64:
        final_lanes = min(final_lanes, block)
    e = vec_bytes // elem_bytes
    head = 0 if misalign_elems % e == 0 else e - misalign_elems % e
    head = min(head, n)
    nvec = (n - head) // e
    step = block * unroll
    chunk = max(1, -(-split // e))
    chunk = max(step, -(-chunk // step) * step)
    if -(-nvec // chunk) > max_workgroups:
        chunk = -(-(-(-nvec // max_workgroups)) // step) * step
    grid = max(1, -(-nvec // chunk))
    return Shape(n, head, e, nvec, block, chunk, grid, step, interleave, final_lanes,
                 bool(lane_form & 2), bool(lane_form & 1))


def _pairwise(values, add):
    """iterate-log2(k)(join o map(reduce-seq(plus, 0)) o split-2) on a power-of-two list.

    Each level folds adjacent pairs; reduce-seq(plus, 0) of a pair is
    plus(plus(0, a), b), written here as add(a, b) because 0 + a == a.
    """
    k = len(values)
    if k & (k - 1):
        raise ValueError("pairwise tree needs a power-of-two length")
    level = list(values)
    while len(level) > 1:
        level = [add(a, b) for a, b in P.split(2)(level)]
    return level[0]


def _block_tree(lane_values, add):
    """Wave butterflies (iterate-6 over 64 lanes) then a fold of the wave
    totals; fewer than 64 lanes (a power of two) meet in one pairwise tree."""
    waves = P.split(64)(lane_values) if len(lane_values) >= 64 else [lane_values]
    totals = [_pairwise(w, add) for w in waves]
    acc = totals[0]
    for t in totals[1:]:
        acc = add(acc, t)
    return acc


def evaluate(x, shape: Shape, add, absval, zero):
    """The low-level expression of one asum launch on the list x.

    add(a, b), absval(a) and zero define the arithmetic (exact integers, or
    binary32).  Returns the single result.
    """
    s = shape
    if len(x) != s.n:
        raise ValueError("input length differs from the launch shape")
    E = s.e
    vec_part = list(x[s.head: s.head + s.nvec * E])
    vectors = P.as_vector(E)(vec_part) if vec_part else []
    abs_and_plus = lambda acc, a: add(acc, absval(a))
    lane_step = P.vect(E, abs_and_plus)                      # vect-E(absAndPlus)
    scalar_step = abs_and_plus
    return _launch(vectors, P.Vec((zero,) * E), x[: s.head], x[s.head + s.nvec * E:], s, lane_step,
                   scalar_step, add, zero)


def evaluate_dot(x, y, shape: Shape, add, fma, zero):
    """The low-level expression of one dot launch on the lists x and y.

    fma(a, b, c) is a * b + c with the arithmetic's rounding (one rounding in
    binary32; exact on integers), add(a, b) the tree's addition.
    """
    s = shape
    if len(x) != s.n or len(y) != s.n:
        raise ValueError("input length differs from the launch shape")
    E = s.e
    lo, hi = s.head, s.head + s.nvec * E
    xv = P.as_vector(E)(list(x[lo:hi])) if hi > lo else []
    yv = P.as_vector(E)(list(y[lo:hi])) if hi > lo else []
    pairs = P.zip_(xv, yv)                                    # zip(asVector x, asVector y)
    mult_and_plus = lambda acc, a, b: fma(a, b, acc)
    lane_vect = P.vect(E, mult_and_plus)                      # vect-E(multAndPlus)
    lane_step = lambda acc, pair: lane_vect(acc, pair[0], pair[1])
    scalar_step = lambda acc, pair: mult_and_plus(acc, pair[0], pair[1])
    zero_vec = P.Vec((zero,) * E)
    head = list(zip(x[:lo], y[:lo]))
    tail = list(zip(x[hi:], y[hi:]))
    return _launch(pairs, (zero_vec, zero_vec), head, tail, s, lane_step, scalar_step, add, zero)


def _launch(vectors, zero_item, head, tail0, s: Shape, lane_step, scalar_step, add, zero):
    """The launch's partition and trees over the vector items (vectors, or
    pairs of vectors for dot); head / tail items enter lane component 0 of
    the first / last work-group through scalar_step."""
    B, C, E, G = s.block, s.chunk, s.e, s.grid
    zero_vec = P.Vec((zero,) * E)
    if s.interleave:
        # steps of B * unroll vectors, the last one padded with zero vectors;
        # work-group b's run is steps b, b + G, ... (join o reorder-stride-G
        # o split-step), each run padded to whole lanes
        steps = P.split(s.step)(vectors + [zero_item] * (-len(vectors) % s.step)) if vectors else []
        runs = [P.join()(steps[b::G]) for b in range(G)]
        width = max(len(r) for r in runs) if runs else 0
        width = -(-max(width, B) // B) * B
        chunks = [r + [zero_item] * (width - len(r)) for r in runs]
    else:
        # ragged last chunk: pad with zero items (neutral in the sum; reading 1)
        vectors = list(vectors) + [zero_item] * (G * C - len(vectors))
        chunks = P.split(C)(vectors)
    lane_fold = P.reduce_seq(lane_step, zero_vec)

    partials = []
    for b, chunk in enumerate(chunks):                              # map-workgroup
        if s.runs:
            lanes = P.split(len(chunk) // B)(chunk)                 # lane t: the t-th run
        else:
            lanes = P.split(len(chunk) // B)(P.reorder_stride(B)(chunk))  # lane t: t, t+B, ...
        lane_acc = [list(lane_fold(v)[0]) for v in lanes]           # map-local(reduce-seq)
        if b == 0:
            for t, h in enumerate(head):                            # scalar head: lane t mod B
                lane_acc[t % B][0] = scalar_step(lane_acc[t % B][0], h)
        if b == G - 1:
            for t, v in enumerate(tail0):                           # scalar tail: lane t mod B
                lane_acc[t % B][0] = scalar_step(lane_acc[t % B][0], v)
        lane_vals = [_pairwise(acc, add) for acc in lane_acc]      # iterate-log2(E)
        if s.seq:
            acc = lane_vals[0]                                      # reduce-seq over the lanes
            for v in lane_vals[1:]:
                acc = add(acc, v)
            partials.append(acc)
        else:
            partials.append(_block_tree(lane_vals, add))            # toLocal tree
    if G == 1:
        return partials[0]
    # final reduce-seq o join over the work-group partials, by F lanes (one
    # wavefront, or a work-group): lane t folds partials t, t+F, ... (from
    # 0), then the tree over the lanes
    F = s.final_lanes
    padded = partials + [zero] * (-(-G // F) * F - G)
    lane_vals = []
    for row in P.split(len(padded) // F)(P.reorder_stride(F)(padded)):
        acc = zero
        for p in row:
            acc = add(acc, p)
        lane_vals.append(acc)
    return _block_tree(lane_vals, add)


def render(shape: Shape) -> str:
    """The expression in the paper's notation (cf. Fig. 9)."""
    s = shape
    lanes_per_chunk = s.chunk // s.block
    waves = max(1, s.block // 64)
    e_log = int(math.log2(s.e))
    combine = ("reduce-seq(plus, 0)" if s.seq else
               "reduce-seq(plus, 0) o map-wave(iterate-6(join o map-local(reduce-seq(plus, 0)) o split-2))"
               " o split-64")
    wg = (f"join o toGlobal(map-local(map-seq(id))) o split-1\n"
          f"      o {combine}\n"
          f"      o join o toLocal(map-local(iterate-{e_log}(join o map(reduce-seq(plus, 0)) o split-2)"
          f" o asScalar o reduce-seq(vect-{s.e}(absAndPlus), vect-{s.e}(0))))\n"
          f"      o split-{lanes_per_chunk}" + ("" if s.runs else f" o reorder-stride-{s.block}"))
    text = (f"reduce-seq o join o map-workgroup(\n      {wg}\n    ) o split-{s.chunk} o asVector-{s.e}"
            f"   [{s.grid} work-groups x {waves} waves; head {s.head}, tail {s.tail} scalars]")
    return text


def evaluate_gemv_rows(rows, x, alpha, beta, y, shape: Shape, add, mul, fma, zero):
    """gemv's low-level expression for the given rows (Fig. 5,
    ``map(scal(alpha) o dot(x))`` over rows zipped with ``scal(beta, y)``):
    each row's dot is the dot expression of ``shape`` with one work-group
    (or one wavefront, block 64) per row -- lane t folds vectors t, t + B,
    ... of the row, the column tail enters lanes' component 0 -- then
    y_i' = fma(alpha, dot_i, beta * y_i), with beta * y_i taken as zero when
    beta is zero (BLAS: y is not read; reading 10) and alpha applied once to
    the finished dot (reading 8).  ``rows`` and ``y`` are parallel lists;
    ``shape`` must describe a single work-group (grid 1)."""
    if shape.grid != 1:
        raise ValueError("a row is reduced by one work-group")
    out = []
    for row, yi in zip(rows, y):
        d = evaluate_dot(list(row)[: shape.n], x, shape, add=add, fma=fma, zero=zero)
        by = zero if beta == 0 else mul(beta, yi)
        out.append(fma(alpha, d, by))
    return out
