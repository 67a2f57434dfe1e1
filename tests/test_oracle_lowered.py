"""The low-level expression of every asum launch configuration the tuner can
choose is a valid derivation of asum (Section 6.2's device-specific lowering,
generalised to the library's knobs): on integer inputs it equals the plain
sum exactly, for every knob point, size and misalignment."""
import random

import numpy as np
import pytest

from oracle import lowered as LW
from oracle import patterns as P
from paper_1502_02389_amd import tune


def ints(n, seed):
    r = random.Random(seed)
    return [r.randint(-9, 9) for _ in range(n)]


EXACT = dict(add=lambda a, b: a + b, absval=abs, zero=0)


def knob_points(storage):
    seen = set()
    for kn in tune.grid("asum", storage):
        key = (kn["block"], kn["vec_bytes"], kn["unroll"], kn["split"] or 1 << 15)
        if key not in seen:
            seen.add(key)
            yield key


@pytest.mark.parametrize("storage,eb", [("f32", 4), ("bf16", 2)])
def test_every_tuner_knob_point_is_a_valid_derivation(storage, eb):
    r = random.Random(1)
    for block, vb, unroll, split in knob_points(storage):
        n = r.choice([0, 1, 5, 1000, 4099, 50_000])
        mis = r.randrange(vb // eb)
        x = ints(n, block + vb + unroll + n)
        for il in (False, True):
            s = LW.launch_shape(n, eb, vb, block, unroll, split, misalign_elems=mis, interleave=il)
            assert LW.evaluate(x, s, **EXACT) == sum(abs(v) for v in x), (block, vb, unroll, split, n, mis, il)


@pytest.mark.parametrize("n", [0, 1, 3, 63, 64, 65, 4095, 70_001])
@pytest.mark.parametrize("mis", [0, 1, 3])
def test_shape_invariants(n, mis):
    for block, vb, unroll, split in [(64, 16, 1, 256), (256, 16, 8, 1 << 15), (1024, 8, 4, 1 << 17)]:
        s = LW.launch_shape(n, 4, vb, block, unroll, split, misalign_elems=mis)
        assert s.chunk % (block * unroll) == 0
        assert s.grid >= 1 and (s.grid - 1) * s.chunk < max(s.nvec, 1) <= s.grid * s.chunk or s.nvec == 0
        assert s.head + s.nvec * s.e + s.tail == n and 0 <= s.tail < s.e and s.head < s.e
        assert s.grid <= 8192


def test_grid_cap_raises_chunk():
    s = LW.launch_shape(64 * 4 * 9000, 4, 16, 64, 1, 256)
    assert s.grid <= 8192 and s.chunk > 64


def test_fig9b_parameters_give_the_fig9b_partition():
    # Fig. 9b: asVector-4 o split-2048, 256 lanes x 2 float4 per work-group
    s = LW.launch_shape(2048 * 6, 4, 16, 256, 2, 2048)
    assert s.chunk == 512 and s.grid == 6 and s.chunk // s.block == 2
    x = ints(2048 * 6, 7)
    assert LW.evaluate(x, s, **EXACT) == P.asum_lowlevel_gpu_vector(2048, 2, 4)(x)[0]


def test_render_names_the_patterns():
    text = LW.render(LW.launch_shape(1 << 20, 4, 16, 256, 8, 1 << 15))
    for piece in ("map-workgroup", "reorder-stride-256", "asVector-4", "iterate-6", "split-64", "toLocal",
                  "toGlobal", "vect-4(absAndPlus)", "split-8192"):
        assert piece in text, piece


def test_binary32_evaluation_distinguishes_trees():
    # a different work-group size is a different tree: same value to 1e-5,
    # but the binary32 bits differ on random data, so a bit-exact comparison
    # with the GPU pins the association, not just the sum
    import numpy as np

    f32 = dict(add=lambda a, b: np.float32(a) + np.float32(b), absval=lambda a: np.float32(abs(a)),
               zero=np.float32(0))
    differ = 0
    for seed in range(6):
        r = np.random.default_rng(seed)
        x = [np.float32(v) for v in r.uniform(-1, 1, 30_000).astype(np.float32)]
        a = LW.evaluate(x, LW.launch_shape(len(x), 4, 16, 64, 1, 256), **f32)
        b = LW.evaluate(x, LW.launch_shape(len(x), 4, 16, 128, 1, 512), **f32)
        assert abs(float(a) - float(b)) <= 1e-5 * float(a)
        differ += a != b
    assert differ >= 1


def test_interleaved_runs_are_a_permutation_of_the_chunks():
    # the same vectors reach the lanes, in a different grouping: with every
    # vector distinct, each work-group run holds steps b, b + G, ... in order
    s = LW.launch_shape(10_000, 4, 16, 64, 2, 1 << 10, interleave=True)
    assert s.step == 128 and s.grid == -(-2500 // s.chunk)
    x = list(range(1, 10_001))
    add = lambda a, b: a + b                                  # noqa: E731
    assert LW.evaluate(x, s, add=add, absval=lambda v: v, zero=0) == sum(x)
    f32 = dict(add=lambda a, b: np.float32(a) + np.float32(b), absval=lambda a: np.float32(abs(a)),
               zero=np.float32(0))
    rng = np.random.default_rng(3)
    vals = [np.float32(v) for v in rng.uniform(-1, 1, 100_000).astype(np.float32)]
    a = LW.evaluate(vals, LW.launch_shape(100_000, 4, 16, 256, 4, 1 << 14), **f32)
    b = LW.evaluate(vals, LW.launch_shape(100_000, 4, 16, 256, 4, 1 << 14, interleave=True), **f32)
    assert a != b          # a different association, visible in binary32


@pytest.mark.parametrize("storage,eb", [("f32", 4), ("bf16", 2)])
def test_every_tuner_knob_point_is_a_valid_dot_derivation(storage, eb):
    # the dot expression (zip of the vectorised operands, lane fold with
    # multAndPlus, the asum trees) equals the dot product exactly on integers
    r = random.Random(2)
    exact = dict(add=lambda a, b: a + b, fma=lambda a, b, c: a * b + c, zero=0)
    for block, vb, unroll, split in list(knob_points(storage))[::3]:
        n = r.choice([0, 1, 5, 1000, 4099, 50_000])
        mis = r.randrange(vb // eb)
        x, y = ints(n, block + n), ints(n, vb + unroll + n)
        want = sum(a * b for a, b in zip(x, y))
        for il in (False, True):
            s = LW.launch_shape(n, eb, vb, block, unroll, split, misalign_elems=mis, interleave=il)
            assert LW.evaluate_dot(x, y, s, **exact) == want, (block, vb, unroll, split, n, mis, il)


def test_dot_expression_is_the_asum_expression_on_abs_values():
    # with y = 1 and x >= 0, multAndPlus(acc, a, 1) = acc + a = absAndPlus:
    # the two expressions must coincide bit for bit in binary32 (same
    # partition, same trees), for both work-group partitions
    from tests import binary32 as F

    rng = np.random.default_rng(4)
    vals = [float(v) for v in rng.uniform(0, 1, 30_011).astype(np.float32)]
    ones = [1.0] * len(vals)
    for il in (False, True):
        s = LW.launch_shape(len(vals), 4, 16, 128, 2, 1 << 12, misalign_elems=1, interleave=il)
        d = LW.evaluate_dot(vals, ones, s, add=F.add, fma=F.fma, zero=0.0)
        a = LW.evaluate(vals, s, add=F.add, absval=abs, zero=0.0)
        assert d == a


def test_dot_expression_fma_is_one_rounding():
    # the lane step is a fused multiply-add.  a = 1 + 2^-23: a * a = 1 + 2^-22
    # + 2^-46 rounds to 1 + 2^-22.  Lane t folds x[t] * y[t] then x[t+64] *
    # y[t+64] (reorder-stride-64, one work-group, one element per vector);
    # with x = (a, ..., -a, ...), y = a: fma leaves the product's low part,
    # -2^-46 per lane, a rounded multiply then add leaves 0
    from tests import binary32 as F

    a = float(np.float32(1 + 2.0 ** -23))
    x = [a] * 64 + [-a] * 64
    y = [a] * 128
    s = LW.launch_shape(128, 4, 4, 64, 1, 128)
    assert s.grid == 1 and s.chunk == 128
    fused = LW.evaluate_dot(x, y, s, add=F.add, fma=F.fma, zero=0.0)
    unfused = LW.evaluate_dot(x, y, s, add=F.add, fma=lambda p, q, c: F.add(F.to_binary32(p * q), c), zero=0.0)
    assert fused == -64 * 2.0 ** -46
    assert unfused == 0.0


@pytest.mark.parametrize("n,vb,block,unroll", [(1000, 16, 64, 4), (1001, 4, 256, 2), (4099, 16, 512, 8), (3, 16, 64, 1),
                                               (0, 16, 64, 1)])
def test_gemv_rows_expression_exact_on_integers(n, vb, block, unroll):
    m = 7
    A = [ints(n, 10 * i + n) for i in range(m)]
    x = ints(n, 99)
    y = ints(m, 98)
    s = LW.launch_shape(n, 4, vb, block, unroll, max(n, 1))
    exact = dict(add=lambda a, b: a + b, mul=lambda a, b: a * b, fma=lambda a, b, c: a * b + c, zero=0)
    for alpha, beta in ((3, 2), (-1, 0), (0, 5)):
        got = LW.evaluate_gemv_rows(A, x, alpha, beta, y, s, **exact)
        want = [alpha * sum(a * b for a, b in zip(row, x)) + beta * yi for row, yi in zip(A, y)]
        assert got == want


def test_gemv_rows_beta_zero_does_not_read_y():
    from tests import binary32 as F

    s = LW.launch_shape(8, 4, 16, 64, 1, 32)
    got = LW.evaluate_gemv_rows([[1.0] * 8], [2.0] * 8, 0.5, 0.0, [float("nan")], s, add=F.add, mul=F.mul, fma=F.fma,
                                zero=0.0)
    assert got == [8.0]


# ---------------------------------------------------------------- lane forms

LANE_FORMS = {1: "reorder-stride lanes, folded in lane order", 2: "contiguous runs, tree",
              3: "contiguous runs, folded in lane order"}


@pytest.mark.parametrize("form", sorted(LANE_FORMS))
def test_lane_forms_are_valid_derivations(form):
    r = random.Random(form)
    blocks = (64, 256, 1024) if form == 2 else (1, 2, 32, 64, 256)
    for block in blocks:
        for _ in range(6):
            eb, vb = r.choice([(4, 4), (4, 16), (2, 2), (2, 8)])
            unroll = r.choice([1, 2, 4, 8])
            split = r.choice([256, 4096, 1 << 15])
            n = r.choice([0, 1, 7, 1000, 4099, 20_001])
            mis = r.randrange(vb // eb)
            x = ints(n, block + n + form)
            s = LW.launch_shape(n, eb, vb, block, unroll, split, misalign_elems=mis, lane_form=form)
            assert s.runs == bool(form & 2) and s.seq == bool(form & 1)
            assert s.final_lanes == min(64, block)
            assert LW.evaluate(x, s, **EXACT) == sum(abs(v) for v in x), (form, block, vb, unroll, split, n, mis)
            y = ints(n, n + 3)
            exact = dict(add=lambda a, b: a + b, fma=lambda a, b, c: a * b + c, zero=0)
            assert LW.evaluate_dot(x, y, s, **exact) == sum(a * b for a, b in zip(x, y))


def _order(n, block, form, unroll=1, chunk_elems=None):
    """The order in which one work-group's expression folds x[0..n) (scalar
    vectors): a tracing arithmetic whose sums are tuple concatenations."""
    s = LW.launch_shape(n, 4, 4, block, unroll, chunk_elems or n, lane_form=form)
    assert s.grid == 1
    trace = dict(add=lambda a, b: a + b, absval=lambda v: () if v == () else (v,), zero=())
    return LW.evaluate(list(range(1, n + 1)), s, **trace)


def test_lane_form_partitions():
    # contiguous runs folded in lane order read the chunk front to back
    assert _order(64, 4, 3) == tuple(range(1, 65))
    # reorder-stride lanes folded in lane order: lane t takes t, t + B, ...
    B = 4
    assert _order(64, B, 1) == tuple(v + 1 for t in range(B) for v in range(t, 64, B))
    # contiguous runs of 16 under the tree: 64 lanes -> runs of one vector
    # for 64 elements; with 256 elements each lane folds its own run of 4
    got = _order(256, 64, 2)
    runs = [tuple(range(4 * t + 1, 4 * t + 5)) for t in range(64)]
    assert sorted(got) == list(range(1, 257))
    pos = {v: i for i, v in enumerate(got)}
    for run in runs:        # each run stays together and in order inside the tree
        idx = [pos[v] for v in run]
        assert idx == list(range(idx[0], idx[0] + 4))


def test_single_lane_form_is_fig9c_on_integers():
    # one lane per work-group over contiguous runs (Fig. 9c): 32768 floats
    # per work-group as 8192 float4, one lane
    s = LW.launch_shape(32768 * 3, 4, 16, 1, 1, 32768, lane_form=3)
    assert s.grid == 3 and s.chunk == 8192 and s.final_lanes == 1
    x = ints(32768 * 3, 9)
    assert LW.evaluate(x, s, **EXACT) == P.asum_lowlevel_cpu(32768, 8192, 4)(x)[0] == sum(abs(v) for v in x)
