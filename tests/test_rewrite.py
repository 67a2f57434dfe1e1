"""The rewrite-driven derivations, checked with the oracle's pattern evaluator.

Every expression on every derivation path -- from the high-level program
through each rule application to the lowered form -- is evaluated on integer
data with oracle/patterns.py and must equal the sum exactly (the rules are
semantics-preserving, Section 4).  The launch knobs read from a derivation
must make the library's documented launch rules cut the input exactly as the
derived expression does.
"""
import random

import numpy as np
import pytest

from oracle import lowered
from oracle import patterns as P
from paper_1502_02389_amd import rewrite as R


ENV = {}   # alpha of scal, x of gemv (bound by the tests below)


def to_fn(e):
    """An executable closure for an expression, built from oracle patterns."""
    if isinstance(e, R.Fun):
        return {"add": P.add, "abs": P.abs_, "mult": lambda pr: P.mult(pr[0], pr[1]), "id": P.identity,
                "scale": lambda v: P.mult(ENV["alpha"], v)}[e.name]
    if isinstance(e, R.ZipX):
        return lambda row: P.zip_(row, ENV["x"])
    if isinstance(e, R.Fused):
        acc, elem = to_fn(e.acc), to_fn(e.elem)
        return lambda a, x: acc(a, elem(x))
    if isinstance(e, R.Comp):
        return P.compose(*[to_fn(p) for p in e.parts])
    if isinstance(e, R.Map):
        return P.map_(to_fn(e.f))
    if isinstance(e, (R.Reduce, R.PartRed)):
        z = P.Vec((e.z,) * e.f.n) if isinstance(e.f, R.Vect) else e.z
        return P.reduce_(to_fn(e.f), z)        # part-red: one valid partial reduction (to one value)
    if isinstance(e, R.Split):
        return P.split(e.n)
    if isinstance(e, R.Join):
        return P.join()
    if isinstance(e, R.Iterate):
        return P.iterate(e.k, to_fn(e.f))
    if isinstance(e, R.Reorder):
        return P.reorder_stride(e.stride) if e.stride else (lambda xs: list(reversed(xs)))
    if isinstance(e, (R.ToLocal, R.ToGlobal)):
        return to_fn(e.f)
    if isinstance(e, R.AsVector):
        return P.as_vector(e.n)
    if isinstance(e, R.AsScalar):
        return P.as_scalar()
    if isinstance(e, R.Vect):
        return P.vect(e.n, to_fn(e.f))
    raise TypeError(type(e))


def run(e, data):
    out = to_fn(e)(data)
    assert len(out) == 1
    return out[0]


N = 1 << 11
SPACE = dict(widths=(1, 2, 4), lanes=(1, 4, 8, 16), min_chunk=1 << 6, max_chunk=1 << 9)


@pytest.fixture(scope="module")
def data():
    rng = random.Random(5)
    x = [rng.randint(-8, 8) for _ in range(N)]
    y = [rng.randint(-8, 8) for _ in range(N)]
    return x, y


@pytest.mark.parametrize("op", ["asum", "dot"])
def test_every_step_of_every_derivation_is_exact(op, data):
    x, y = data
    inp = x if op == "asum" else list(zip(x, y))
    want = sum(abs(v) for v in x) if op == "asum" else sum(a * b for a, b in zip(x, y))
    ds = R.derive_reduction(op, N, **SPACE)
    assert len(ds) > 50
    forms = set()
    for d in ds:
        assert run(d.start, inp) == want
        for name, params, e in d.steps:
            assert run(e, inp) == want, (name, params, str(e))
        forms.add(str(d.expr))
    assert len(forms) == len(ds)          # distinct lowered expressions


def test_fig9b_shape_is_derived():
    # the AMD expression of Fig. 9b: 2048 floats per work-group as 512 float4,
    # split-2 per lane, 256 lanes behind reorder-stride, iterate-8
    d = R.derive_one("asum", R.Choice(2048, 4, 2, True, True))
    assert str(d.expr) == (
        "reduce-seq(plus, 0) o asScalar o join o map-workgroup("
        "iterate-8(join o map-local(reduce-seq(vect-4(plus), vect-4(0))) o split-2) o join o "
        "map-local(reduce-seq(vect-4(absAndPlus), vect-4(0))) o split-2 o reorder-stride-256) o "
        "split-512 o asVector-4")
    assert R.kernel_knobs(d) == {"block": 256, "vec_bytes": 16, "split": 2048, "interleave": R.INTERLEAVE_CHUNK}
    # Fig. 9c: one lane per work-group, no reorder -- the kernel of the
    # contiguous-runs form folded in lane order, with a block of one lane
    d = R.derive_one("asum", R.Choice(32768, 4, 8192, False, False))
    assert str(d.expr) == ("reduce-seq(plus, 0) o asScalar o join o map-workgroup(reduce-seq(vect-4(absAndPlus), "
                           "vect-4(0))) o split-8192 o asVector-4")
    assert R.kernel_knobs(d) == {"block": 1, "vec_bytes": 16, "split": 32768, "interleave": R.INTERLEAVE_CHUNK,
                                 "lane_form": R.LANES_SEQ | R.LANES_RUNS}
    # past 1024 lanes no kernel exists
    assert R.kernel_knobs(R.derive_one("asum", R.Choice(1 << 13, 1, 4, True, True))) is None
    assert R.kernel_knobs(R.derive_one("asum", R.Choice(1 << 14, 1, 8, True, True))) is None


def test_fig8_prefix_is_the_papers_derivation():
    d = R.derive_one("asum", R.Choice(1024, 1, 4, True, True))
    texts = [str(e) for _, _, e in d.steps[:5]]
    assert texts == [
        "reduce(plus, 0) o part-red(plus, 0) o map(abs)",
        "reduce(plus, 0) o join o map(part-red(plus, 0)) o split-1024 o map(abs)",
        "reduce(plus, 0) o join o map(part-red(plus, 0)) o split-1024 o join o map(map(abs)) o split-1024",
        "reduce(plus, 0) o join o map(part-red(plus, 0)) o map(map(abs)) o split-1024",
        "reduce(plus, 0) o join o map(part-red(plus, 0) o map(abs)) o split-1024",
    ]


@pytest.mark.parametrize("op", ["asum", "dot"])
def test_knobs_reproduce_the_derived_partition(op):
    n = 1 << 24
    pts = R.derived_knob_points(op, n)
    assert len(pts) > 100
    dealt = 0
    for k, d in pts:
        c = R._choice_of(d)
        e = k["vec_bytes"] // 4
        il = k["interleave"] == R.INTERLEAVE_STRIDE
        shape = lowered.launch_shape(n, 4, k["vec_bytes"], k["block"], k["unroll"], k["split"], interleave=il)
        assert shape.e == c.width == e
        assert shape.block == c.lanes
        assert shape.chunk == c.chunk // e              # vectors per work-group
        assert shape.grid == n // c.chunk
        assert shape.head == 0 and shape.tail == 0
        if il:                                          # the dealt steps and their groups
            dealt += 1
            assert shape.step == c.interleave and shape.grid == c.groups
    assert dealt > 50


def test_rules_check_their_preconditions():
    with pytest.raises(R.RuleError):
        R.split_join(R.Map(R.ABS, "seq"), 4)
    with pytest.raises(R.RuleError):
        R.reduction(R.Reduce(R.ADD, 0, True))
    with pytest.raises(R.RuleError):
        R.simplify_split_join(R.comp(R.Split(4), R.Join(), R.Map(R.Map(R.ABS)), R.Split(8)), 0)
    with pytest.raises(R.RuleError):
        R.fuse_maps(R.comp(R.Map(R.ABS, "local"), R.Map(R.ABS, "seq")), 0)
    with pytest.raises(R.RuleError):
        R.lower_reorder(R.Reorder(4), 8)
    with pytest.raises(R.RuleError):
        R.derive_one("asum", R.Choice(4096, 1, 3, True, True))   # 4096/3 lanes: not a power of two


def test_every_derived_reduction_gets_its_lane_form():
    # every derivation of the search has a launch: the default kernel for
    # reorder-stride lanes under the tree, the lane-form kernel for the
    # other three forms (down to one lane per work-group), each knob set
    # naming the partition the derivation chose
    for op in ("asum", "dot"):
        for n in (1 << 20, 1 << 24):
            ds = list(R.derive_reduction(op, n))
            assert len(ds) > 1000
            forms = set()
            for d in ds:
                c = R._choice_of(d)
                k = R.kernel_knobs(d)
                assert k is not None and 1 <= c.lanes <= 1024, str(d.expr)
                form = k.get("lane_form", 0)
                forms.add(form)
                assert form == (0 if c.tree else R.LANES_SEQ) | (0 if c.reorder else R.LANES_RUNS)
                assert k["block"] == c.lanes and k["split"] == c.chunk
                assert k["block"] >= 64 or form == R.LANES_SEQ | R.LANES_RUNS
            assert forms == {0, 1, 2, 3}


def test_scal_derivations_are_exact_and_match_the_launch_rules():
    rng = random.Random(6)
    x = [rng.randint(-9, 9) for _ in range(1 << 12)]
    ENV["alpha"] = 3
    want = [3 * v for v in x]
    for c in (64, 256, 1024, 4096):
        for w in (1, 2, 4):
            d = R.derive_scal(R.ScalChoice(c, w))
            for _, _, e in d.steps:
                assert to_fn(e)(x) == want, str(e)
    n = 1 << 24
    pts = R.scal_knob_points(n)
    assert len(pts) > 100
    for k, d in pts:
        e = k["vec_bytes"] // 4
        shape = lowered.launch_shape(n, 4, k["vec_bytes"], k["block"], k["unroll"], k["split"])
        assert shape.chunk == k["split"] // e and shape.grid == n // k["split"]


def test_fig2b_shape_is_derived():
    d = R.derive_scal(R.ScalChoice(1024, 4))
    assert str(d.expr) == "asScalar o join o map-workgroup(map-local(vect-4(mult(a)))) o split-256 o asVector-4"


def test_gemv_derivations_are_exact():
    rng = random.Random(7)
    m, n = 8, 64
    A = [[rng.randint(-8, 8) for _ in range(n)] for _ in range(m)]
    ENV["x"] = [rng.randint(-8, 8) for _ in range(n)]
    want = [sum(a * b for a, b in zip(row, ENV["x"])) for row in A]
    cs = list(R.gemv_choices(n, 4, wave_lanes=4, lanes=(2, 4, 8), rows_wg=(1, 2), rows_wave=(1, 2, 4),
                              waves=(1, 2), widths=(1, 2, 4)))
    assert {c.form for c in cs} == {"workgroup", "wave"} and len(cs) > 20
    def rows_of(out):   # each row's dot is a one-element array (reduce: T[] -> T[1])
        return [r[0] for r in out]

    for c in cs:
        d = R.derive_gemv(c)
        assert rows_of(to_fn(d.start)(A)) == want
        for name, params, e in d.steps:
            assert rows_of(to_fn(e)(A)) == want, (c, name, str(e))


def test_gemv_knobs_follow_the_lowering():
    pts = R.gemv_knob_points(8192)
    forms = {}
    for k, d in pts:
        levels = [p["level"] for nm, p, _ in d.steps if nm == "lower_map"]
        if k["row_split"] == 1:
            assert "wave" in levels and k["block"] % 64 == 0 and k["rows_per_wave"] in (1, 2, 4)
        else:
            assert "wave" not in levels and k["rows_per_wave"] in (1, 2) and k["vec_bytes"] in (4, 16)
            assert k["unroll"] in (2, 4, 8)
        forms[k["row_split"]] = forms.get(k["row_split"], 0) + 1
    assert forms[1] > 50 and forms[2] > 20
    # 16-bit storage: element or 16-byte loads for the work-group form
    for k, _ in R.gemv_knob_points(16384, 2):
        if k["row_split"] == 2:
            assert k["vec_bytes"] in (2, 16)
