"""Rewrite-driven derivation of the kernels' low-level expressions (the paper's Section 4 rules).

The paper expresses a program as a composition of algorithmic patterns and
derives device-specific low-level expressions by applying semantics-preserving
rewrite rules: the algorithmic rules of Fig. 3 (iterate decomposition 3a,
reorder commutativity 3b, split-join 3c, the reduction and partial-reduction
rules 3d, simplification 3e, fusion 3f) and the lowering rules of Fig. 4 (map
3 ways, reduce to reduce-seq, reorder to reorder-stride, local/global memory,
vectorisation).  Its prototype search over derivations is not described beyond
its existence (Section 6.3); this module is this library's own.

* Expressions are immutable trees (``Map``, ``Reduce``, ``PartRed``,
  ``Split``, ``Join``, ``Iterate``, ``Reorder``, ``Comp`` for composition, the
  low-level ``ToLocal``/``ToGlobal``/``AsVector``/``AsScalar``/``Vect``), and
  print in the paper's notation.
* Every rule is a function that checks its own precondition and returns the
  rewritten sub-expression; ``Derivation.apply`` rewrites at a located
  sub-term and records the step, so a derivation is a checked sequence of
  rule instances.
* ``derive_reduction`` searches the derivations of ``asum`` or ``dot`` along
  the paper's route (Fig. 8, then Fig. 9's shape): at every rule with a
  parameter or an alternative -- the work-group chunk, the vector width, the
  per-lane split, whether lanes read through ``reorder``, whether lane
  partials are combined by a tree (``iterate`` of pairwise ``part-red``) or by
  one sequential ``reduce``, whether the work-groups' input is reordered so
  that they take steps dealt round-robin -- it branches, and every branch
  ends in a fully lowered expression.
* ``kernel_knobs`` recognises the expressions this library's streaming
  reduction kernel implements (work-group chunk C, B lanes reading through
  reorder-stride-B, vectors of E elements, a tree over the lanes) and returns
  the launch knobs that execute exactly that partition of the input; other
  expressions (one lane per work-group, lanes on contiguous runs, a
  sequential combine of the lanes) have no kernel here and give ``None``.
* ``derive_scal`` lowers ``map(mult(a))`` along Fig. 2b (vectorise, split
  into work-group chunks, map-workgroup / map-local), and ``derive_gemv``
  splits gemv's map over rows into groups of R rows, lowered to work-groups
  or, through a ``map-wave`` level for the 64-lane wavefront, to wavefronts,
  each row's dot being the reduction derivation; ``scal_knob_points`` and
  ``gemv_knob_points`` map them to launches the same way.

The autotuner times the kernels of the derived expressions
(``tune.py --space derived``); the tests evaluate every step of every
derivation with the oracle's pattern evaluator.  Nothing here evaluates an
expression.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field
from typing import Callable, Iterator, Optional, Tuple

# lift_knobs.interleave values (the work-group partition of asum / dot)
INTERLEAVE_STRIDE, INTERLEAVE_CHUNK = 1, 2

# ---------------------------------------------------------------- expressions


class Node:
    """Base of all pattern expressions (immutable; children are Nodes)."""

    def children(self) -> Tuple["Node", ...]:
        return ()

    def with_children(self, kids: Tuple["Node", ...]) -> "Node":
        return self


@dataclass(frozen=True)
class Fun(Node):
    """A user function: abs, mult (of a pair), add, id."""

    name: str

    def __str__(self):
        return {"add": "plus", "scale": "mult(a)"}.get(self.name, self.name)


@dataclass(frozen=True)
class Fused(Node):
    """lambda (acc, a): acc_f(acc, elem_f(a)) -- the fused reduction operator
    of rule 3f (reduce-seq(f) o map-seq(g))."""

    acc: Node
    elem: Node

    def children(self):
        return (self.acc, self.elem)

    def with_children(self, kids):
        return Fused(*kids)

    def __str__(self):
        names = {("add", "abs"): "absAndPlus", ("add", "mult"): "multAndPlus"}
        key = (getattr(self.acc, "name", ""), getattr(self.elem, "name", ""))
        return names.get(key, f"(\\acc a. {self.acc}(acc, {self.elem}(a)))")


@dataclass(frozen=True)
class Comp(Node):
    """f1 o f2 o ... o fk: parts[-1] is applied first."""

    parts: Tuple[Node, ...]

    def children(self):
        return self.parts

    def with_children(self, kids):
        return comp(*kids)

    def __str__(self):
        return " o ".join(str(p) for p in self.parts)


LEVELS = ("", "workgroup", "wave", "local", "seq", "global")  # "wave": a 64-lane wavefront (CDNA)


@dataclass(frozen=True)
class Map(Node):
    """map(f); after lowering (Fig. 4a) map-workgroup, map-local or map-seq,
    and map-wave for the level between the two that a CDNA wavefront forms."""

    f: Node
    level: str = ""

    def children(self):
        return (self.f,)

    def with_children(self, kids):
        return Map(kids[0], self.level)

    def __str__(self):
        return f"map{'-' + self.level if self.level else ''}({self.f})"


@dataclass(frozen=True)
class Reduce(Node):
    """reduce(f, z); reduce-seq after the lowering of Fig. 4b."""

    f: Node
    z: object = 0
    seq: bool = False

    def children(self):
        return (self.f,)

    def with_children(self, kids):
        return Reduce(kids[0], self.z, self.seq)

    def __str__(self):
        return f"reduce{'-seq' if self.seq else ''}({self.f}, {_zero(self.z, self.f)})"


@dataclass(frozen=True)
class PartRed(Node):
    """part-red(f, z): a partial reduction (Fig. 3d)."""

    f: Node
    z: object = 0

    def children(self):
        return (self.f,)

    def with_children(self, kids):
        return PartRed(kids[0], self.z)

    def __str__(self):
        return f"part-red({self.f}, {_zero(self.z, self.f)})"


@dataclass(frozen=True)
class Split(Node):
    n: int

    def __str__(self):
        return f"split-{self.n}"


@dataclass(frozen=True)
class Join(Node):
    def __str__(self):
        return "join"


@dataclass(frozen=True)
class Iterate(Node):
    k: int
    f: Node

    def children(self):
        return (self.f,)

    def with_children(self, kids):
        return Iterate(self.k, kids[0])

    def __str__(self):
        return f"iterate-{self.k}({self.f})"


@dataclass(frozen=True)
class Reorder(Node):
    """reorder (any permutation); reorder-stride-s once lowered (Fig. 4c)."""

    stride: int = 0

    def __str__(self):
        return f"reorder-stride-{self.stride}" if self.stride else "reorder"


@dataclass(frozen=True)
class ToLocal(Node):
    f: Node

    def children(self):
        return (self.f,)

    def with_children(self, kids):
        return ToLocal(kids[0])

    def __str__(self):
        return f"toLocal({self.f})"


@dataclass(frozen=True)
class ToGlobal(Node):
    f: Node

    def children(self):
        return (self.f,)

    def with_children(self, kids):
        return ToGlobal(kids[0])

    def __str__(self):
        return f"toGlobal({self.f})"


@dataclass(frozen=True)
class AsVector(Node):
    n: int

    def __str__(self):
        return f"asVector-{self.n}"


@dataclass(frozen=True)
class AsScalar(Node):
    def __str__(self):
        return "asScalar"


@dataclass(frozen=True)
class Vect(Node):
    """vect-n(f): f applied componentwise to n-wide vectors."""

    n: int
    f: Node

    def children(self):
        return (self.f,)

    def with_children(self, kids):
        return Vect(self.n, kids[0])

    def __str__(self):
        return f"vect-{self.n}({self.f})"


def _zero(z, f=None):
    return f"vect-{f.n}({z})" if isinstance(f, Vect) else str(z)


def comp(*parts: Node) -> Node:
    """Composition, flattened; a single part is returned as itself."""
    flat = []
    for p in parts:
        flat.extend(p.parts if isinstance(p, Comp) else (p,))
    if not flat:
        return Fun("id")
    return flat[0] if len(flat) == 1 else Comp(tuple(flat))


ADD, ABS, MULT, ID = Fun("add"), Fun("abs"), Fun("mult"), Fun("id")


def high_level(op: str) -> Node:
    """asum = reduce(+, 0) o map(abs); dot = reduce(+, 0) o map(mult) (on zip(x, y))."""
    if op == "asum":
        return comp(Reduce(ADD, 0), Map(ABS))
    if op == "dot":
        return comp(Reduce(ADD, 0), Map(MULT))
    raise ValueError(f"no high-level expression for {op!r}")


# ---------------------------------------------------------------- addressing

Path = Tuple[int, ...]


def subterm(e: Node, path: Path) -> Node:
    for i in path:
        e = e.children()[i]
    return e


def replace_at(e: Node, path: Path, new: Node) -> Node:
    if not path:
        return new
    kids = list(e.children())
    kids[path[0]] = replace_at(kids[path[0]], path[1:], new)
    return e.with_children(tuple(kids))


def walk(e: Node, path: Path = ()) -> Iterator[Tuple[Path, Node]]:
    """Pre-order traversal."""
    yield path, e
    for i, c in enumerate(e.children()):
        yield from walk(c, path + (i,))


def find(e: Node, pred: Callable[[Node], bool], nth: int = 0) -> Path:
    hits = [p for p, n in walk(e) if pred(n)]
    if len(hits) <= nth:
        raise RuleError("no sub-term matches")
    return hits[nth]


class RuleError(ValueError):
    """A rule was applied where its precondition does not hold."""


# ---------------------------------------------------------------- rules (Fig. 3)
# Each rule takes the sub-term it rewrites (for rules on a composition: the
# Comp and the index of the first part involved) and returns its replacement.


def split_join(e: Node, n: int) -> Node:
    """3c: map(f) -> join o map(map(f)) o split-n."""
    if not isinstance(e, Map) or e.level:
        raise RuleError("split-join applies to a high-level map")
    return comp(Join(), Map(Map(e.f)), Split(n))


def reduction(e: Node) -> Node:
    """3d: reduce(f, z) -> reduce(f, z) o part-red(f, z)."""
    if not isinstance(e, Reduce) or e.seq:
        raise RuleError("the reduction rule applies to a high-level reduce")
    return comp(e, PartRed(e.f, e.z))


def part_red_to_reduce(e: Node) -> Node:
    """3d: part-red(f, z) -> reduce(f, z)."""
    if not isinstance(e, PartRed):
        raise RuleError("expects part-red")
    return Reduce(e.f, e.z)


def part_red_reorder(e: Node) -> Node:
    """3d: part-red(f, z) -> part-red(f, z) o reorder."""
    if not isinstance(e, PartRed):
        raise RuleError("expects part-red")
    return comp(e, Reorder())


def part_red_split(e: Node, n: int) -> Node:
    """3d: part-red(f, z) -> join o map(part-red(f, z)) o split-n."""
    if not isinstance(e, PartRed):
        raise RuleError("expects part-red")
    return comp(Join(), Map(e), Split(n))


def part_red_iterate(e: Node, k: int) -> Node:
    """3d: part-red(f, z) -> iterate-k(part-red(f, z))."""
    if not isinstance(e, PartRed) or k < 1:
        raise RuleError("expects part-red and k >= 1")
    return Iterate(k, e)


def iterate_peel(e: Node) -> Node:
    """3a: iterate-(k+1)(f) -> iterate-k(f) o f (iterate-1(f) is f)."""
    if not isinstance(e, Iterate) or e.k < 1:
        raise RuleError("expects iterate with k >= 1")
    if e.k == 1:
        return e.f
    return comp(Iterate(e.k - 1, e.f) if e.k > 2 else e.f, e.f)


def _comp_parts(e: Node, i: int, count: int):
    if not isinstance(e, Comp) or not 0 <= i or i + count > len(e.parts):
        raise RuleError("expects a composition with enough parts")
    return list(e.parts)


def reorder_commute(e: Node, i: int) -> Node:
    """3b: reorder o map(f) -> map(f) o reorder (parts i, i+1 of a composition)."""
    parts = _comp_parts(e, i, 2)
    a, b = parts[i], parts[i + 1]
    if isinstance(a, Reorder) and isinstance(b, Map) and not b.level:
        parts[i], parts[i + 1] = b, a
        return comp(*parts)
    raise RuleError("expects reorder o map(f)")


def simplify_split_join(e: Node, i: int) -> Node:
    """3e: split-n o join o map(map(f)) o split-n -> map(map(f)) o split-n
    (the join rebuilt from chunks of n is cut again at n)."""
    parts = _comp_parts(e, i, 4)
    s1, j, m, s2 = parts[i:i + 4]
    if (isinstance(s1, Split) and isinstance(j, Join) and isinstance(m, Map) and isinstance(m.f, Map)
            and isinstance(s2, Split) and s1.n == s2.n):
        return comp(*(parts[:i] + [m, s2] + parts[i + 4:]))
    raise RuleError("expects split-n o join o map(map f) o split-n")


def fuse_maps(e: Node, i: int) -> Node:
    """3f: map(f) o map(g) -> map(f o g) (same level)."""
    parts = _comp_parts(e, i, 2)
    a, b = parts[i], parts[i + 1]
    if isinstance(a, Map) and isinstance(b, Map) and a.level == b.level:
        return comp(*(parts[:i] + [Map(comp(a.f, b.f), a.level)] + parts[i + 2:]))
    raise RuleError("expects map(f) o map(g)")


def fuse_reduce_seq(e: Node, i: int) -> Node:
    """3f: reduce-seq(f, z) o map-seq(g) -> reduce-seq(lambda acc a: f(acc, g(a)), z)."""
    parts = _comp_parts(e, i, 2)
    a, b = parts[i], parts[i + 1]
    if isinstance(a, Reduce) and a.seq and isinstance(b, Map) and b.level == "seq":
        if isinstance(a.f, Vect) and isinstance(b.f, Vect) and a.f.n == b.f.n:
            fused = Vect(a.f.n, Fused(a.f.f, b.f.f))      # vect-n(absAndPlus)
        else:
            fused = Fused(a.f, b.f)
        return comp(*(parts[:i] + [Reduce(fused, a.z, True)] + parts[i + 2:]))
    raise RuleError("expects reduce-seq(f) o map-seq(g)")


# ---------------------------------------------------------------- rules (Fig. 4)


def lower_map(e: Node, level: str) -> Node:
    """4a: map(f) -> map-workgroup(f) / map-local(f) / map-seq(f)."""
    if not isinstance(e, Map) or e.level or level not in LEVELS[1:]:
        raise RuleError("expects a high-level map and a level")
    return Map(e.f, level)


def lower_reduce(e: Node) -> Node:
    """4b: reduce(f, z) -> reduce-seq(f, z)."""
    if not isinstance(e, Reduce) or e.seq:
        raise RuleError("expects a high-level reduce")
    return Reduce(e.f, e.z, True)


def lower_reorder(e: Node, stride: int) -> Node:
    """4c: reorder -> reorder-stride-s."""
    if not isinstance(e, Reorder) or e.stride:
        raise RuleError("expects an unlowered reorder")
    return Reorder(stride)


def lower_reorder_blocks(e: Node, stride: int, block: int) -> Node:
    """4c on blocks: reorder -> join o reorder-stride-s o split-b, the
    permutation that deals blocks of b elements round-robin to s groups."""
    if not isinstance(e, Reorder) or e.stride:
        raise RuleError("expects an unlowered reorder")
    return comp(Join(), Reorder(stride), Split(block))


def to_local(e: Node) -> Node:
    """4d: f -> toLocal(f) (results kept in local memory)."""
    return ToLocal(e)


def to_global(e: Node) -> Node:
    """4d: f -> toGlobal(f) (results written to global memory)."""
    return ToGlobal(e)


def vectorize(e: Node, n: int) -> Node:
    """4e: map(f) -> asScalar o map(vect-n(f)) o asVector-n."""
    if not isinstance(e, Map):
        raise RuleError("expects a map")
    return comp(AsScalar(), Map(Vect(n, e.f), e.level), AsVector(n))


# ---------------------------------------------------------------- derivations


@dataclass
class Derivation:
    """A start expression and the checked rule steps applied to it."""

    start: Node
    steps: list = field(default_factory=list)   # (rule name, params, expression after)

    @property
    def expr(self) -> Node:
        return self.steps[-1][2] if self.steps else self.start

    def apply(self, rule: Callable, where: Path, **params) -> "Derivation":
        """Rewrite the sub-term at `where` with `rule(sub-term, **params)`."""
        e = self.expr
        new = replace_at(e, where, rule(subterm(e, where), **params))
        return Derivation(self.start, self.steps + [(rule.__name__, dict(params), new)])

    def apply_first(self, rule: Callable, pred: Callable[[Node], bool], nth: int = 0, **params):
        return self.apply(rule, find(self.expr, pred, nth), **params)

    def text(self) -> str:
        lines = [f"   {self.start}"]
        for name, params, e in self.steps:
            p = ", ".join(f"{k}={v}" for k, v in params.items())
            lines.append(f"={name}({p})\n   {e}")
        return "\n".join(lines)


def _is(cls, **attrs):
    return lambda n: isinstance(n, cls) and all(getattr(n, k) == v for k, v in attrs.items())


def _comp_with(pred_at: Callable[[Tuple[Node, ...]], Optional[int]]):
    """Locate a Comp and an index inside it where pred_at(parts) is not None."""
    def locate(e: Node):
        for path, n in walk(e):
            if isinstance(n, Comp):
                i = pred_at(n.parts)
                if i is not None:
                    return path, i
        raise RuleError("no composition matches")
    return locate


def _index(parts, test, width):
    for i in range(len(parts) - width + 1):
        if test(parts[i:i + width]):
            return i
    return None


def _on_comp(d: Derivation, rule, test, width) -> Derivation:
    path, i = _comp_with(lambda parts: _index(parts, test, width))(d.expr)
    return d.apply(rule, path, i=i)


@dataclass(frozen=True)
class Choice:
    """The branch a derivation took at each rule with an alternative."""

    chunk: int        # elements per work-group (split of the input)
    width: int        # vector width E (1 = no vectorisation)
    per_lane: int     # vectors per lane (split inside a work-group)
    reorder: bool     # lanes read through reorder (-stride) or contiguous runs
    tree: bool        # lane partials combined by iterate(part-red) or one reduce
    interleave: int = 0   # > 0: work-groups take steps of `interleave` vectors
    #                       round-robin (a reorder of the input by blocks)
    groups: int = 0       # the number of work-groups the steps are dealt to

    @property
    def lanes(self) -> int:
        return self.chunk // (self.width * self.per_lane)


def _log2(v: int) -> int:
    k = v.bit_length() - 1
    if v <= 0 or (1 << k) != v:
        raise RuleError(f"{v} is not a power of two")
    return k


def vector_partial(e: Node, i: int) -> Node:
    """3d on vectors: reduce(f, z) o asScalar -> reduce(f, z) o asScalar o
    part-red(vect-n(f), z): the n component streams are partially reduced
    separately (f associative and commutative, z its identity)."""
    parts = _comp_parts(e, i, 3)
    r, s, m = parts[i:i + 3]
    if isinstance(r, Reduce) and not r.seq and isinstance(s, AsScalar) and isinstance(m, Map) \
            and isinstance(m.f, Vect):
        return comp(*(parts[:i + 2] + [PartRed(Vect(m.f.n, r.f), r.z)] + parts[i + 2:]))
    raise RuleError("expects reduce o asScalar o map(vect-n(f))")


def _element_map(n: Node) -> bool:
    """map(abs) / map(mult), possibly vectorised: the per-element function."""
    if not isinstance(n, Map) or n.level:
        return False
    f = n.f.f if isinstance(n.f, Vect) else n.f
    return f in (ABS, MULT)


def _split_join_fuse(d: Derivation, n: int, lane: bool) -> Derivation:
    """Move the element map under the split made by part-red's split rule:
    split-join (3c), simplify (3e) and fuse (3f) -- Fig. 8 steps 2 to 5."""
    d = d.apply_first(split_join, _element_map, n=n)
    d = _on_comp(d, simplify_split_join, lambda p: isinstance(p[0], Split) and isinstance(p[1], Join), 4)
    return _on_comp(d, fuse_maps, lambda p: isinstance(p[0], Map) and isinstance(p[1], Map)
                    and (not lane or _head_is(p[0].f, PartRed)), 2)


def _head_is(f: Node, cls) -> bool:
    return isinstance(f.parts[0] if isinstance(f, Comp) else f, cls)


def derive_one(op: str, c: Choice) -> Derivation:
    """One derivation of `op` along the paper's route, with the branches `c`.

    Vectorise the element map (4e) when E > 1; split the reduction into
    work-group partial reductions and fuse the element map into them
    (Fig. 8); inside a work-group, a partial reduction to one value: one
    sequential reduce when there is a single lane (Fig. 9c's shape), else
    lanes on runs of the chunk (behind reorder or not) whose partials a
    tree (iterate of pairwise part-red, Fig. 9a/9b) or one reduce combines;
    then the lowering of Fig. 4.
    """
    d = Derivation(high_level(op))
    vecs = c.chunk // c.width
    lanes = c.lanes
    if c.width > 1:
        d = d.apply_first(vectorize, _element_map, n=c.width)              # asScalar o map(vect f) o asVector
        d = _on_comp(d, vector_partial, lambda p: isinstance(p[0], Reduce) and isinstance(p[1], AsScalar), 3)
    else:
        d = d.apply_first(reduction, _is(Reduce, seq=False))               # reduce o part-red
    if c.interleave:                                                       # work-groups on dealt steps
        d = d.apply_first(part_red_reorder, _is(PartRed))
        d = _on_comp(d, reorder_commute, lambda p: isinstance(p[0], Reorder) and isinstance(p[1], Map), 2)
    d = d.apply_first(part_red_split, _is(PartRed), n=vecs)                # join o map(part-red) o split
    d = _split_join_fuse(d, vecs, lane=False)                              # map(part-red o map(f)) o split
    if lanes == 1:
        return _lower(d.apply_first(part_red_to_reduce, _is(PartRed)), c)
    if c.tree:
        k = _log2(lanes)
        d = d.apply_first(part_red_iterate, _is(PartRed), k=k + 1)        # iterate-(k+1)(part-red)
        d = d.apply_first(iterate_peel, _is(Iterate, k=k + 1))            # iterate-k(part-red) o part-red
    else:
        d = d.apply_first(part_red_iterate, _is(PartRed), k=2)
        d = d.apply_first(iterate_peel, _is(Iterate, k=2))                # part-red o part-red
    if c.reorder:                                                          # lanes: the second part-red
        d = d.apply_first(part_red_reorder, _is(PartRed), nth=1)
        d = _on_comp(d, reorder_commute, lambda p: isinstance(p[0], Reorder) and isinstance(p[1], Map), 2)
    d = d.apply_first(part_red_split, _is(PartRed), nth=1, n=c.per_lane)
    d = _split_join_fuse(d, c.per_lane, lane=True)
    d = d.apply_first(part_red_to_reduce, _is(PartRed), nth=1)            # each lane reduces its run
    if c.tree:                                                             # pairwise tree over the lanes
        d = d.apply_first(part_red_split, _is(PartRed), n=2)
    d = d.apply_first(part_red_to_reduce, _is(PartRed))
    return _lower(d, c)


def _lower(d: Derivation, c: Choice) -> Derivation:
    """Fig. 4: the work-group map, lane and tree maps, element maps, reduces,
    reorder; then fuse each lane's reduce-seq with its map-seq (3f)."""
    d = d.apply_first(lower_map, lambda n: isinstance(n, Map) and not n.level and not _element_map(n),
                      level="workgroup")
    while any(isinstance(n, Map) and not n.level and not _element_map(n) for _, n in walk(d.expr)):
        d = d.apply_first(lower_map, lambda n: isinstance(n, Map) and not n.level and not _element_map(n),
                          level="local")
    while any(_element_map(n) for _, n in walk(d.expr)):
        d = d.apply_first(lower_map, _element_map, level="seq")
    while any(isinstance(n, Reduce) and not n.seq for _, n in walk(d.expr)):
        d = d.apply_first(lower_reduce, _is(Reduce, seq=False))
    in_wg = [p for p, n in walk(d.expr) if isinstance(n, Reorder) and not n.stride and len(p) > 1]
    if in_wg:                                        # lanes: reorder-stride-B inside the work-group
        d = d.apply(lower_reorder, in_wg[0], stride=c.lanes)
    if c.interleave:                                 # work-groups: steps dealt round-robin
        d = d.apply_first(lower_reorder_blocks, _is(Reorder, stride=0), stride=c.groups, block=c.interleave)
    while True:
        try:
            d = _on_comp(d, fuse_reduce_seq, lambda p: isinstance(p[0], Reduce) and p[0].seq
                         and isinstance(p[1], Map) and p[1].level == "seq", 2)
        except RuleError:
            return d


def choices(n: int, widths=(1, 2, 4), lanes=(1, 64, 128, 256, 512, 1024), min_chunk: int = 1 << 11,
            max_chunk: int = 1 << 20, interleave: bool = True) -> Iterator[Choice]:
    """The branches explored for an input of n elements (powers of two that
    divide n): work-group chunk, vector width, lanes, reorder, tree, and
    whether work-groups take one chunk or steps dealt round-robin."""
    c = min_chunk
    while c <= min(max_chunk, n):
        if n % c == 0:
            for w, b in itertools.product(widths, lanes):
                if c % (w * b) == 0:
                    forms = [(False, False)] if b == 1 else itertools.product((True, False), (True, False))
                    for reorder, tree in forms:
                        yield Choice(c, w, c // (w * b), reorder, tree)
                    if b > 1 and interleave:
                        p = c // (w * b)
                        for u in (1, 2, 4, 8):
                            if p % u == 0 and n // c > 1:
                                yield Choice(c, w, p, True, True, interleave=b * u, groups=n // c)
        c *= 2


def derive_reduction(op: str, n: int, **space) -> list:
    """Every derivation of asum or dot for n elements over the search space."""
    return [derive_one(op, c) for c in choices(n, **space)]


# ---------------------------------------------------------------- kernels


LANES_SEQ, LANES_RUNS = 1, 2      # lift_lane_form bits (include/lift.h)


def kernel_knobs(d: Derivation, elem_bytes: int = 4) -> Optional[dict]:
    """Launch knobs of the streaming reduction kernel that executes the
    partition of this derivation, or None when no kernel implements the
    expression (more than 1024 lanes, vectors wider than 16 bytes, a tree
    over fewer than 64 lanes, the other lane forms with work-groups dealt
    steps round-robin).

    The kernel's work-group b takes vectors [b C/E, (b+1) C/E); its lane t
    folds vectors t, t + B, ... of the chunk (reorder-stride-B), or with the
    lane form's RUNS bit the t-th run of C/(E B) vectors (a plain split), and
    the B lane partials meet in a tree, or with its SEQ bit in one reduce-seq
    in lane order -- the expression's partition.
    """
    c = _choice_of(d)
    if c is None or c.lanes > 1024 or (c.tree and c.lanes < 64):
        return None
    form = (0 if c.tree else LANES_SEQ) | (0 if c.reorder else LANES_RUNS)
    if form and c.interleave:
        return None
    vb = c.width * elem_bytes
    if vb > 16 or vb < min(4, elem_bytes):
        return None
    k = {"block": c.lanes, "vec_bytes": vb, "split": c.chunk, "interleave": INTERLEAVE_CHUNK}
    if form:
        k["lane_form"] = form
    if c.interleave:                                 # the dealt step is block x unroll
        k.update(interleave=INTERLEAVE_STRIDE, unroll=c.interleave // c.lanes)
    return k


def _choice_of(d: Derivation) -> Optional[Choice]:
    """Read the branch back from the derivation's rule parameters."""
    splits = [p["n"] for name, p, _ in d.steps if name == "part_red_split"]
    widths = [p["n"] for name, p, _ in d.steps if name == "vectorize"]
    strides = [p["stride"] for name, p, _ in d.steps if name == "lower_reorder"]
    iters = [p["k"] for name, p, _ in d.steps if name == "part_red_iterate"]
    if not splits:
        return None
    width = widths[0] if widths else 1
    vecs = splits[0]
    per_lane = splits[1] if len(splits) > 1 else vecs
    tree = bool(iters) and len(splits) > 2 and splits[2] == 2
    blocks = [(p["stride"], p["block"]) for name, p, _ in d.steps if name == "lower_reorder_blocks"]
    il, groups = (blocks[0][1], blocks[0][0]) if blocks else (0, 0)
    c = Choice(vecs * width, width, per_lane, bool(strides), tree, il, groups)
    if strides and strides[0] != c.lanes:
        return None
    if tree and iters[0] != _log2(c.lanes) + 1:
        return None
    return c


def derived_knob_points(op: str, n: int, elem_bytes: int = 4, unrolls=(1, 2, 4, 8), max_workgroups: int = 8192,
                        **space) -> list:
    """(knobs, derivation) pairs to time: each implementable derivation with
    every loads-in-flight count U that divides its per-lane run (so the
    kernel's chunk is exactly the derived one), and at most max_workgroups
    work-groups (the kernel's grid cap would otherwise merge chunks)."""
    if "widths" not in space:
        space["widths"] = tuple(w for w in (1, 2, 4, 8) if 4 <= w * elem_bytes <= 16 or
                                (elem_bytes == 2 and w == 1))
    out, seen = [], set()
    for d in derive_reduction(op, n, **space):
        k = kernel_knobs(d, elem_bytes)
        if k is None or n // k["split"] > max_workgroups:
            continue
        per_lane = k["split"] // (k["vec_bytes"] // elem_bytes) // k["block"]
        if "unroll" in k:                      # the derivation fixes the step
            key = tuple(sorted(k.items()))
            if key not in seen:
                seen.add(key)
                out.append((k, d))
            continue
        for u in unrolls:
            if per_lane % u == 0:
                kk = dict(k, unroll=u)
                key = tuple(sorted(kk.items()))
                if key not in seen:
                    seen.add(key)
                    out.append((kk, d))
    return out


# ---------------------------------------------------------------- scal and gemv


@dataclass(frozen=True)
class ZipX(Node):
    """zip(row, x): pairs a row of A with the vector x (gemv's dot(x))."""

    def __str__(self):
        return "zip(x)"


SCALE = Fun("scale")   # mult(a): the element function of scal


def high_level_map(op: str) -> Node:
    """scal = map(mult(a)); gemv (its matrix-vector part) =
    map(reduce(+, 0) o map(mult) o zip(x)) over the rows of A -- Fig. 5; the
    scaling by alpha and the zip with beta * y are fused into the store."""
    if op == "scal":
        return Map(SCALE)
    if op == "gemv":
        return Map(comp(Reduce(ADD, 0), Map(MULT), ZipX()))
    raise ValueError(f"no high-level expression for {op!r}")


@dataclass(frozen=True)
class ScalChoice:
    chunk: int   # elements per work-group
    width: int   # vector width E


def derive_scal(c: ScalChoice) -> Derivation:
    """scal along Fig. 2b: vectorise (4e), split into work-group chunks (3c),
    map-workgroup over chunks and map-local over the vectors of a chunk (4a)."""
    d = Derivation(high_level_map("scal"))
    if c.width > 1:
        d = d.apply_first(vectorize, _is(Map, level=""), n=c.width)
    d = d.apply_first(split_join, lambda n: isinstance(n, Map) and not n.level, n=c.chunk // c.width)
    d = d.apply_first(lower_map, _is(Map, level=""), level="workgroup")
    return d.apply_first(lower_map, _is(Map, level=""), level="local")


@dataclass(frozen=True)
class GemvChoice:
    """A lowering of gemv's map over rows: one work-group per R rows, its B
    lanes splitting each row ("workgroup"), or one wavefront per R rows with
    W wavefronts per work-group ("wave"); rows read as vectors of E elements,
    per_lane vectors per lane."""

    form: str
    rows: int
    lanes: int      # B for the work-group form, the wavefront width for the wave form
    waves: int      # W (wave form; 1 otherwise)
    width: int
    per_lane: int


def _row_dot(d: Derivation, lanes: int, per_lane: int, width: int) -> Derivation:
    """One row's dot(x) reduced by `lanes` lanes behind reorder and a tree --
    the work-group body of the reduction derivation applied to a whole row."""
    elem = lambda n: _element_map(n)                                        # noqa: E731
    if width > 1:
        d = d.apply_first(vectorize, elem, n=width)
        d = _on_comp(d, vector_partial, lambda p: isinstance(p[0], Reduce) and isinstance(p[1], AsScalar), 3)
    else:
        d = d.apply_first(reduction, _is(Reduce, seq=False))
    k = _log2(lanes)
    d = d.apply_first(part_red_iterate, _is(PartRed), k=k + 1)
    d = d.apply_first(iterate_peel, _is(Iterate, k=k + 1))
    d = d.apply_first(part_red_reorder, _is(PartRed), nth=1)
    d = _on_comp(d, reorder_commute, lambda p: isinstance(p[0], Reorder) and isinstance(p[1], Map), 2)
    d = d.apply_first(part_red_split, _is(PartRed), nth=1, n=per_lane)
    d = _split_join_fuse(d, per_lane, lane=True)
    d = d.apply_first(part_red_to_reduce, _is(PartRed), nth=1)
    d = d.apply_first(part_red_split, _is(PartRed), n=2)
    return d.apply_first(part_red_to_reduce, _is(PartRed))


def derive_gemv(c: GemvChoice) -> Derivation:
    """gemv: split the row map into groups of R rows (3c) -- and, in the wave
    form, those into groups of W (3c) -- derive each row's dot with its lanes,
    then lower: row groups to map-workgroup (wave form: map-workgroup over W
    wavefronts, map-wave), the R rows of a group to map-seq, lanes and tree to
    map-local, elements to map-seq (4a-4c), fusing each lane's reduce-seq (3f)."""
    if c.form not in ("workgroup", "wave"):
        raise RuleError("gemv forms: workgroup, wave")
    d = Derivation(high_level_map("gemv"))
    row_map = lambda n: isinstance(n, Map) and not n.level and not _element_map(n)  # noqa: E731
    d = d.apply_first(split_join, row_map, n=c.rows)
    if c.form == "wave":
        d = d.apply_first(split_join, row_map, n=c.waves)
    d = _row_dot(d, c.lanes, c.per_lane, c.width)
    levels = ["workgroup"] + (["wave"] if c.form == "wave" else []) + ["seq"]
    for lvl in levels:
        d = d.apply_first(lower_map, row_map, level=lvl)
    while any(row_map(n) for _, n in walk(d.expr)):
        d = d.apply_first(lower_map, row_map, level="local")
    while any(_element_map(n) for _, n in walk(d.expr)):
        d = d.apply_first(lower_map, _element_map, level="seq")
    while any(isinstance(n, Reduce) and not n.seq for _, n in walk(d.expr)):
        d = d.apply_first(lower_reduce, _is(Reduce, seq=False))
    d = d.apply_first(lower_reorder, _is(Reorder, stride=0), stride=c.lanes)
    while True:
        try:
            d = _on_comp(d, fuse_reduce_seq, lambda p: isinstance(p[0], Reduce) and p[0].seq
                         and isinstance(p[1], Map) and p[1].level == "seq", 2)
        except RuleError:
            return d


def gemv_choices(n: int, elem_bytes: int = 4, wave_lanes: int = 64, lanes=(64, 128, 256, 512, 1024),
                 rows_wg=(1, 2), rows_wave=(1, 2, 4), waves=(1, 2, 4, 8, 16), widths=None) -> Iterator[GemvChoice]:
    """Branches for rows of n elements: both forms, rows per group, lanes or
    wavefronts, vector widths E with E lanes x per-lane runs covering the row."""
    if widths is None:
        widths = tuple(w for w in (1, 2, 4, 8) if w * elem_bytes <= 16)
    for w in widths:
        for b in lanes:
            if n % (b * w) == 0:
                for r in rows_wg:
                    yield GemvChoice("workgroup", r, b, 1, w, n // (b * w))
        if n % (wave_lanes * w) == 0:
            for r, nw in itertools.product(rows_wave, waves):
                yield GemvChoice("wave", r, wave_lanes, nw, w, n // (wave_lanes * w))


def _params(d: Derivation, name: str, key: str) -> list:
    return [p[key] for nm, p, _ in d.steps if nm == name]


def scal_knob_points(n: int, blocks=(64, 128, 256, 512, 1024), unrolls=(1, 2, 4, 8), min_chunk: int = 1 << 11,
                     max_chunk: int = 1 << 20) -> list:
    """(knobs, derivation) for scal: every derived chunk and width, with each
    work-group size B and loads in flight U that make whole steps of the chunk
    (map-local leaves the work-group size to the launch)."""
    out = []
    c = min_chunk
    while c <= min(max_chunk, n):
        for w in (1, 2, 4):
            d = derive_scal(ScalChoice(c, w))
            vecs = c // w
            for b, u in itertools.product(blocks, unrolls):
                if vecs % (b * u) == 0:
                    out.append(({"block": b, "vec_bytes": 4 * w, "unroll": u, "split": c}, d))
        c *= 2
    return out


def gemv_kernel_knobs(d: Derivation, elem_bytes: int = 4) -> Optional[dict]:
    """Launch knobs of the gemv kernel that executes this derivation's
    lowering (without loads in flight, a launch parameter), or None."""
    levels = [p["level"] for nm, p, _ in d.steps if nm == "lower_map"]
    rows = _params(d, "split_join", "n")[0]
    width = (_params(d, "vectorize", "n") or [1])[0]
    lanes = _params(d, "lower_reorder", "stride")[0]
    vb = width * elem_bytes
    if "wave" in levels:
        if lanes != 64 or rows not in (1, 2, 4) or vb > 16:
            return None
        waves = _params(d, "split_join", "n")[1]
        return {"row_split": 1, "rows_per_wave": rows, "block": 64 * waves, "vec_bytes": vb}
    if rows not in (1, 2) or (vb != 16 and vb != elem_bytes) or not 64 <= lanes <= 1024:
        return None
    return {"row_split": 2, "rows_per_wave": rows, "block": lanes, "vec_bytes": vb}


def gemv_knob_points(n: int, elem_bytes: int = 4, **space) -> list:
    """(knobs, derivation) for gemv rows of n elements, crossed with the
    loads in flight each kernel form supports."""
    out = []
    for c in gemv_choices(n, elem_bytes, **space):
        d = derive_gemv(c)
        k = gemv_kernel_knobs(d, elem_bytes)
        if k is None:
            continue
        for u in ((2, 4, 8) if k["row_split"] == 2 else (1, 2, 4, 8)):
            out.append((dict(k, unroll=u), d))
    return out
