"""Bit-exact parity of asum with its low-level expression in binary32.

For an explicit knob point the launch (chunking, head / tail, grid) follows
the documented rules, and the kernel's reduction tree is the expression built
by oracle/lowered.py (lane reduce-seq over vect-E accumulators, pairwise
iterate over the vector components and over the 64 lanes of a wave, fold of
the wave totals, the same tree over work-group partials).  Evaluated with
IEEE binary32 additions on the same stored values, that expression must
reproduce the GPU's result bit for bit on random (non-integer) data -- a
check of the association itself, beyond the 1e-5 bound against the binary64
oracle."""
import numpy as np
import pytest
import torch

import paper_1502_02389_amd as L
import workloads as W
from oracle import lowered as LW
from tests.gpu_util import banner, o_asum, o_dot, rel

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
EB = {"f32": 4, "bf16": 2, "f16": 2}
BATCH_LDS_X = 16320   # floats of LDS for copies of x in the batched form's gemv tiles (include/lift.h)
F32 = dict(add=lambda a, b: np.float32(a) + np.float32(b), absval=lambda a: np.float32(abs(a)),
           zero=np.float32(0))

CASES = [
    # n, offset (elements), storage, block, vec_bytes, unroll, split[, interleave]
    (70_001, 0, "f32", 256, 16, 8, 1 << 15, 1),
    (1 << 20, 0, "f32", 256, 16, 4, 1 << 16, 1),
    (300_007, 2, "f32", 128, 4, 2, 1 << 12, 1),
    (100_000, 1, "bf16", 256, 16, 4, 1 << 15, 1),
    (70_001, 0, "f32", 256, 16, 8, 1 << 15),
    (70_001, 1, "f32", 64, 16, 1, 256),
    (200_003, 3, "f32", 1024, 8, 4, 1 << 17),
    (5, 0, "f32", 256, 16, 8, 1 << 15),
    (1 << 20, 0, "f32", 256, 16, 8, 1 << 16),
    (300_007, 2, "f32", 128, 4, 2, 1 << 12),
    (100_000, 1, "bf16", 256, 16, 4, 1 << 15),
    (100_000, 3, "f16", 512, 8, 2, 1 << 14),
    (65_536 * 3 + 5, 0, "bf16", 64, 4, 8, 1 << 11),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[2]}-n{c[0]}-o{c[1]}-b{c[3]}-v{c[4]}-u{c[5]}-s{c[6]}"
                                             f"{'-il' if len(c) > 7 else ''}" for c in CASES])
def test_asum_matches_lowered_expression_bitwise(gpu_device, case):
    n, off, storage, block, vb, unroll, split = case[:7]
    il = len(case) > 7 and case[7] == 1
    x = W.uniform(n, W.gen(800 + n % 1000 + off), storage)
    buf = torch.empty(n + off, dtype=x.dtype, device=DEV)
    xd = buf[off:]
    xd.copy_(x.to(DEV))
    assert xd.data_ptr() % vb == (off * EB[storage]) % vb
    banner("lowered asum", case)
    k = L.knobs(block=block, vec_bytes=vb, unroll=unroll, split=split,
                interleave=L.LIFT_INTERLEAVE_STRIDE if il else L.LIFT_INTERLEAVE_CHUNK)
    g = L.asum(xd, knobs=k).item()
    shape = LW.launch_shape(n, EB[storage], vb, block, unroll, split, misalign_elems=off % (vb // EB[storage]),
                            interleave=il)
    vals = [np.float32(v) for v in x.float().numpy()]
    pred = LW.evaluate(vals, shape, **F32)
    assert np.float32(g).view(np.uint32) == np.float32(pred).view(np.uint32), (g, float(pred), LW.render(shape))
    assert rel(g, o_asum(x)) <= 1e-5


# dot: n, x offset, y offset (elements), storage, block, vec_bytes, unroll, split, interleave
DOT_CASES = [
    (70_001, 0, 0, "f32", 256, 16, 4, 1 << 15, True),
    (70_001, 0, 0, "f32", 256, 16, 4, 1 << 15, False),
    (1 << 20, 0, 0, "f32", 256, 16, 4, 1 << 16, True),
    (300_007, 2, 2, "f32", 128, 8, 2, 1 << 12, True),
    (200_003, 3, 3, "f32", 1024, 16, 1, 1 << 17, False),
    (100_000, 1, 1, "bf16", 256, 16, 4, 1 << 15, True),
    (100_000, 5, 5, "f16", 512, 8, 2, 1 << 14, False),
    (50_003, 0, 1, "f32", 256, 16, 4, 1 << 13, True),       # phases differ: element loads
    (7, 0, 0, "f32", 256, 16, 8, 1 << 15, True),
]


@pytest.mark.parametrize("case", DOT_CASES, ids=[f"{c[3]}-n{c[0]}-o{c[1]}.{c[2]}-b{c[4]}-v{c[5]}-u{c[6]}-s{c[7]}"
                                                 f"{'-il' if c[8] else ''}" for c in DOT_CASES])
def test_dot_matches_lowered_expression_bitwise(gpu_device, case):
    from tests import binary32 as F32B

    n, ox, oy, storage, block, vb, unroll, split, il = case
    g = W.gen(900 + n % 1000 + ox + 7 * oy)
    x = W.uniform(n, g, storage)
    y = W.uniform(n, g, storage)
    bx = torch.empty(n + ox, dtype=x.dtype, device=DEV)
    by = torch.empty(n + oy, dtype=y.dtype, device=DEV)
    xd, yd = bx[ox:], by[oy:]
    xd.copy_(x.to(DEV))
    yd.copy_(y.to(DEV))
    banner("lowered dot", case)
    k = L.knobs(block=block, vec_bytes=vb, unroll=unroll, split=split,
                interleave=L.LIFT_INTERLEAVE_STRIDE if il else L.LIFT_INTERLEAVE_CHUNK)
    got = L.dot(xd, yd, knobs=k).item()
    eb = EB[storage]
    same_phase = (ox * eb) % vb == (oy * eb) % vb
    vbytes = vb if same_phase else eb                         # different phases: element loads
    shape = LW.launch_shape(n, eb, vbytes, block, unroll, split, misalign_elems=(ox * eb % vb) // eb if same_phase
                            else 0, interleave=il)
    xs = [float(v) for v in x.float().numpy()]
    ys = [float(v) for v in y.float().numpy()]
    pred = LW.evaluate_dot(xs, ys, shape, add=F32B.add, fma=F32B.fma, zero=0.0)
    assert np.float32(got).view(np.uint32) == np.float32(pred).view(np.uint32), (got, pred, LW.render(shape))
    r, mass = o_dot(x, y)
    assert abs(got - r) <= 1e-5 * mass


# lane forms: form, n, x offset, y offset (elements), storage, block, vec_bytes, unroll, split
LANE_CASES = [
    (1, 70_001, 0, 0, "f32", 256, 16, 4, 1 << 15),
    (1, 30_011, 3, 3, "bf16", 16, 8, 2, 1 << 11),
    (2, 70_001, 1, 1, "f32", 256, 16, 2, 1 << 15),
    (2, 100_000, 0, 0, "bf16", 64, 8, 8, 1 << 13),
    (3, 70_001, 2, 2, "f32", 128, 8, 4, 1 << 13),
    (3, 20_003, 0, 0, "f32", 1, 16, 1, 1 << 12),            # one lane per work-group (Fig. 9c's shape)
    (3, 30_001, 1, 1, "bf16", 4, 2, 8, 1 << 10),
    (3, 40_000, 0, 1, "f32", 32, 16, 2, 1 << 12),           # phases differ: element loads
]


@pytest.mark.parametrize("case", LANE_CASES, ids=[f"form{c[0]}-{c[4]}-n{c[1]}-o{c[2]}.{c[3]}-b{c[5]}-v{c[6]}-u{c[7]}"
                                                  for c in LANE_CASES])
def test_lane_forms_match_lowered_expressions_bitwise(gpu_device, case):
    """asum and dot in the other lane forms (reorder-stride lanes folded in
    lane order, contiguous runs under the tree or folded in lane order, down
    to one lane per work-group): every result bit for bit against the
    expression of that form, and within the plain bars of the oracle."""
    from tests import binary32 as F32B

    form, n, ox, oy, storage, block, vb, unroll, split = case
    g = W.gen(950 + form + n % 1000)
    x = W.uniform(n, g, storage)
    y = W.uniform(n, g, storage)
    bx = torch.empty(n + ox, dtype=x.dtype, device=DEV)
    by = torch.empty(n + oy, dtype=y.dtype, device=DEV)
    xd, yd = bx[ox:], by[oy:]
    xd.copy_(x.to(DEV))
    yd.copy_(y.to(DEV))
    banner("lowered lane form", case)
    k = L.knobs(block=block, vec_bytes=vb, unroll=unroll, split=split, lane_form=form)
    eb = EB[storage]
    xs = [float(v) for v in x.float().numpy()]
    ys = [float(v) for v in y.float().numpy()]
    got = L.asum(xd, knobs=k).item()
    shape = LW.launch_shape(n, eb, vb, block, unroll, split, misalign_elems=(ox * eb % vb) // eb, lane_form=form)
    pred = LW.evaluate([np.float32(v) for v in xs], shape, **F32)
    assert np.float32(got).view(np.uint32) == np.float32(pred).view(np.uint32), ("asum", got, float(pred))
    assert rel(got, o_asum(x)) <= 1e-5
    got = L.dot(xd, yd, knobs=k).item()
    same_phase = (ox * eb) % vb == (oy * eb) % vb
    vbytes = vb if same_phase else eb
    shape = LW.launch_shape(n, eb, vbytes, block, unroll, split,
                            misalign_elems=(ox * eb % vb) // eb if same_phase else 0, lane_form=form)
    pred = LW.evaluate_dot(xs, ys, shape, add=F32B.add, fma=F32B.fma, zero=0.0)
    assert np.float32(got).view(np.uint32) == np.float32(pred).view(np.uint32), ("dot", got, pred)
    r, mass = o_dot(x, y)
    assert abs(got - r) <= 1e-5 * mass


_STEP = {}


def _step_run():
    """The bench step's asum and dot (n = 2^24, seed 1) through the plain
    entry points with the library's default launch; results and inputs."""
    if not _STEP:
        x, y, _ = W.stream_vectors()
        n = x.numel()
        xd, yd = x.to(DEV), y.to(DEV)
        ws = L.workspace(DEV)
        res = torch.zeros(2, dtype=torch.float32, device=DEV)
        s = torch.cuda.current_stream().cuda_stream
        banner("step kernels 2^24 default launch")
        assert L.lift_asum(n, xd.data_ptr(), res[0:].data_ptr(), ws.data_ptr(), ws.numel(), s) == 0
        assert L.lift_dot(n, xd.data_ptr(), yd.data_ptr(), res[1:].data_ptr(), ws.data_ptr(), ws.numel(), s) == 0
        _STEP.update(res=res.cpu().numpy(), xs=[float(v) for v in x.numpy()], ys=[float(v) for v in y.numpy()],
                     cus=torch.cuda.get_device_properties(0).multi_processor_count)
    return _STEP


def _plain_call_shape(op, n, cus):
    """Launch shape of a plain asum / dot call (no knobs) on this device: the
    knobs lift_default_knobs reports (the tuned entry, if any), with the
    built-in default for every zero field -- 256 lanes, 16-byte vectors, 8
    loads in flight (dot: 4), one work-group per compute unit, contiguous
    chunks for asum and interleaved steps for dot."""
    _, k = L.lift_default_knobs(op, L.LIFT_F32, 0, n)
    block = k["block"] or 256
    vb = k["vec_bytes"] or 16
    unroll = k["unroll"] or (4 if op == "dot" else 8)
    interleave = {0: op == "dot", 1: True, 2: False}[k["interleave"]]
    e = vb // 4
    split = k["split"] or -(-(n // e) // (cus * (k["wg_per_cu"] or 1))) * e
    return LW.launch_shape(n, 4, vb, block, unroll, split, interleave=interleave)


def test_step_asum_2p24_default_launch_matches_its_expression(gpu_device):
    """asum of the bench step through the plain entry point (the library's
    own launch on this device): bit for bit."""
    from tests import binary32 as F32B

    st = _step_run()
    n = len(st["xs"])
    sa = _plain_call_shape("asum", n, st["cus"])
    pa = LW.evaluate(st["xs"], sa, add=F32B.add, absval=abs, zero=0.0)
    assert np.float32(st["res"][0]).view(np.uint32) == np.float32(pa).view(np.uint32), \
        (float(st["res"][0]), pa, LW.render(sa))


def test_step_dot_2p24_default_launch_matches_its_expression(gpu_device):
    """dot of the bench step (the roofline kernel) through the plain entry
    point: bit for bit."""
    from tests import binary32 as F32B

    st = _step_run()
    n = len(st["xs"])
    sd = _plain_call_shape("dot", n, st["cus"])
    pd = LW.evaluate_dot(st["xs"], st["ys"], sd, add=F32B.add, fma=F32B.fma, zero=0.0)
    assert np.float32(st["res"][1]).view(np.uint32) == np.float32(pd).view(np.uint32), \
        (float(st["res"][1]), pd, LW.render(sd))


# gemv: m, n, lda, storage, knobs (row_split, block, rows_per_wave, unroll, vec_bytes) -> the
# row expression's lanes (64 for a wavefront per row, the work-group size otherwise)
GEMV_CASES = [
    (97, 1001, 1008, "f32", dict(row_split=1, rows_per_wave=1, unroll=4, vec_bytes=16), 64),
    (97, 1001, 1008, "f32", dict(row_split=1, rows_per_wave=2, unroll=2, vec_bytes=16), 64),
    (61, 5000, 5000, "f32", dict(row_split=2, block=256, rows_per_wave=1, unroll=4, vec_bytes=16), 256),
    (61, 3000, 3004, "f32", dict(row_split=2, block=256, rows_per_wave=2, unroll=4, vec_bytes=16), 256),
    (50, 1001, 1001, "f32", dict(row_split=2, block=128, rows_per_wave=1, unroll=8, vec_bytes=16), 128),
    (64, 9000, 9000, "bf16", dict(row_split=2, block=256, rows_per_wave=1, unroll=8, vec_bytes=16), 256),
    (33, 777, 784, "f16", dict(row_split=1, rows_per_wave=4, unroll=2, vec_bytes=8), 64),
]


def _gemv_model_rows(A, x, y, alpha, beta, rows, lanes, unroll, vec_bytes, eb, misalign_elems=0):
    from tests import binary32 as F32B

    n = x.numel()
    shape = LW.launch_shape(n, eb, vec_bytes, lanes, unroll, max(n, 1),    # one chunk: the whole row
                            misalign_elems=misalign_elems)
    xs = [float(v) for v in x.numpy()]
    Af = A.float().numpy()
    return LW.evaluate_gemv_rows([[float(v) for v in Af[i, :n]] for i in rows], xs, float(alpha), float(beta),
                                 [float(y[i]) for i in rows], shape, add=F32B.add, mul=F32B.mul, fma=F32B.fma,
                                 zero=0.0)


@pytest.mark.parametrize("case", GEMV_CASES, ids=[f"{c[3]}-{c[0]}x{c[1]}-lda{c[2]}-rs{c[4]['row_split']}-"
                                                  f"r{c[4]['rows_per_wave']}-u{c[4]['unroll']}" for c in GEMV_CASES])
def test_gemv_matches_lowered_rows_bitwise(gpu_device, case):
    m, n, lda, storage, kn, lanes = case
    g = W.gen(950 + m + n)
    A = W.normal((m, lda), g, storage)
    x = W.normal(n, g)
    y = W.normal(m, g)
    alpha, beta = 0.75, -1.25
    banner("lowered gemv", case)
    yd = y.to(DEV)
    L.gemv(alpha, A.to(DEV), x.to(DEV), beta, yd, lda=lda, knobs=L.knobs(**kn))
    eb = EB[storage]
    aligned = (lda * eb) % kn["vec_bytes"] == 0
    pred = _gemv_model_rows(A, x, y, alpha, beta, range(m), lanes, kn["unroll"],
                            kn["vec_bytes"] if aligned else eb, eb)
    got = yd.cpu().numpy()
    bad = [i for i in range(m) if np.float32(got[i]).view(np.uint32) != np.float32(pred[i]).view(np.uint32)]
    assert not bad, (bad[:5], [(float(got[i]), pred[i]) for i in bad[:3]])


@pytest.mark.parametrize("size,sample", [(4096, 128), (8192, 48), (16384, 16)])
def test_gemv_default_launch_sampled_rows_bitwise(gpu_device, size, sample):
    """gemv fp32 at the bench's sizes through the plain entry point (no
    knobs: the library's tuned entry for the size on this device, else its
    default -- a work-group per row sized to it, x in registers, 8 loads in
    flight): the call equals, bit for bit, the same call with the reported
    knobs passed explicitly, and sampled rows equal the row expression of
    that launch bit for bit."""
    A, x, y, alpha, beta = W.gemv_square(size)
    banner("lowered gemv default", size)
    yd = y.to(DEV)
    Ad, xd = A.to(DEV), x.to(DEV)
    s = torch.cuda.current_stream().cuda_stream
    assert L.lift_gemv(size, size, alpha, Ad.data_ptr(), size, xd.data_ptr(), beta, yd.data_ptr(), s) == 0
    got = yd.cpu().numpy()
    src, k = L.lift_default_knobs("gemv", L.LIFT_F32, 0, size * size, row_length=size)
    if src:
        ye = y.to(DEV)
        assert L.lift_gemv_ex(size, size, alpha, L.LIFT_F32, Ad.data_ptr(), size, xd.data_ptr(), beta,
                              ye.data_ptr(), 0, L.knobs(**k), s) == 0
        assert np.array_equal(ye.cpu().numpy().view(np.uint32), got.view(np.uint32))
    unroll = k["unroll"] or 8
    vb = k["vec_bytes"] or 16
    row_split = k["row_split"] or (2 if size // 4 <= 512 * unroll else 1)
    if row_split == 1:
        lanes = 64                                  # a wavefront per row group; each row's dot over 64 lanes
    else:
        if vb != 16:
            vb = 4                                  # the work-group form reads 16 bytes or one element
        lanes = k["block"]
        if not lanes:                               # the documented choice: smallest work-group whose
            lanes = 64                              # one step covers the row
            while lanes * unroll < size // (vb // 4) and lanes < 512:
                lanes *= 2
    rows = sorted(np.random.default_rng(size).choice(size, sample, replace=False).tolist())
    # a work-group above 256 threads may be lowered to the instance's launch
    # bound (512 or 256, lift.h): the rows must be the row expression of one
    # of the sizes the launch can have used
    candidates = [lanes] + [b for b in (512, 256) if b < lanes] if row_split == 2 and lanes > 256 else [lanes]
    misses = {}
    for cand in candidates:
        pred = _gemv_model_rows(A, x, y, alpha, beta, rows, cand, unroll, vb, 4)
        misses[cand] = [i for i, p in zip(rows, pred)
                        if np.float32(got[i]).view(np.uint32) != np.float32(p).view(np.uint32)]
        if not misses[cand]:
            break
    assert any(not m for m in misses.values()), {c: m[:5] for c, m in misses.items()}


BATCH_KNOBS = [dict(block=256, vec_bytes=16, unroll=4, split=65536, wg_per_cu=2),
               dict(block=64, vec_bytes=4, unroll=1, split=256, wg_per_cu=1),
               dict(block=512, vec_bytes=16, unroll=8, split=1 << 15, wg_per_cu=4),
               dict(block=256, vec_bytes=8, unroll=2, split=4096, wg_per_cu=8)]


@pytest.mark.parametrize("storage", ["f32", "bf16"])
@pytest.mark.parametrize("kn", BATCH_KNOBS, ids=[str(i) for i in range(len(BATCH_KNOBS))])
def test_batch_matches_lowered_expressions_bitwise(gpu_device, storage, kn):
    """The batched form runs each reduction as the per-call expression with
    the batch's tiles for work-group chunks (split rounded up to whole steps,
    partials folded by the last tile's work-group like the per-call combine)
    and each gemv row as the row expression of a wavefront (64 lanes, U
    loads in flight); where the rows do not all start on a vector boundary
    (or x is not aligned), each row from its own start, with a scalar head
    up to its first boundary (vectors of at most 8 bytes, rows filling a
    step, x copies fitting in LDS), else element loads.
    Every result bit for bit."""
    from tests import binary32 as F32B
    from tests.test_gpu_batch import build, small_spec

    cpu, problems = build(small_spec(seed=48, n_red=100, n_gemv=10), storage=storage, seed=49)
    banner("lowered batch", storage, kn)
    b = L.Batch(problems, knobs=L.knobs(**kn))
    b.run()
    torch.cuda.synchronize()
    eb = EB[storage]
    B, U, vb, split = kn["block"], kn["unroll"], kn["vec_bytes"], kn["split"]
    E = vb // eb
    for i, (item, pr) in enumerate(zip(cpu, problems)):
        if item[0] == "gemv":
            alpha, A, x, beta, y, n = item[1]
            xd, yd = pr[3], pr[5]
            lda = A.shape[1]
            ad = pr[2].data_ptr()
            vec = n > 0 and ad % vb == 0 and (lda * eb) % vb == 0 and xd.data_ptr() % min(E * 4, 16) == 0
            heads = not vec and E > 1 and vb <= 8 and n >= 64 * E and E * (-(-n // 4) * 4) <= BATCH_LDS_X
            if heads:
                # each row from its own start: a head up to its first vector boundary
                pred = [None] * A.shape[0]
                by_mis = {}
                for r in range(A.shape[0]):
                    by_mis.setdefault(((ad + r * lda * eb) % vb) // eb, []).append(r)
                for mis, rows in by_mis.items():
                    for r, v in zip(rows, _gemv_model_rows(A, x[:n].contiguous(), y, alpha, beta, rows, 64, U,
                                                           vb, eb, misalign_elems=mis)):
                        pred[r] = v
            else:
                pred = _gemv_model_rows(A, x[:n].contiguous(), y, alpha, beta, range(A.shape[0]), 64, U,
                                        vb if vec else eb, eb)
            got = yd.cpu().numpy()
            bad = [r for r in range(A.shape[0])
                   if np.float32(got[r]).view(np.uint32) != np.float32(pred[r]).view(np.uint32)]
            assert not bad, (i, "gemv", bad[:4])
        else:
            kind, x, y = item
            xd = pr[1]
            n = x.numel()
            mis = (xd.data_ptr() % vb) // eb
            same = kind == "asum" or pr[2].data_ptr() % vb == xd.data_ptr() % vb
            shape = LW.launch_shape(n, eb, vb if same else eb, B, U, split, misalign_elems=mis if same else 0,
                                    max_workgroups=1 << 30, final_lanes=B)
            xs = [float(v) for v in x.float().numpy()]
            if kind == "asum":
                pred = LW.evaluate(xs, shape, add=F32B.add, absval=abs, zero=0.0)
            else:
                ys = [float(v) for v in y.float().numpy()]
                pred = LW.evaluate_dot(xs, ys, shape, add=F32B.add, fma=F32B.fma, zero=0.0)
            got = b.results[i].item()
            assert np.float32(got).view(np.uint32) == np.float32(pred).view(np.uint32), (i, kind, n, got, pred)
    b.close()


@pytest.mark.parametrize("storage", ["bf16", "f16", "f32"])
def test_batch_gemv_row_heads_bitwise(gpu_device, storage):
    """gemv rows that start inside a vector (row pitch not a multiple of the
    8-byte vector, or x misaligned), long enough for the head form (from one
    vector per lane up; row counts that are not a multiple of the 2E rows a
    pair block spans, and a problem of 3 rows): every head length occurs, and
    each row matches the row expression of 64 lanes with its own misaligned
    start, bit for bit."""
    from tests.test_gpu_batch import _dev_copy

    kn = dict(block=512, vec_bytes=8, unroll=4, split=262144, wg_per_cu=8)
    eb, vb, U = EB[storage], 8, 4
    E = vb // eb
    g = W.gen(77)
    cases = []          # (A on the CPU, x, y, device A, device x, device y, alpha, beta)
    for j, (m, n) in enumerate([(37, 64 * U * E + 1), (29, 64 * U * E + 3), (23, 64 * U * E + 5), (19, 2047),
                                (31, 64 * E + 3), (13, 64 * E * 2 + 1), (3, 64 * E + 1), (17, 64 * U * E)]):
        A = W.normal((m, n), g, storage)
        x = W.normal(n, g)
        y = W.normal(m, g)
        xd = _dev_copy(x, 1 if j == 7 else 0)     # the last: aligned rows, misaligned x
        cases.append((A, x, y, A.to(DEV), xd, y.to(DEV), 1.25, 0.5 if j % 2 == 0 else 0.0))
    problems = [("gemv", a, Ad, xd, b, yd) for (_, _, _, Ad, xd, yd, a, b) in cases]
    banner("batch gemv row heads", storage)
    b = L.Batch(problems, knobs=L.knobs(**kn))
    b.run()
    torch.cuda.synchronize()
    for (A, x, y, Ad, xd, yd, alpha, beta) in cases:
        m, n = A.shape
        ad = Ad.data_ptr()
        assert (n * eb) % vb != 0 or xd.data_ptr() % 16 != 0      # every case takes the head form
        got = yd.cpu().numpy()
        by_mis = {}
        for r in range(m):
            by_mis.setdefault(((ad + r * n * eb) % vb) // eb, []).append(r)
        if storage != "f32":
            assert len(by_mis) == min(E, m) or n % E == 0    # all head lengths occur when the pitch is odd
        for mis, rows in by_mis.items():
            pred = _gemv_model_rows(A, x, y, alpha, beta, rows, 64, U, vb, eb, misalign_elems=mis)
            bad = [r for r, p in zip(rows, pred) if np.float32(got[r]).view(np.uint32) != np.float32(p).view(np.uint32)]
            assert not bad, (storage, m, n, mis, bad[:4])
    b.close()
