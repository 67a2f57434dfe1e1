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
from tests.gpu_util import banner, o_asum, rel

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
EB = {"f32": 4, "bf16": 2, "f16": 2}
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
