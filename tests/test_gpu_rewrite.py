"""The kernels of derived expressions, on the GPU.

For a sample of the knob points that the rewrite search derives for asum and
dot (each one the launch that executes one derived low-level expression), the
library's result on integer-valued inputs equals the exact sum, in binary32
and with 16-bit storage.
"""
import pytest
import torch

import paper_1502_02389_amd as L
import workloads as W
from paper_1502_02389_amd import rewrite as R
from tests.gpu_util import banner, o_asum, o_dot

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_derived_knob_points_integer_exact(gpu_device, storage):
    n = 1 << 20
    g = W.gen(81)
    x = W.integers(n, -8, 8, g, storage)
    y = W.integers(n, -4, 4, g, storage)
    ra, rd = o_asum(x), o_dot(x, y)[0]
    xd, yd = x.to(DEV), y.to(DEV)
    eb = 4 if storage == "f32" else 2
    for op in ("asum", "dot"):
        pts = R.derived_knob_points(op, n, elem_bytes=eb)
        assert len(pts) > 100
        for kn, d in pts[::17]:
            banner("derived", storage, op, kn)
            k = L.knobs(**kn)
            got = L.asum(xd, knobs=k).item() if op == "asum" else L.dot(xd, yd, knobs=k).item()
            assert got == (ra if op == "asum" else rd), (kn, str(d.expr))
