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


def test_derived_scal_and_gemv_points(gpu_device):
    from tests.gpu_util import o_gemv
    import numpy as np

    g = W.gen(82)
    n = 1 << 20
    x = W.uniform(n, g)
    xd = x.to(DEV)
    want = (x.double() * 2.5).float()
    for kn, d in R.scal_knob_points(n)[::13]:
        banner("derived scal", kn)
        assert torch.equal(L.scal(2.5, xd, knobs=L.knobs(**kn)).cpu(), want), (kn, str(d.expr))
    for storage, eb in (("f32", 4), ("bf16", 2)):
        m, cols = 300, 2048
        A = W.integers((m, cols), -8, 8, g, storage)
        xv = W.integers(cols, -8, 8, g)
        y = W.integers(m, -8, 8, g)
        r, _ = o_gemv(1.0, A, xv, 0.5, y)
        Ad, xvd = A.to(DEV), xv.to(DEV)
        pts = R.gemv_knob_points(cols, elem_bytes=eb)
        assert len(pts) > 50
        for kn, d in pts[::7]:
            banner("derived gemv", storage, kn)
            yd = y.to(DEV)
            L.gemv(1.0, Ad, xvd, 0.5, yd, knobs=L.knobs(**kn))
            assert np.array_equal(yd.cpu().numpy().astype(np.float64), r), (kn, str(d.expr))


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_every_lane_form_derivation_runs_integer_exact(gpu_device, storage):
    """Every derived asum / dot expression in the other lane forms (lanes on
    contiguous runs, lanes folded in order, one lane per work-group) at
    n = 2^16: its launch gives the exact sum on integer inputs."""
    n = 1 << 16
    g = W.gen(83)
    x = W.integers(n, -8, 8, g, storage)
    y = W.integers(n, -4, 4, g, storage)
    ra, rd = o_asum(x), o_dot(x, y)[0]
    xd, yd = x.to(DEV), y.to(DEV)
    eb = 4 if storage == "f32" else 2
    for op in ("asum", "dot"):
        pts = [(kn, d) for kn, d in R.derived_knob_points(op, n, elem_bytes=eb) if kn.get("lane_form")]
        assert len(pts) > 50 and {kn["lane_form"] for kn, _ in pts} == {1, 2, 3}
        assert any(kn["block"] == 1 for kn, _ in pts)
        banner("derived lane forms", storage, op, len(pts))
        for kn, d in pts:
            k = L.knobs(**kn)
            got = L.asum(xd, knobs=k).item() if op == "asum" else L.dot(xd, yd, knobs=k).item()
            assert got == (ra if op == "asum" else rd), (kn, str(d.expr))


@pytest.mark.parametrize("form", [1, 2, 3])
def test_lane_forms_small_and_ragged_sizes_exact(gpu_device, form):
    """The other lane forms at empty, tiny and ragged sizes, misaligned
    starts and the smallest blocks: exact sums on integer inputs."""
    g = W.gen(84 + form)
    blocks = (64, 256) if form == 2 else (1, 4, 64)
    for n in (0, 1, 5, 63, 64, 65, 1000, 4099):
        x = W.integers(n + 3, -8, 8, g)
        y = W.integers(n + 3, -4, 4, g)
        for off in (0, 1, 3):
            xs, ys = x[off:off + n], y[off:off + n]
            xd, yd = x.to(DEV)[off:off + n], y.to(DEV)[off:off + n]
            ra, rd = o_asum(xs), o_dot(xs, ys)[0]
            for block in blocks:
                for vb, u in ((16, 2), (4, 1)):
                    k = L.knobs(block=block, vec_bytes=vb, unroll=u, split=block * u * 8, lane_form=form)
                    banner("lane form small", form, n, off, block, vb, u)
                    assert L.asum(xd, knobs=k).item() == ra, (form, n, off, block, vb, u)
                    assert L.dot(xd, yd, knobs=k).item() == rd, (form, n, off, block, vb, u)


def test_lane_forms_binary64_result(gpu_device):
    """A lane form with a binary64 result: the binary32 value widened, equal
    to the binary32-result call's value."""
    g = W.gen(88)
    x = W.uniform((1 << 18) + 5, g).to(DEV)
    y = W.uniform((1 << 18) + 5, g).to(DEV)
    for form in (1, 2, 3):
        k = L.knobs(block=64 if form == 2 else 16, vec_bytes=16, unroll=2, split=1 << 12, lane_form=form)
        a32, a64 = L.asum(x, knobs=k).item(), L.asum(x, knobs=k, result_dtype=torch.float64).item()
        d32, d64 = L.dot(x, y, knobs=k).item(), L.dot(x, y, knobs=k, result_dtype=torch.float64).item()
        assert a64 == a32 and d64 == d32, form
