"""The allocation-free dot (lift_dot_ex_noalloc) against lift_dot_ex.

Both run the same kernels with the same partition; only the home of the
arrival counters and partial slots differs (a static device array inside
the library against a caller workspace), so the results must be equal bit
for bit.  Two calls in a row, the second on a smaller input (the array keeps
the first call's partials and must still give the second call's result),
for binary32 and bfloat16 storage, both result types and explicit knobs; a
third pass with integer inputs checks the exact value too.
"""
import numpy as np
import pytest
import torch

import paper_1502_02389_amd as L
import workloads as W
from tests.gpu_util import banner, o_dot

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _pair(n, storage, seed):
    g = W.gen(seed)
    return W.uniform(n, g, storage), W.uniform(n, g, storage)


@pytest.mark.parametrize("storage,code", [("f32", L.LIFT_F32), ("bf16", L.LIFT_BF16)])
@pytest.mark.parametrize("rt", [L.LIFT_F32, L.LIFT_F64])
@pytest.mark.parametrize("kn", [None, dict(block=512, vec_bytes=8, unroll=2, split=1 << 14)])
def test_noalloc_equals_workspace_form_twice_shrinking(gpu_device, storage, code, rt, kn):
    s = torch.cuda.current_stream().cuda_stream
    ws = L.workspace(torch.device(DEV))
    knobs = L.knobs(**kn) if kn else None
    rdt = torch.float32 if rt == L.LIFT_F32 else torch.float64
    for n in ((1 << 24) + 3, 100003):      # second call smaller: fewer work-groups, stale slots beyond
        x, y = _pair(n, storage, 3000 + n % 97)
        xd, yd = x.to(DEV), y.to(DEV)
        a = torch.full((1,), float("nan"), dtype=rdt, device=DEV)
        b = torch.full((1,), float("nan"), dtype=rdt, device=DEV)
        banner("noalloc dot", storage, "rt", rt, "n", n, "knobs", kn)
        assert L.lift_dot_ex_noalloc(n, code, xd.data_ptr(), yd.data_ptr(), 0, rt, a.data_ptr(), knobs, s) == 0
        assert L.lift_dot_ex(n, code, xd.data_ptr(), yd.data_ptr(), 0, rt, b.data_ptr(), ws.data_ptr(),
                             ws.numel(), knobs, s) == 0
        torch.cuda.synchronize()
        assert torch.equal(a.view(torch.uint8), b.view(torch.uint8)), (a.item(), b.item())
        r, mass = o_dot(x, y)
        assert abs(a.item() - r) <= 1e-5 * mass


def test_noalloc_integer_exact_and_empty(gpu_device):
    s = torch.cuda.current_stream().cuda_stream
    for n in (1 << 20, 4099, 0):
        g = W.gen(3100 + n)
        x, y = W.integers(n, -4, 4, g), W.integers(n, -4, 4, g)
        xd, yd = x.to(DEV), y.to(DEV)
        a = torch.full((1,), float("nan"), device=DEV)
        banner("noalloc dot integers n", n)
        assert L.lift_dot_ex_noalloc(n, L.LIFT_F32, xd.data_ptr(), yd.data_ptr(), 0, L.LIFT_F32, a.data_ptr(),
                                     None, s) == 0
        torch.cuda.synchronize()
        assert a.item() == float(np.dot(x.numpy().astype(np.float64), y.numpy().astype(np.float64)))
