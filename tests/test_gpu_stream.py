"""The bandwidth reference kernels (flat read and copy) on the GPU.

The copy must reproduce its input bit for bit at every launch shape the
benchmark's sweep uses (and ragged sizes); the read kernel must load every
vector it owns, which a constructed input shows: with one vector whose four
words XOR to the kernel's tag, exactly that fold reaches the sink.
"""
import itertools

import numpy as np
import pytest
import torch

import paper_1502_02389_amd as L
import workloads as W
from tests.gpu_util import banner

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TAG = 0x5EED1E55


def _sh():
    return torch.cuda.current_stream().cuda_stream


@pytest.mark.parametrize("n", [4, 1024, (1 << 20) + 12, (1 << 22) + 4])
def test_copy_is_bitwise_at_every_sweep_shape(gpu_device, n):
    x = W.uniform(n, W.gen(900 + n % 7)).to(DEV)
    for b, u, w, il in itertools.product((256, 512, 1024), (4, 8), (1, 2, 8),
                                         (L.LIFT_INTERLEAVE_CHUNK, L.LIFT_INTERLEAVE_STRIDE)):
        out = torch.full_like(x, float("nan"))
        banner("stream copy n", n, "knobs", b, u, w, il)
        kn = L.knobs(block=b, unroll=u, wg_per_cu=w, interleave=il)
        assert L.lift_stream_copy(n, x.data_ptr(), out.data_ptr(), kn, _sh()) == 0
        assert torch.equal(out.view(torch.int32), x.view(torch.int32)), (b, u, w, il)


def test_read_loads_the_tagged_vector(gpu_device):
    words = np.array([0x12345678, 0x0F0F0F0F, 0xA5A5A5A5, 0], dtype=np.uint32)
    words[3] = np.uint32(TAG) ^ words[0] ^ words[1] ^ words[2]
    x = torch.from_numpy(words.view(np.float32).copy()).to(DEV)
    sink = torch.zeros(1, dtype=torch.int32, device=DEV)
    banner("stream read tag")
    assert L.lift_stream_read(4, x.data_ptr(), sink.data_ptr(), None, _sh()) == 0
    assert int(sink.item()) & 0xFFFFFFFF == TAG
    # an all-zero input folds to 0 everywhere: nothing is written
    z = torch.zeros(1 << 20, device=DEV)
    sink.zero_()
    for il in (L.LIFT_INTERLEAVE_CHUNK, L.LIFT_INTERLEAVE_STRIDE):
        assert L.lift_stream_read(z.numel(), z.data_ptr(), sink.data_ptr(), L.knobs(interleave=il), _sh()) == 0
    assert int(sink.item()) == 0
