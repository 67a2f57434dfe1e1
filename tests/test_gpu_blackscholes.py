"""GPU parity of BlackScholes (map(BSComputation) over stock prices).

Bar: every call and put within 2e-6 of the binary64 oracle, measured against
the magnitude of the two terms of the formula, s + K e^{-rT} (deep
out-of-the-money prices are tiny differences of those terms, so a plain
relative error is unbounded there).  The kernel is binary32 with the
hardware log2 / exp2 / reciprocal and a fitted polynomial for the normal
tail; the expected error is ~5e-7 of that scale (a few binary32 roundings
of each term), so 2e-6 leaves a factor of 4 and still catches an error of
8e-5 absolute at the workload's strike of 20.
"""
import math

import numpy as np
import pytest
import torch

import paper_1502_02389_amd as L
import workloads as W
from tests.gpu_util import banner

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
BAR = 2e-6


def oracle_pairs(s, params):
    import oracle

    return oracle.blackscholes(s.numpy(), *params)


def check(got, s, params):
    K, r, _, T = params
    ref = oracle_pairs(s, params)
    scale = s.numpy().astype(np.float64) + K * math.exp(-r * T)
    g = got.cpu().numpy().astype(np.float64).reshape(-1, 2)
    err = np.abs(g - ref) / scale[:, None]
    assert np.all(np.isfinite(g))
    worst = float(err.max()) if err.size else 0.0
    assert worst <= BAR, worst
    return worst


@pytest.mark.parametrize("launch", ["plain entry point", "library defaults"])
def test_full_size_prices(gpu_device, launch):
    s, params = W.blackscholes_prices()
    banner("blackscholes 2^22", params, launch)
    sd = s.to(DEV)
    out = torch.empty((s.numel(), 2), dtype=torch.float32, device=DEV)
    if launch == "plain entry point":   # no knobs (the tuned entry on this device): the call the benchmark times
        assert L.lift_blackscholes(s.numel(), sd.data_ptr(), *params, out.data_ptr(),
                                   torch.cuda.current_stream().cuda_stream) == 0
    else:                               # explicit all-zero knobs: the built-in defaults
        assert L.lift_blackscholes_ex(s.numel(), sd.data_ptr(), *params, out.data_ptr(), L.knobs(),
                                      torch.cuda.current_stream().cuda_stream) == 0
    check(out, s, params)
    # put-call parity holds on the GPU result too
    K, r, _, T = params
    g = out.cpu().numpy().astype(np.float64)
    par = g[:, 0] - g[:, 1] - (s.numpy() - K * math.exp(-r * T))
    assert float(np.max(np.abs(par) / (s.numpy() + K))) <= BAR


KNOBS = [dict(block=64, vec_bytes=4, unroll=1), dict(block=256, vec_bytes=8, unroll=2),
         dict(block=1024, vec_bytes=16, unroll=4, wg_per_cu=2), dict(block=128, vec_bytes=16, unroll=8, split=4096),
         dict(block=512, vec_bytes=8, unroll=4, wg_per_cu=32), dict(block=256, vec_bytes=4, unroll=8, split=100)]


@pytest.mark.parametrize("kn", KNOBS, ids=[str(i) for i in range(len(KNOBS))])
def test_every_knob_point_offsets_and_ragged_tail(gpu_device, kn):
    g = W.gen(61)
    n = 3 * 4096 + 37
    s = torch.rand(n + 3, generator=g) * 25 + 5
    params = (20.0, 0.02, 0.3, 1.0)
    sd = s.to(DEV)
    buf = torch.empty(2 * n + 8, device=DEV)
    for so in (0, 1, 2, 3):            # price misalignment in elements
        for oo in (0, 2):              # output offset in floats (one pair)
            banner("blackscholes knobs", kn, so, oo)
            out = buf[oo: oo + 2 * n]
            st = L.lift_blackscholes_ex(n, sd[so:].data_ptr(), *params, out.data_ptr(), L.knobs(**kn),
                                        torch.cuda.current_stream().cuda_stream)
            assert st == L.LIFT_OK
            check(out, s[so: so + n].contiguous(), params)


def test_small_and_extreme_inputs(gpu_device):
    params = (20.0, -0.01, 0.45, 2.5)
    cases = [torch.tensor([20.0]), torch.tensor([1e-3, 19.999, 20.0, 20.001, 1e4]),
             torch.linspace(0.5, 200.0, 333)]
    for s in cases:
        banner("blackscholes small", s.numel())
        check(L.blackscholes(s.to(DEV), *params), s, params)
    out = L.blackscholes(torch.zeros(0, device=DEV), *params)
    assert out.shape == (0, 2)


def test_parameter_sweep(gpu_device):
    s = torch.rand(5000, generator=W.gen(62)) * 60 + 1
    sd = s.to(DEV)
    for params in [(40.0, 0.1, 0.2, 0.5), (10.0, 0.0, 0.8, 10.0), (100.0, 0.05, 0.05, 0.02),
                   (3.0, -0.02, 0.3, 1.0)]:
        banner("blackscholes params", params)
        check(L.blackscholes(sd, *params), s, params)


def test_bitwise_deterministic(gpu_device):
    s, params = W.blackscholes_prices(n=1 << 20)
    sd = s.to(DEV)
    a = L.blackscholes(sd, *params)
    for _ in range(5):
        assert torch.equal(L.blackscholes(sd, *params), a)
