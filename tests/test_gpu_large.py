"""Sizes past 2^31 elements: every index of the streaming kernels is 64-bit.

The inputs are built on the GPU from short periodic patterns whose results
have closed forms in exact integer arithmetic, so a dropped, duplicated or
misplaced element changes the result.  For the reductions and gemv the
values are small integers: every lane, work-group and (with the binary64
combine) final partial sum is an exactly representable integer, so those
checks are exact; scal is compared with one binary32 multiply per element,
and BlackScholes checks that equal prices give equal pairs at every position
and that those pairs match the oracle.  Sizes are ragged (not a multiple of
any vector width or step), and misaligned views exercise the scalar heads.
About 35 GB of device memory at most (one case holds a 32 GB vector);
the tests free it as they go.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1502_02389_amd as L
from tests.gpu_util import banner

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
N = (1 << 31) + 4099


@pytest.fixture(autouse=True)
def _big_device(gpu_device):
    if torch.cuda.get_device_properties(0).total_memory < (64 << 30):
        pytest.skip("needs a device with at least 64 GiB")
    yield
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def periodic(n, values):
    """x[i] = values[i % len(values)] (binary32, on the device)."""
    base = torch.tensor(values, dtype=torch.float32, device=DEV)
    return base.repeat(-(-n // len(values)))[:n]


def periodic_sum(n, values, f=lambda v: v):
    """sum over i in [0, n) of f(values[i % p]), exactly (Python integers
    and exact binary fractions)."""
    p = len(values)
    full, rest = divmod(n, p)
    return full * sum(f(v) for v in values) + sum(f(values[k]) for k in range(rest))


def test_asum_and_dot_past_2p31():
    xv, yv = [-1.0, 0.0, 1.0], [1.0, 1.0, 0.0, -1.0]
    x = periodic(N, xv)
    y = periodic(N, yv)
    banner("asum / dot n = 2^31 + 4099")
    want_asum = periodic_sum(N, xv, f=abs)
    g = L.asum(x, acc="f64combine", result_dtype=torch.float64).item()
    assert g == want_asum, (g, want_asum)
    # plain binary32 combine: the final sum of ~256 exact partials rounds
    assert abs(L.asum(x).item() - want_asum) <= 1e-6 * want_asum
    # x y has period 12
    prod = [xv[i % 3] * yv[i % 4] for i in range(12)]
    want_dot = periodic_sum(N, prod)
    g = L.dot(x, y, acc="f64combine", result_dtype=torch.float64).item()
    assert g == want_dot, (g, want_dot)
    # misaligned views (scalar heads) over the same buffers: x[1:], y[1:]
    prod1 = [xv[(i + 1) % 3] * yv[(i + 1) % 4] for i in range(12)]
    want1 = periodic_sum(N - 1, prod1)
    g = L.dot(x[1:], y[1:], acc="f64combine", result_dtype=torch.float64).item()
    assert g == want1, (g, want1)
    want_a1 = periodic_sum(N - 1, [xv[(i + 1) % 3] for i in range(3)], f=abs)
    assert L.asum(x[1:], acc="f64combine", result_dtype=torch.float64).item() == want_a1
    del x, y


def test_scal_past_2p31():
    x = periodic(N, [1.5, -2.25, 3.0, 0.1, -7.0])
    banner("scal n = 2^31 + 4099")
    out = L.scal(2.5, x)
    assert torch.equal(out, x * 2.5)         # one binary32 multiply per element
    del out
    v = x[3:]                                  # in place on a misaligned view
    before = v[-5:].clone()
    L.scal(-0.5, v, out=v)
    assert torch.equal(v[-5:], before * -0.5)
    assert torch.equal(x[:3].cpu(), torch.tensor([1.5, -2.25, 3.0]))
    assert torch.equal(v[:5].cpu(), torch.tensor([0.1, -7.0, 1.5, -2.25, 3.0]) * -0.5)
    del x, v


def test_gemv_past_2p31_elements():
    m, n, lda = 65536, 32771, 32772           # m * lda > 2^31; ragged row tail
    i = torch.arange(m, device=DEV)[:, None]
    j = torch.arange(lda, device=DEV)[None, :]
    A = ((i + j) % 3).to(torch.float32) - 1.0
    del i, j
    torch.cuda.empty_cache()
    x = torch.ones(n, device=DEV)
    y0 = periodic(m, [1.0, 2.0])
    y = y0.clone()
    banner("gemv 65536 x 32771 (lda 32772)")
    L.gemv(1.0, A, x, 0.5, y, lda=lda)
    got = y.cpu().numpy()
    del A
    # row i sums ((i + j) % 3) - 1 over j < n: counts of each residue
    want = np.empty(m)
    for r in range(3):
        c = [sum(1 for k in range(3) if (r + k) % 3 == res) * (n // 3) for res in range(3)]
        for k in range(n % 3):
            c[(r + (n // 3) * 3 + k) % 3] += 1
        want[r::3] = c[2] - c[0]
    want += 0.5 * np.tile([1.0, 2.0], m // 2)
    assert np.array_equal(got.astype(np.float64), want)


def test_blackscholes_past_2p31():
    prices = [10.0, 20.0, 30.0, 25.5]
    n = (1 << 31) + 3
    s = periodic(n, prices)
    strike, rate, vol, years = 20.0, 0.02, 0.3, 1.0
    banner("blackscholes n = 2^31 + 3")
    out = L.blackscholes(s, strike, rate, vol, years)
    del s
    # the same price gives the same pair at every position (head, vector
    # body and tail alike); the four pairs match the oracle
    first = out[:4].cpu()
    for k in range(4):
        col = out[k::4]
        assert torch.equal(col, first[k].to(DEV).expand_as(col)), k
    ref = oracle.blackscholes(np.array(prices, dtype=np.float32), strike, rate, vol, years)
    scale = np.array(prices, dtype=np.float64) + strike * math.exp(-rate * years)
    err = np.abs(first.numpy().astype(np.float64) - ref) / scale[:, None]
    assert float(err.max()) <= 1e-5
    del out


def test_batch_with_a_problem_past_2p31():
    xv, yv = [-1.0, 0.0, 1.0], [1.0, 1.0, 0.0, -1.0]
    x = periodic(N, xv)
    y = periodic(N, yv)
    small = periodic(1000, [2.0, -1.0])
    A = torch.ones((3, 5), device=DEV)
    v = torch.ones(5, device=DEV)
    yg = torch.zeros(3, device=DEV)
    banner("batch with dot n = 2^31 + 4099")
    b = L.Batch([("dot", x, y), ("asum", small), ("gemv", 2.0, A, v, 0.0, yg), ("asum", x[1:])],
                acc="f64combine", result_dtype=torch.float64)
    b.run()
    torch.cuda.synchronize()
    prod = [xv[i % 3] * yv[i % 4] for i in range(12)]
    assert b.results[0].item() == periodic_sum(N, prod)
    assert b.results[1].item() == 1500.0
    assert torch.equal(yg.cpu(), torch.full((3,), 10.0))
    assert b.results[3].item() == periodic_sum(N - 1, [xv[(i + 1) % 3] for i in range(3)], f=abs)
    b.close()
    del x, y


def test_scal_grid_capped_below_2p32_work_items():
    # 2^33 + 5 elements with 1024-thread work-groups of one 4-byte load each:
    # the requested split would need 2^33 work-items; the library enlarges the
    # chunks so one dispatch stays below 2^32, and every element is still scaled
    n = (1 << 33) + 5
    vals = [1.0, -2.0, 0.5, 3.0, -0.25, 8.0, 6.0]
    x = periodic(n, vals)
    banner("scal 2^33 + 5 in place, tiny split")
    L.scal(2.5, x, out=x, knobs=L.knobs(block=1024, vec_bytes=4, unroll=1, split=1))
    torch.cuda.synchronize()
    for lo in (0, n // 3, n // 2 + 1, n - (1 << 20)):
        got = x[lo:lo + (1 << 20)].cpu().numpy()
        want = np.array([vals[(lo + i) % 7] * 2.5 for i in range(len(got))], dtype=np.float32)
        assert np.array_equal(got, want), lo
    del x
