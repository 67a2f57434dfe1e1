"""GPU parity at the paper's large sizes, in the launches the benchmark times.

Section 7.2 of the paper runs scal, asum and dot on 128M-element vectors
(2^27 binary32, 512 MiB each) and gemv on an 8192 x 16384 matrix with a
vector of 8192.  Which side the 8192-vector is on is ambiguous (the map over
rows makes x as long as a row), so both shapes run: 8192 rows of 16384
columns and 16384 rows of 8192 columns.  Every call goes through the plain C
entry points with no knobs, the calls bench.py times; the whole output is
compared with the binary64 oracle:
  scal : bit-exact (one correctly rounded binary32 multiply per element)
  asum : |g - r| / r <= 1e-5
  dot  : |g - r| / sum |x_i y_i| <= 1e-5, and |g - r| / |r| <= 1e-5 (|r| is
         far from 0 for these inputs, ~sqrt(n) / 3)
  gemv : every row |g_i - r_i| <= 1e-5 (|alpha| sum_j |A_ij x_j| + |beta y_i|)
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1502_02389_amd as L
import workloads as W
from tests.gpu_util import banner

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = 1e-5


@pytest.fixture(scope="module")
def vectors(gpu_device):
    x, y, alpha = W.stream_vectors(W.LARGE_N)
    return x, y, alpha


def test_scal_asum_dot_2p27_default_launch(vectors):
    x, y, alpha = vectors
    n = x.numel()
    xd, yd = x.to(DEV), y.to(DEV)
    out = torch.empty_like(xd)
    ws = L.workspace(torch.device(DEV))
    res = torch.zeros(2, dtype=torch.float32, device=DEV)
    sh = torch.cuda.current_stream().cuda_stream
    banner("scal / asum / dot fp32 n = 2^27, plain entry points")
    assert L.lift_scal(n, alpha, xd.data_ptr(), out.data_ptr(), sh) == 0
    assert L.lift_asum(n, xd.data_ptr(), res.data_ptr(), ws.data_ptr(), ws.numel(), sh) == 0
    assert L.lift_dot(n, xd.data_ptr(), yd.data_ptr(), res.data_ptr() + 4, ws.data_ptr(), ws.numel(), sh) == 0
    torch.cuda.synchronize()
    xs, ys = x.numpy(), y.numpy()
    want = oracle.scal(alpha, xs).astype(np.float32)
    assert np.array_equal(out.cpu().numpy().view(np.uint32), want.view(np.uint32))
    del out
    ga, gd = (float(v) for v in res.cpu())
    ra = oracle.asum(xs)
    assert abs(ga - ra) <= TOL * ra, (ga, ra)
    rd = oracle.dot(xs, ys)
    mass = oracle.dot_absmass(xs, ys)
    assert abs(gd - rd) <= TOL * mass, (gd, rd, mass)
    assert abs(rd) > 1e-3 * mass ** 0.5
    assert abs(gd - rd) <= TOL * abs(rd), (gd, rd)


@pytest.mark.parametrize("m,n", [(8192, 16384), (16384, 8192)])
def test_gemv_paper_large_shape_default_launch(gpu_device, m, n):
    A, x, y, alpha, beta = W.gemv_rect(m, n)
    Ad, xd, yd = A.to(DEV), x.to(DEV), y.to(DEV)
    sh = torch.cuda.current_stream().cuda_stream
    banner("gemv fp32", m, "x", n, "plain entry point")
    assert L.lift_gemv(m, n, alpha, Ad.data_ptr(), n, xd.data_ptr(), beta, yd.data_ptr(), sh) == 0
    torch.cuda.synchronize()
    del Ad
    r = oracle.gemv(alpha, A.numpy(), x.numpy(), beta, y.numpy())
    mass = oracle.gemv_absmass(alpha, A.numpy(), x.numpy(), beta, y.numpy())
    g = yd.cpu().numpy().astype(np.float64)
    err = np.abs(g - r) / mass
    assert float(err.max()) <= TOL, float(err.max())
