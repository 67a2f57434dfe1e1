"""GPU parity: the HIP kernels against the binary64 oracle.

Bar (stated per test): integer-valued inputs whose partial sums stay below
2^24 in magnitude are bit-exact under every knob set; binary32 results are
within relative error 1e-5 of the oracle, measured as
  asum : |g - r| / r
  dot  : |g - r| / sum |x_i y_i|             (r can be ~0 by cancellation);
         for the seeded uniform workloads, whose |r| is far from 0, also
         |g - r| / |r|
  gemv : |g_i - r_i| / (|alpha| sum_j |A_ij x_j| + |beta y_i|)   per row
and scal is bit-exact: one correctly rounded binary32 multiply per element,
which is the binary64 oracle's exact product rounded to binary32.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1502_02389_amd as L
import workloads as W
from tests.gpu_util import banner, o_asum, o_dot, o_gemv, rel

pytestmark = pytest.mark.gpu

TOL = 1e-5
DEV = "cuda:0"


def sync():
    torch.cuda.synchronize()


# ------------------------------------------------------------------ asum


def test_asum_2p20_uniform(gpu_device):
    x = W.asum_small_vector()
    banner("asum uniform n", x.numel())
    g = L.asum(x.to(DEV)).item()
    r = o_asum(x)
    assert rel(g, r) <= TOL, (g, r)


def test_asum_2p20_integer_bitexact(gpu_device):
    x = W.asum_small_vector(integer=True)
    banner("asum integers n", x.numel())
    g = L.asum(x.to(DEV)).item()
    assert g == o_asum(x) == float(x.abs().sum().item())


SIZES = [0, 1, 3, 63, 64, 65, 255, 4095, 4096, 65537, (1 << 20) + 7]


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("offset", [0, 1, 2, 3])
def test_asum_sizes_offsets_integer(gpu_device, n, offset):
    g0 = W.gen(100 + n % 97 + offset)
    base = W.integers(n + offset, -8, 8, g0)
    banner("asum integers n", n, "offset", offset)
    dev = base.to(DEV)[offset:]
    g = L.asum(dev).item()
    assert g == o_asum(base[offset:].contiguous())


@pytest.mark.parametrize("n", [1, 5, 1000, (1 << 18) + 3])
def test_asum_sizes_uniform(gpu_device, n):
    x = W.uniform(n, W.gen(7 + n))
    banner("asum uniform n", n)
    assert rel(L.asum(x.to(DEV)).item(), o_asum(x)) <= TOL


def test_asum_special_values(gpu_device):
    x = torch.tensor([-0.0, -0.0, 3.0, -2.5], dtype=torch.float32)
    banner("asum special values")
    assert L.asum(x.to(DEV)).item() == 5.5
    xn = torch.tensor([1.0, float("nan"), 2.0])
    assert math.isnan(L.asum(xn.to(DEV)).item())
    xi = torch.tensor([-float("inf"), 1.0])
    assert L.asum(xi.to(DEV)).item() == math.inf


# ------------------------------------------------------------------ dot


def test_dot_2p24(gpu_device):
    x, y, _ = W.stream_vectors()
    banner("dot n", x.numel())
    g = L.dot(x.to(DEV), y.to(DEV)).item()
    r, mass = o_dot(x, y)
    assert abs(g - r) <= TOL * mass, (g, r, mass)
    # this input does not cancel (|r| ~ sqrt(n) / 3 >> 0): the plain relative
    # bar holds as well
    assert abs(r) > 1e-3 * mass ** 0.5
    assert abs(g - r) <= TOL * abs(r), (g, r)


def test_asum_2p24(gpu_device):
    x, _, _ = W.stream_vectors()
    banner("asum n", x.numel())
    assert rel(L.asum(x.to(DEV)).item(), o_asum(x)) <= TOL


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("ox,oy", [(0, 0), (1, 1), (3, 3), (1, 2), (0, 3)])
def test_dot_sizes_offsets_integer(gpu_device, n, ox, oy):
    g0 = W.gen(200 + n % 89 + 5 * ox + oy)
    bx = W.integers(n + ox, -4, 4, g0)
    by = W.integers(n + oy, -4, 4, g0)
    banner("dot integers n", n, "offsets", ox, oy)
    g = L.dot(bx.to(DEV)[ox:], by.to(DEV)[oy:]).item()
    r, _ = o_dot(bx[ox:].contiguous(), by[oy:].contiguous())
    assert g == r


def test_dot_orthogonal_and_hadamard(gpu_device):
    n = 1 << 16
    ones = torch.ones(n)
    alt = torch.where(torch.arange(n) % 2 == 0, 1.0, -1.0)
    banner("dot orthogonal")
    assert L.dot(ones.to(DEV), alt.to(DEV)).item() == 0.0
    H = torch.ones(1, 1)
    for _ in range(8):
        H = torch.cat([torch.cat([H, H], 1), torch.cat([H, -H], 1)], 0)
    Hd = H.to(DEV)
    for i, j in [(0, 0), (3, 3), (1, 2), (5, 200), (255, 17)]:
        assert L.dot(Hd[i], Hd[j]).item() == (256.0 if i == j else 0.0)


# ------------------------------------------------------------------ knob sweep


KNOB_POINTS = [(b, v, u, s) for b in (64, 256, 1024) for v in (4, 8, 16) for u in (1, 2, 4, 8)
               for s in (0, 4096, 1 << 17)]


def test_reduce_every_knob_point_integer_bitexact(gpu_device):
    n = (1 << 20) + 13
    g0 = W.gen(300)
    x = W.integers(n, -4, 4, g0)
    y = W.integers(n, -4, 4, g0)
    ra = o_asum(x)
    rd, _ = o_dot(x, y)
    xd, yd = x.to(DEV), y.to(DEV)
    for b, v, u, s in KNOB_POINTS:
        for il in (L.LIFT_INTERLEAVE_CHUNK, L.LIFT_INTERLEAVE_STRIDE):
            k = L.knobs(block=b, vec_bytes=v, unroll=u, split=s, interleave=il)
            banner("knobs", b, v, u, s, il)
            assert L.asum(xd, knobs=k).item() == ra, (b, v, u, s, il)
            assert L.dot(xd, yd, knobs=k).item() == rd, (b, v, u, s, il)


def test_interleave_default_is_stride_for_dot_chunk_for_asum(gpu_device):
    # interleave 0 leaves the partition to the library: grid-stride steps for
    # dot, contiguous chunks for asum.  The input is built so the two
    # partitions give different, exactly known sums.  Knobs: 256 lanes x 4
    # loads = steps of 1024 vectors, split 2^15 elements -> G = 128
    # work-groups over n = 2^22.  Step s holds v_s in its first element;
    # v_1 = v_2 = v_3 = 100, v_G = 2^30, everything else 0.
    #   chunk:  work-group 0 owns steps 0..S-1 (S >= 4): partial 300 exactly;
    #           2^30 sits in another work-group; combine: 2^30 + 300 -> 2^30 + 256
    #   stride: work-group 0 owns steps 0, G, ...: partial 2^30; work-groups
    #           1, 2, 3 hold 100 each; any balanced combine tree rounds
    #           2^30 + 100 up to 2^30 + 128, then + 200 to 2^30 + 384
    # (binary32 spacing at 2^30 is 128).
    n, G = 1 << 22, 128
    chunk, stride = L.LIFT_INTERLEAVE_CHUNK, L.LIFT_INTERLEAVE_STRIDE
    base = dict(block=256, vec_bytes=16, unroll=4, split=1 << 15)
    want = {chunk: 2.0 ** 30 + 256, stride: 2.0 ** 30 + 384}
    for storage, eb in (("f32", 4), ("bf16", 2)):
        e = 16 // eb
        x = torch.zeros(n)
        x[[1024 * e, 2048 * e, 3072 * e]] = 100.0
        x[G * 1024 * e] = 2.0 ** 30
        xd = x.to(W.STORAGE[storage]).to(DEV)
        yd = torch.ones(n, dtype=W.STORAGE[storage], device=DEV)
        banner("interleave default", storage)
        for il in (chunk, stride):
            assert L.asum(xd, knobs=L.knobs(**base, interleave=il)).item() == want[il], (storage, il)
            assert L.dot(xd, yd, knobs=L.knobs(**base, interleave=il)).item() == want[il], (storage, il)
        assert L.asum(xd, knobs=L.knobs(**base)).item() == want[chunk]
        assert L.dot(xd, yd, knobs=L.knobs(**base)).item() == want[stride]


def test_reduce_every_knob_point_uniform(gpu_device):
    n = (1 << 20) + 13
    g0 = W.gen(301)
    x = W.uniform(n, g0)
    y = W.uniform(n, g0)
    ra = o_asum(x)
    rd, mass = o_dot(x, y)
    xd, yd = x.to(DEV), y.to(DEV)
    for i, (b, v, u, s) in enumerate(KNOB_POINTS[::3]):
        k = L.knobs(block=b, vec_bytes=v, unroll=u, split=s,
                    interleave=(L.LIFT_INTERLEAVE_CHUNK, L.LIFT_INTERLEAVE_STRIDE)[i % 2])
        banner("knobs uniform", b, v, u, s, i % 2)
        assert rel(L.asum(xd, knobs=k).item(), ra) <= TOL
        assert abs(L.dot(xd, yd, knobs=k).item() - rd) <= TOL * mass


def test_grid_capped_at_max_workgroups(gpu_device):
    n = 64 * 4 * (L.lift_max_workgroups() + 100)
    x = W.integers(n, -2, 2, W.gen(302))
    banner("asum grid cap n", n)
    k = L.knobs(block=64, vec_bytes=16, unroll=1, split=256)
    assert L.asum(x.to(DEV), knobs=k).item() == float(x.abs().sum().item())


# ------------------------------------------------------------------ determinism / workspace


def test_reduce_bitwise_deterministic(gpu_device):
    x = W.asum_small_vector().to(DEV)
    y = W.uniform(x.numel(), W.gen(9)).to(DEV)
    banner("determinism")
    a0 = L.asum(x)
    d0 = L.dot(x, y)
    outs_a = torch.stack([L.asum(x) for _ in range(1000)])
    outs_d = torch.stack([L.dot(x, y) for _ in range(200)])
    assert torch.equal(outs_a, a0.expand(1000))
    assert torch.equal(outs_d, d0.expand(200))


def test_workspace_zero_after_calls_and_poisoned_slots(gpu_device):
    x = W.asum_small_vector()
    ws = L.workspace(torch.device(DEV))
    banner("workspace reset")
    r = o_asum(x)
    xd = x.to(DEV)
    hdr = L.lift_workspace_bytes() - 16 * L.lift_max_workgroups()   # counters precede the slots
    for k in (None, L.knobs(block=64, vec_bytes=16, unroll=1, split=256)):   # 1 and many arrival groups
        L.asum(xd, knobs=k)
        sync()
        assert int(ws[:hdr].count_nonzero().item()) == 0
        ws[hdr:].fill_(0xFF)                   # NaN / garbage in every partial slot
        g = L.asum(xd, knobs=k).item()
        assert rel(g, r) <= TOL
        assert int(ws[:hdr].count_nonzero().item()) == 0


def test_result_f64_and_raw_entry_point(gpu_device):
    x = W.asum_small_vector(integer=True)
    xd = x.to(DEV)
    banner("raw entry point")
    res = torch.zeros((), dtype=torch.float32, device=DEV)
    ws = L.workspace(torch.device(DEV))
    s = torch.cuda.current_stream().cuda_stream
    assert L.lift_asum(x.numel(), xd.data_ptr(), res.data_ptr(), ws.data_ptr(), ws.numel(), s) == 0
    r64 = L.asum(xd, result_dtype=torch.float64)
    assert res.item() == r64.item() == o_asum(x)


# ------------------------------------------------------------------ scal


def _scal_check(x: torch.Tensor, alpha: float, got: torch.Tensor):
    want = oracle.scal(alpha, x.numpy()).astype(np.float32)
    assert np.array_equal(got.cpu().numpy().view(np.uint32), want.view(np.uint32))


def test_scal_2p24_bitexact(gpu_device):
    x, _, alpha = W.stream_vectors()
    banner("scal 2^24")
    _scal_check(x, alpha, L.scal(alpha, x.to(DEV)))


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("offset", [0, 1, 3])
def test_scal_sizes_offsets(gpu_device, n, offset):
    base = W.uniform(n + offset, W.gen(400 + n % 31))
    banner("scal n", n, "offset", offset)
    xd = base.to(DEV)[offset:]
    _scal_check(base[offset:].contiguous(), 2.5, L.scal(2.5, xd))


def test_scal_in_place_and_mismatched_phase(gpu_device):
    base = W.uniform(10001, W.gen(401))
    banner("scal in place / phase")
    xd = base.to(DEV)
    L.scal(-0.75, xd, out=xd)
    _scal_check(base, -0.75, xd)
    src = W.uniform(5000, W.gen(402))
    buf = torch.empty(5003, device=DEV)
    out = buf[1:5001]                          # out and x differ in 16-byte phase
    L.scal(3.0, src.to(DEV), out=out)
    _scal_check(src, 3.0, out)


def test_scal_subnormals_and_specials(gpu_device):
    x = torch.tensor([1e-45, -1e-45, 1e-40, 0.0, -0.0, 3.4e38, float("inf"), float("nan")] * 9,
                     dtype=torch.float32)
    banner("scal specials")
    got = L.scal(2.5, x.to(DEV)).cpu().numpy()
    with np.errstate(all="ignore"):
        want = (np.float32(2.5) * x.numpy())
    nan = np.isnan(want)
    assert np.array_equal(np.isnan(got), nan)
    assert np.array_equal(got[~nan].view(np.uint32), want[~nan].view(np.uint32))


def test_scal_knob_points(gpu_device):
    x = W.uniform((1 << 20) + 5, W.gen(403))
    xd = x.to(DEV)
    for b in (64, 256, 1024):
        for v in (4, 8, 16):
            for u in (1, 2, 4, 8):
                for s in (0, 1 << 16):
                    banner("scal knobs", b, v, u, s)
                    _scal_check(x, 1.5, L.scal(1.5, xd, knobs=L.knobs(block=b, vec_bytes=v, unroll=u, split=s)))


# ------------------------------------------------------------------ gemv


def _gemv_check(alpha, A, x, beta, y0, got, n=None, tol=TOL):
    r, mass = o_gemv(alpha, A, x, beta, y0, n)
    g = got.cpu().numpy().astype(np.float64)
    err = np.abs(g - r)
    assert np.all(err <= tol * mass + 1e-30), (float(np.max(err / np.maximum(mass, 1e-300))))


@pytest.mark.parametrize("size", W.GEMV_SIZES)
def test_gemv_square(gpu_device, size):
    A, x, y, alpha, beta = W.gemv_square(size)
    banner("gemv square", size)
    yd = y.to(DEV)
    L.gemv(alpha, A.to(DEV), x.to(DEV), beta, yd)
    _gemv_check(alpha, A, x, beta, y, yd)


def test_gemv_integer_bitexact_nonsquare_lda(gpu_device):
    g0 = W.gen(500)
    m, n, lda = 1000, 777, 800
    A = W.integers((m, lda), -8, 8, g0)
    x = W.integers(n, -8, 8, g0)
    y = W.integers(m, -8, 8, g0)
    banner("gemv integers", m, n, lda)
    r, _ = o_gemv(1.0, A, x, 0.5, y)
    Ad, xd = A.to(DEV), x.to(DEV)
    for rows in (1, 2, 4):
        for v in (4, 8, 16):
            for u in (1, 2, 4, 8):
                for b in (64, 256, 1024):
                    yd = y.to(DEV)
                    L.gemv(1.0, Ad, xd, 0.5, yd, lda=lda,
                           knobs=L.knobs(block=b, vec_bytes=v, unroll=u, rows_per_wave=rows, row_split=1))
                    assert np.array_equal(yd.cpu().numpy().astype(np.float64), r), (rows, v, u, b)
    # work-group-per-row form
    for rows in (1, 2):
        for v in (4, 16):
            for u in (2, 4, 8):
                for b in (64, 256, 1024):
                    yd = y.to(DEV)
                    L.gemv(1.0, Ad, xd, 0.5, yd, lda=lda,
                           knobs=L.knobs(block=b, vec_bytes=v, unroll=u, rows_per_wave=rows, row_split=2))
                    assert np.array_equal(yd.cpu().numpy().astype(np.float64), r), ("split", rows, v, u, b)


@pytest.mark.parametrize("m,n,lda", [(20011, 37, 40), (50, 3, 4), (333, 2048, 2048)])
def test_gemv_row_split_many_rows_per_workgroup_integer_bitexact(gpu_device, m, n, lda):
    # wg_per_cu=1 caps the grid at one work-group per compute unit, so each
    # work-group visits many rows (several flushes of 16 parked rows, both LDS
    # banks, a partial last flush); n=3 has no whole vector, only the tail;
    # n=2048 with small block * unroll streams x instead of holding it.
    g0 = W.gen(503)
    A = W.integers((m, lda), -8, 8, g0)
    x = W.integers(n, -8, 8, g0)
    y = W.integers(m, -8, 8, g0)
    r, _ = o_gemv(1.0, A, x, 0.5, y)
    Ad, xd = A.to(DEV), x.to(DEV)
    for rows in (1, 2):
        for v in (4, 16):
            for u in (2, 8):
                for b in (64, 256):
                    banner("gemv row split rows", m, n, lda, rows, v, u, b)
                    yd = y.to(DEV)
                    L.gemv(1.0, Ad, xd, 0.5, yd, lda=lda,
                           knobs=L.knobs(block=b, vec_bytes=v, unroll=u, rows_per_wave=rows, row_split=2,
                                         wg_per_cu=1))
                    assert np.array_equal(yd.cpu().numpy().astype(np.float64), r), (rows, v, u, b)


@pytest.mark.parametrize("size", W.GEMV_SIZES)
def test_gemv_square_row_split(gpu_device, size):
    A, x, y, alpha, beta = W.gemv_square(size)
    banner("gemv square row split", size)
    Ad, xd = A.to(DEV), x.to(DEV)
    for rows, u in ((1, 8), (2, 4)):
        yd = y.to(DEV)
        L.gemv(alpha, Ad, xd, beta, yd, knobs=L.knobs(block=256, vec_bytes=16, unroll=u, rows_per_wave=rows,
                                                     row_split=2))
        _gemv_check(alpha, A, x, beta, y, yd)


@pytest.mark.parametrize("m,n,lda", [(1, 1, 1), (3, 5, 5), (7, 64, 64), (65, 257, 259), (130, 4099, 4100),
                                     (9, 1000, 1003)])
def test_gemv_shapes(gpu_device, m, n, lda):
    g0 = W.gen(501 + m)
    A = W.normal((m, lda), g0)
    x = W.normal(n, g0)
    y = W.normal(m, g0)
    banner("gemv shape", m, n, lda)
    yd = y.to(DEV)
    L.gemv(1.25, A.to(DEV), x.to(DEV), -0.5, yd, lda=lda)
    _gemv_check(1.25, A, x, -0.5, y, yd)


def test_gemv_beta_zero_ignores_nan_y_and_empty(gpu_device):
    g0 = W.gen(502)
    A = W.normal((33, 100), g0)
    x = W.normal(100, g0)
    banner("gemv beta 0 / empty")
    yd = torch.full((33,), float("nan"), device=DEV)
    L.gemv(2.0, A.to(DEV), x.to(DEV), 0.0, yd)
    assert torch.isfinite(yd).all()
    _gemv_check(2.0, A, x, 0.0, torch.zeros(33), yd)
    # n = 0: y = beta * y
    y = W.normal(5, g0)
    yd = y.to(DEV)
    L.gemv(2.0, torch.zeros((5, 1), device=DEV), torch.zeros(0, device=DEV), 0.5, yd, lda=1)
    assert torch.equal(yd.cpu(), 0.5 * y)
    # m = 0: nothing happens
    L.gemv(1.0, torch.zeros((0, 4), device=DEV), torch.zeros(4, device=DEV), 1.0, torch.zeros(0, device=DEV))
    sync()


# ------------------------------------------------------------------ profiling hook


def test_time_next_launch_brackets_one_kernel(gpu_device):
    x = W.uniform(1 << 22, W.gen(700)).to(DEV)
    ev = L.HipEvents(2)
    banner("timing hook")
    try:
        assert L.lift_time_next_launch(ev.events[0], ev.events[1]) == 0
        r1 = L.asum(x)                      # timed launch
        r2 = L.asum(x)                      # hook already cleared: plain launch
        sync()
        ms = ev.elapsed_ms(0, 1)
        assert 0.0 < ms < 50.0
        assert r1.item() == r2.item()
    finally:
        ev.close()
