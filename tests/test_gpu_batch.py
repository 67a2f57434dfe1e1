"""GPU parity of the batched form (a run of two persistent launches, reduction
tiles then gemv tiles, over many problems).

Each problem's result is held to the same bar as the per-call form: integer
inputs bit-exact; binary32 within 1e-5 (asum relative, dot over sum|x y|,
gemv per row over |alpha| sum|A x| + |beta y|); 16-bit storage against the
oracle on the stored values.  Graph replays are checked against an eager run.
"""
import math

import numpy as np
import pytest
import torch

import paper_1502_02389_amd as L
import workloads as W
from tests.gpu_util import banner, o_asum, o_dot, o_gemv, rel

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
BOUND = {"f32": 1e-5, "comp": 1e-6, "f64combine": 1e-5}


def _dev_copy(t, offset):
    """t on the GPU, starting `offset` elements past an allocation start."""
    buf = torch.empty(t.numel() + offset, dtype=t.dtype, device=DEV)
    v = buf[offset:]
    v.copy_(t.to(DEV))
    return v


def build(spec, storage="f32", integer=False, seed=41, offsets=True, pad_lda=True, beta_zero=True):
    """CPU inputs, device problems and expected oracle values for a spec."""
    g = W.gen(seed)
    cpu, problems = [], []
    for i, (kind, n) in enumerate(zip(spec.red_kind, spec.red_len)):
        mk = (lambda k: W.integers(k, -4, 4, g, storage)) if integer else (lambda k: W.uniform(k, g, storage))
        x = mk(n)
        y = mk(n) if kind == "dot" else None
        ox = (i % 5 == 1) and offsets
        oy = (i % 7 == 3) and offsets
        xd = _dev_copy(x, 1 if ox else 0)
        if kind == "dot":
            problems.append(("dot", xd, _dev_copy(y, 1 if (oy or ox) else 0)))
        else:
            problems.append(("asum", xd))
        cpu.append((kind, x, y))
    for j, (m, n) in enumerate(spec.gemv_mn):
        lda = n + (3 if (pad_lda and j % 3 == 0) else 0)
        if integer:
            A = W.integers((m, lda), -4, 4, g, storage)
            x = W.integers(n, -4, 4, g)
            y = W.integers(m, -4, 4, g)
        else:
            A = W.normal((m, lda), g, storage)
            x = W.normal(n, g)
            y = W.normal(m, g)
        beta = 0.0 if (beta_zero and j % 4 == 0) else 0.5
        alpha = 1.0 if integer else 1.25
        yd = y.to(DEV) if beta != 0.0 else torch.full((m,), float("nan"), device=DEV)
        problems.append(("gemv", alpha, A.to(DEV), _dev_copy(x, 1 if (offsets and j % 5 == 2) else 0), beta, yd))
        cpu.append(("gemv", (alpha, A, x, beta, y, n)))
    return cpu, problems


def check(cpu, batch, problems, bound, exact=False):
    worst = 0.0
    for i, item in enumerate(cpu):
        if item[0] == "gemv":
            alpha, A, x, beta, y, n = item[1]
            r, mass = o_gemv(alpha, A, x, beta, y, n)
            g = problems[i][5].cpu().numpy().astype(np.float64)
            if exact:
                assert np.array_equal(g, r), i
            else:
                e = float(np.max(np.abs(g - r) / np.maximum(mass, 1e-300))) if len(r) else 0.0
                worst = max(worst, e)
                assert e <= bound, (i, e)
        else:
            kind, x, y = item
            got = batch.results[i].item()
            if kind == "asum":
                r = o_asum(x)
                e = 0.0 if exact else rel(got, r)
            else:
                r, mass = o_dot(x, y)
                e = 0.0 if exact else (abs(got - r) / mass if mass else abs(got))
            if exact:
                assert got == r, (i, kind, got, r)
            worst = max(worst, e)
            assert e <= bound, (i, kind, got, r, e)
    return worst


def small_spec(seed=40, n_red=240, n_gemv=24):
    return W.batch_shapes(n_red=n_red, n_gemv=n_gemv, lo_exp=0.0, hi_exp=17.0, mn_lo=1, mn_hi=700, seed=seed)


def test_batch_small_mixed_f32(gpu_device):
    cpu, problems = build(small_spec())
    banner("batch small f32")
    b = L.Batch(problems)
    b.run()
    torch.cuda.synchronize()
    check(cpu, b, problems, 1e-5)
    b.close()


def test_batch_degenerate_problems(gpu_device):
    g = W.gen(45)
    x0 = torch.zeros(0, device=DEV)
    x1 = W.uniform(1, g).to(DEV)
    x3 = W.uniform(3, g).to(DEV)
    y5 = W.normal(5, g)
    yd = y5.to(DEV)
    banner("batch degenerate")
    b = L.Batch([("asum", x0), ("dot", x0, x0), ("asum", x1), ("dot", x3, x3),
                 ("gemv", 2.0, torch.zeros((5, 1), device=DEV), torch.zeros(0, device=DEV), 0.5, yd),
                 ("gemv", 1.0, torch.zeros((0, 4), device=DEV), torch.zeros(4, device=DEV), 1.0,
                  torch.zeros(0, device=DEV))])
    b.run()
    torch.cuda.synchronize()
    assert b.results[0].item() == 0.0 and b.results[1].item() == 0.0
    assert b.results[2].item() == abs(x1.item())
    assert rel(b.results[3].item(), float((x3.double() * x3.double()).sum().item())) <= 1e-6
    assert torch.equal(yd.cpu(), 0.5 * y5)
    b.close()


KNOBS = [dict(), dict(block=64, vec_bytes=4, unroll=1, split=256, wg_per_cu=1),
         dict(block=512, vec_bytes=16, unroll=8, split=1 << 18, wg_per_cu=4),
         dict(block=256, vec_bytes=8, unroll=2, split=4096, wg_per_cu=8),
         dict(block=512, vec_bytes=16, unroll=4, split=1 << 15, wg_per_cu=2)]


@pytest.mark.parametrize("kn", KNOBS, ids=[str(i) for i in range(len(KNOBS))])
def test_batch_integer_bitexact_every_knob_point(gpu_device, kn):
    cpu, problems = build(small_spec(seed=46, n_red=120, n_gemv=12), integer=True, seed=47)
    banner("batch integers knobs", kn)
    b = L.Batch(problems, knobs=L.knobs(**kn))
    b.run()
    torch.cuda.synchronize()
    check(cpu, b, problems, 0.0, exact=True)
    b.close()


@pytest.mark.parametrize("storage", ["bf16", "f16"])
@pytest.mark.parametrize("acc", ["f32", "comp", "f64combine"])
def test_batch_16bit_storage_variants(gpu_device, storage, acc):
    cpu, problems = build(small_spec(seed=48, n_red=120, n_gemv=12), storage=storage, seed=49)
    banner("batch", storage, acc)
    b = L.Batch(problems, acc=acc, result_dtype=torch.float64)
    b.run()
    torch.cuda.synchronize()
    check(cpu, b, problems, BOUND[acc])
    b.close()


def test_batch_bitwise_deterministic_across_runs(gpu_device):
    cpu, problems = build(small_spec(seed=50, n_red=200, n_gemv=0), seed=51)
    banner("batch determinism")
    b = L.Batch(problems)
    b.run()
    first = torch.stack([r for r in b.results])
    for _ in range(20):
        b.run()
    again = torch.stack([r for r in b.results])
    assert torch.equal(first, again)
    b.close()


def test_batch_graph_replays_match_eager(gpu_device):
    cpu, problems = build(small_spec(seed=52, n_red=160, n_gemv=16), seed=53, beta_zero=False)
    gemv_ys = [p[5] for p in problems if p[0] == "gemv"]
    y0 = [y.clone() for y in gemv_ys]
    banner("batch graph")
    b = L.Batch(problems)
    b.run()
    torch.cuda.synchronize()
    eager_red = [r.clone() if r is not None else None for r in b.results]
    eager_y = [y.clone() for y in gemv_ys]
    check(cpu, b, problems, 1e-5)
    side = torch.cuda.Stream()
    g = b.capture(side)
    scratch = W.uniform(1 << 20, W.gen(54)).to(DEV)
    for rep in range(4):
        for y, y_init in zip(gemv_ys, y0):        # eager work between replays
            y.copy_(y_init)
        for r in b.results:
            if r is not None:
                r.fill_(-1.0)
        L.asum(scratch)
        torch.cuda.synchronize()
        g.launch(side)
        side.synchronize()
        for r, e in zip(b.results, eager_red):
            if r is not None:
                assert torch.equal(r, e), rep
        for y, e in zip(gemv_ys, eager_y):
            assert torch.equal(y, e), rep
    b.close()


@pytest.mark.parametrize("storage,knobs", [("f32", "default"), ("f32", "tuned"), ("bf16", "tuned")])
def test_batch_full_size_sampled(gpu_device, storage, knobs):
    # the benchmarked workload and launch (no knobs: the library's tuned
    # entry on this device, as the benchmark runs it), and the built-in
    # defaults (explicit all-zero knobs)
    spec = W.batch_shapes()
    code = {"f32": L.LIFT_F32, "bf16": L.LIFT_BF16}[storage]
    kn = None if knobs == "tuned" else L.knobs()
    if knobs == "tuned":
        assert L.lift_default_knobs("batch", code, 0, 0)[0] == 1
    banner(f"batch 4096 reductions + 256 gemv, full size, {storage}, {knobs} knobs")
    reds, gemvs = W.batch_values(spec, storage)
    problems = []
    for kind, x, y in reds:
        problems.append(("dot", x.to(DEV), y.to(DEV)) if kind == "dot" else ("asum", x.to(DEV)))
    gd = []
    for (A, x, y) in gemvs:
        gd.append(("gemv", 1.0, A.to(DEV), x.to(DEV), 0.5, y.to(DEV)))
    b = L.Batch(problems + gd, knobs=kn)
    b.run()
    torch.cuda.synchronize()
    for i in range(0, len(reds), 17):
        kind, x, y = reds[i]
        got = b.results[i].item()
        if kind == "asum":
            assert rel(got, o_asum(x)) <= 1e-5, i
        else:
            r, mass = o_dot(x, y)
            assert abs(got - r) <= 1e-5 * mass, i
    for j in range(0, len(gemvs), 23):
        A, x, y = gemvs[j]
        r, mass = o_gemv(1.0, A, x, 0.5, y)
        g = gd[j][5].cpu().numpy().astype(np.float64)
        assert float(np.max(np.abs(g - r) / mass)) <= 1e-5, j
    b.close()
