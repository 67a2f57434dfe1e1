"""Per-call entry points captured into one HIP graph and replayed.

The calls enqueue kernels only (no allocation, host copy or memset inside a
call), and asum / dot leave their workspace counters at zero when they end,
so a captured sequence of scal, asum, dot, gemv, BlackScholes and MD replays
to the same bits as the same calls made eagerly.  The replays are separated
by eager work on the same stream (inputs rewritten, other kernels run), and
every replay is compared with the eager results bit for bit: the kernels
combine their partial results in a fixed order, so equal inputs give equal
bits.  One eager result per operation is also held to the oracle, so the
graph is not merely consistent with itself.
"""
import numpy as np
import pytest
import torch

import paper_1502_02389_amd as L
import workloads as W
from tests.gpu_util import banner, o_asum, o_dot, rel

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
REPLAYS = 4


def _inputs():
    g = W.gen(700)
    n = (1 << 20) + 13
    x = W.normal(n, g)
    y = W.normal(n, g)
    xh = W.normal(n, g, "bf16")
    yh = W.normal(n, g, "bf16")
    A = W.normal((513, 5000), g)
    Ah = W.normal((300, 9000), g, "bf16")
    gx = W.normal(5000, g)
    gxh = W.normal(9000, g)
    gy = W.normal(513, g)
    gyh = W.normal(300, g)
    s, bs = W.blackscholes_prices(100003, seed=8)
    pos, nbr, md = W.md_system(box=(12, 11, 10), seed=9)
    return dict(x=x, y=y, xh=xh, yh=yh, A=A, Ah=Ah, gx=gx, gxh=gxh, gy=gy, gyh=gyh, s=s, pos=pos, nbr=nbr), bs, md


def _program(d, gy, gyh, bs, md, outs):
    """The captured sequence; writes into preallocated `outs` where the
    operation has an output argument."""
    L.scal(1.5, d["x"], out=outs["scal"])
    ra = L.asum(d["x"])
    rd = L.dot(d["x"], d["y"])
    rdh = L.dot(d["xh"], d["yh"], acc="comp")
    L.gemv(0.75, d["A"], d["gx"], 0.5, gy)
    L.gemv(1.25, d["Ah"], d["gxh"], -0.5, gyh)
    L.blackscholes(d["s"], *bs, out=outs["bs"])
    L.md(d["pos"], d["nbr"], *md, out=outs["md"])
    return ra, rd, rdh


def test_graph_replays_match_eager(gpu_device):
    h, bs, md = _inputs()
    s = torch.cuda.Stream(device=DEV)
    with torch.cuda.stream(s):
        d = {k: v.to(DEV) for k, v in h.items()}
        outs = {"scal": torch.empty_like(d["x"]),
                "bs": torch.empty((d["s"].numel(), 2), dtype=torch.float32, device=DEV),
                "md": torch.empty((d["pos"].shape[0], 4), dtype=torch.float32, device=DEV)}
        gy, gyh = d["gy"].clone(), d["gyh"].clone()

        banner("graph: eager pass")
        ra, rd, rdh = _program(d, gy, gyh, bs, md, outs)
        eager = {"asum": ra.clone(), "dot": rd.clone(), "doth": rdh.clone(), "gemv": gy.clone(),
                 "gemvh": gyh.clone(), "scal": outs["scal"].clone(), "bs": outs["bs"].clone(),
                 "md": outs["md"].clone()}
        s.synchronize()

    # the eager pass against the oracle (the kernels' own parity tests cover
    # every form; this keeps the comparison below anchored)
    assert rel(eager["asum"].item(), o_asum(h["x"])) <= 1e-5
    r, mass = o_dot(h["x"], h["y"])
    assert abs(eager["dot"].item() - r) <= 1e-5 * mass
    r, mass = o_dot(h["xh"], h["yh"])
    assert abs(eager["doth"].item() - r) <= 1e-6 * mass
    assert torch.equal(eager["scal"].cpu(), h["x"] * 1.5)

    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        gy.copy_(d["gy"])
        gyh.copy_(d["gyh"])
        s.synchronize()
        banner("graph: capture")
        with torch.cuda.graph(graph, stream=s):
            ra, rd, rdh = _program(d, gy, gyh, bs, md, outs)
        s.synchronize()

    for rep in range(REPLAYS):
        banner("graph: replay", rep)
        with torch.cuda.stream(s):
            # eager work between replays: reset the in-place gemv operands,
            # scribble over the outputs, run unrelated kernels
            gy.copy_(d["gy"])
            gyh.copy_(d["gyh"])
            for t in (outs["scal"], outs["bs"], outs["md"], ra, rd, rdh):
                t.fill_(float("nan"))
            junk = (d["x"] * 2.0).sum()
            graph.replay()
            s.synchronize()
        assert torch.isfinite(junk).item()
        got = {"asum": ra, "dot": rd, "doth": rdh, "gemv": gy, "gemvh": gyh, "scal": outs["scal"],
               "bs": outs["bs"], "md": outs["md"]}
        for k, v in eager.items():
            assert torch.equal(got[k], v), (rep, k)
    graph.reset()


def test_graph_replays_follow_new_inputs(gpu_device):
    """A replay reads the inputs' current contents: rewrite x in place and
    the captured asum reports the new sum."""
    n = (1 << 18) + 5
    s = torch.cuda.Stream(device=DEV)
    with torch.cuda.stream(s):
        x = torch.ones(n, device=DEV)
        L.asum(x)                    # the stream's workspace exists before capture
        s.synchronize()
        graph = torch.cuda.CUDAGraph()
        banner("graph: capture asum")
        with torch.cuda.graph(graph, stream=s):
            r = L.asum(x)
        for k in (1, 2, 3):
            x.fill_(float(k))
            graph.replay()
            s.synchronize()
            assert r.item() == float(k * n), (k, r.item())
        x.copy_(torch.arange(n, dtype=torch.float32, device=DEV) % 7)
        graph.replay()
        s.synchronize()
        ref = float(np.sum(np.arange(n) % 7))
        assert r.item() == ref
    graph.reset()
