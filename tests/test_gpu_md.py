"""GPU parity of MD (Fig. 7): forces from neighbour lists, Lennard-Jones.

Both sides take the cutoff decision in binary32 the same way, so the set of
interacting pairs is identical; the forces are then held to 1e-5 of the
magnitude of their terms, per particle and component (sum over the
interacting neighbours of |repulsive| + |attractive| times |d|: the sum of
the forces cancels, so a plain relative error is unbounded).
"""
import numpy as np
import pytest
import torch

import paper_1502_02389_amd as L
import workloads as W
from tests.gpu_util import banner

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
BAR = 1e-5


def check(got, pos, nbr, params):
    import oracle

    ref, mass = oracle.md(pos.numpy(), nbr.numpy(), *params, with_mass=True)
    g = got.cpu().numpy().astype(np.float64)
    assert np.all(g[:, 3] == 0.0)
    err = np.abs(g[:, :3] - ref)
    bad = err > BAR * mass + 1e-30
    assert not bad.any(), (int(bad.sum()), float((err / np.maximum(mass, 1e-30)).max()))
    return ref


def test_paper_size_system(gpu_device):
    pos, nbr, params = W.md_system()
    banner("md 12288 particles", nbr.shape)
    f = L.md(pos.to(DEV), nbr.to(DEV), *params)
    ref = check(f, pos, nbr, params)
    # the lists are symmetric, so the forces sum to ~0 (Newton's third law)
    tot = f.cpu().double()[:, :3].sum(0)
    assert float(tot.abs().max()) <= 1e-5 * float(np.abs(ref).sum())


KNOBS = [dict(lanes_per_item=l, vec_bytes=v, unroll=u, block=b)
         for l, v, u, b in [(1, 4, 1, 64), (1, 16, 4, 256), (2, 8, 2, 128), (4, 16, 1, 1024), (8, 16, 2, 256),
                            (8, 4, 4, 512), (16, 16, 4, 256), (16, 8, 1, 64), (4, 4, 2, 256)]]


@pytest.mark.parametrize("kn", KNOBS, ids=[str(i) for i in range(len(KNOBS))])
def test_every_knob_point_and_list_shapes(gpu_device, kn):
    pos, nbr, params = W.md_system(box=(9, 7, 11), slots=96, seed=71)
    n = pos.shape[0]
    pd = pos.to(DEV)
    for k in (96, 37, 1, 0):     # 37: odd length (one index per load), 0: no neighbours
        sub = nbr[:, :k].contiguous()
        banner("md knobs", kn, "k", k)
        out = torch.empty((n, 4), device=DEV)
        st = L.lift_md_ex(n, pd.data_ptr(), k, sub.to(DEV).data_ptr() if k else 0, *params, out.data_ptr(),
                          L.knobs(**kn), torch.cuda.current_stream().cuda_stream)
        assert st == L.LIFT_OK
        check(out, pos, sub, params)
    # lists starting 4 bytes past a 16-byte boundary
    buf = torch.empty(n * 96 + 1, dtype=torch.int32, device=DEV)
    view = buf[1:].view(n, 96)
    view.copy_(nbr.to(DEV))
    out = torch.empty((n, 4), device=DEV)
    assert L.lift_md_ex(n, pd.data_ptr(), 96, view.data_ptr(), *params, out.data_ptr(), L.knobs(**kn),
                        torch.cuda.current_stream().cuda_stream) == L.LIFT_OK
    check(out, pos, nbr, params)


def test_empty_slots_and_degenerate_sizes(gpu_device):
    pos, nbr, params = W.md_system(box=(5, 5, 5), slots=64, seed=72)
    n = pos.shape[0]
    junk = nbr.clone()
    junk[:, ::5] = -1
    junk[:, 1::7] = n
    junk[:, 2::11] = 2 ** 31 - 1
    junk[:, 3::13] = -(2 ** 31)
    banner("md empty slots")
    check(L.md(pos.to(DEV), junk.to(DEV), *params), pos, junk, params)
    one = torch.tensor([[0.5, 0.5, 0.5, 0.0]])
    lone = torch.tensor([[-1, 1, 5]], dtype=torch.int32)
    f = L.md(one.to(DEV), lone.to(DEV), *params)
    assert torch.equal(f.cpu(), torch.zeros(1, 4))
    assert L.md(torch.zeros((0, 4), device=DEV), torch.zeros((0, 8), dtype=torch.int32, device=DEV),
                *params).shape == (0, 4)


def test_cutoff_boundary_decided_like_the_oracle(gpu_device):
    # pairs placed exactly at and just inside the cutoff
    t = 1.25
    pos = torch.zeros((4, 4))
    pos[1, 0] = t
    pos[3, 0] = float(np.nextafter(np.float32(t), np.float32(0)))
    pos[2, 1] = 3.0
    pos[3, 1] = 3.0
    nbr = torch.tensor([[1], [0], [3], [2]], dtype=torch.int32)
    banner("md cutoff boundary")
    f = L.md(pos.to(DEV), nbr.to(DEV), t, 1.0, 1.0).cpu()
    assert torch.all(f[:2] == 0)
    assert torch.all(f[2:, 0] != 0)
    check(f, pos, nbr, (t, 1.0, 1.0))


def test_bitwise_deterministic(gpu_device):
    pos, nbr, params = W.md_system()
    pd, nd = pos.to(DEV), nbr.to(DEV)
    a = L.md(pd, nd, *params)
    for _ in range(5):
        assert torch.equal(L.md(pd, nd, *params), a)


def _md_plain(pos, nbr, params):
    """Forces through the plain entry point (the library's own launch): the
    call the benchmark times."""
    pd, nd = pos.to(DEV), nbr.to(DEV)
    out = torch.empty((pos.shape[0], 4), dtype=torch.float32, device=DEV)
    assert L.lift_md(pos.shape[0], pd.data_ptr(), nbr.shape[1], nd.data_ptr(), *params, out.data_ptr(),
                     torch.cuda.current_stream().cuda_stream) == 0
    return out


def test_paper_size_system_library_default_launch(gpu_device):
    pos, nbr, params = W.md_system()
    banner("md 12288 particles, library default launch")
    check(_md_plain(pos, nbr, params), pos, nbr, params)


@pytest.mark.parametrize("launch,shuffle", [("tuned", True), ("library default", True), ("library default", False)])
def test_large_system_sampled(gpu_device, launch, shuffle):
    import oracle

    pos, nbr, params = W.md_system(W.MD_BOX_LARGE, shuffle=shuffle)
    banner("md 2^20 particles", launch, "random order" if shuffle else "lattice order")
    if launch == "tuned":
        f = L.md(pos.to(DEV), nbr.to(DEV), *params)
    else:
        f = _md_plain(pos, nbr, params)
    f = f.cpu().numpy().astype(np.float64)
    ref, mass = oracle.md(pos.numpy(), nbr.numpy(), *params, with_mass=True)
    err = np.abs(f[:, :3] - ref)
    assert np.all(err <= BAR * mass + 1e-30)
