"""Seeded synthetic inputs for the paper's linear-algebra workloads.

Shared by the tests, the smoke check and the benchmark; it draws random
numbers and converts storage types, and holds none of the arithmetic of the
operations themselves (neither the GPU library nor the oracle is imported).

Every array is generated on the CPU with ``torch.Generator('cpu')`` so the
oracle and the GPU see identical bits; callers copy to the device.

Recipes (Section 7.2 of the paper fixes the sizes: 16M and 128M-element
vectors, a 4096x4096 matrix with a 4096-vector, and an 8192x16384 matrix):

* uniform  : ``torch.rand(n) * 2 - 1`` in float32 -- exact multiples of 2^-24
             in [-1, 1)
* normal   : ``torch.randn``; draw order A, then x, then y
* integer  : ``torch.randint(lo, hi + 1).float()`` -- integer-valued floats
* bf16/f16 : float32 values as above, then ``.to(dtype)`` (round to nearest even)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import torch

STORAGE = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}


def gen(seed: int) -> torch.Generator:
    g = torch.Generator("cpu")
    g.manual_seed(seed)
    return g


def uniform(n: int, g: torch.Generator, storage: str = "f32") -> torch.Tensor:
    return (torch.rand(n, generator=g, dtype=torch.float32) * 2 - 1).to(STORAGE[storage])


def normal(shape, g: torch.Generator, storage: str = "f32") -> torch.Tensor:
    return torch.randn(shape, generator=g, dtype=torch.float32).to(STORAGE[storage])


def integers(shape, lo: int, hi: int, g: torch.Generator, storage: str = "f32") -> torch.Tensor:
    """Integer-valued floats uniform in [lo, hi] (inclusive)."""
    return torch.randint(lo, hi + 1, shape if isinstance(shape, tuple) else (shape,),
                         generator=g).to(torch.float32).to(STORAGE[storage])


# --------------------------------------------------------------------------
# the workloads: sizes and value recipes
# --------------------------------------------------------------------------

ASUM_SMALL_N = 1 << 20      # asum, single vector
STREAM_N = 1 << 24          # scal/asum/dot, 64 MiB per fp32 vector
LARGE_N = 1 << 27           # scal/asum/dot, 512 MiB per fp32 vector (the paper's 128M size)
STREAM_ALPHA = 2.5
GEMV_SIZES = (4096, 8192)   # square gemv
GEMV_ALPHA, GEMV_BETA = 1.0, 0.5
HALF_N = 1 << 26            # 16-bit storage asum/dot
HALF_GEMV = 16384           # bf16 A, square
BATCH_NRED, BATCH_NGEMV = 4096, 256
BS_N = 1 << 22              # BlackScholes: "4 million" stock prices
MD_BOX = (16, 16, 48)       # MD: 12288 particles
MD_BOX_LARGE = (128, 128, 64)   # 2^20 particles
MD_SLOTS = 128              # neighbour slots per particle
MD_CUTOFF, MD_EPSILON, MD_SIGMA = 2.5, 1.0, 1.0
BS_STRIKE, BS_RATE, BS_VOLATILITY, BS_YEARS = 20.0, 0.02, 0.30, 1.0


def asum_small_vector(integer: bool = False):
    """asum, n = 2^20, seed 0: uniform, or integers in [-8, 8]."""
    g = gen(0)
    if integer:
        return integers(ASUM_SMALL_N, -8, 8, g)
    return uniform(ASUM_SMALL_N, g)


def stream_vectors(n: int = STREAM_N):
    """scal/asum/dot vectors x then y, uniform, seed 1; alpha = 2.5."""
    g = gen(1)
    x = uniform(n, g)
    y = uniform(n, g)
    return x, y, STREAM_ALPHA


def gemv_square(size: int):
    """gemv operands A (size x size), x, y ~ normal(0, 1), seed 2."""
    g = gen(2)
    A = normal((size, size), g)
    x = normal(size, g)
    y = normal(size, g)
    return A, x, y, GEMV_ALPHA, GEMV_BETA


def gemv_rect(m: int, n: int):
    """gemv operands A (m x n), x (n), y (m) ~ normal(0, 1), seed 2, drawn in
    the order A, x, y; alpha 1, beta 0.5."""
    g = gen(2)
    A = normal((m, n), g)
    x = normal(n, g)
    y = normal(m, g)
    return A, x, y, GEMV_ALPHA, GEMV_BETA


def half_vectors(storage: str, n: int = HALF_N):
    """16-bit-stored x, y for asum/dot, uniform, seed 3."""
    g = gen(3)
    x = uniform(n, g, storage)
    y = uniform(n, g, storage)
    return x, y


def half_gemv(size: int = HALF_GEMV):
    """bf16-stored A with fp32 x, y ~ normal, seed 3; alpha 1, beta 0.5."""
    g = gen(3)
    A = normal((size, size), g, "bf16")
    x = normal(size, g)
    y = normal(size, g)
    return A, x, y, GEMV_ALPHA, GEMV_BETA


@dataclass
class BatchSpec:
    """Shapes of the batched workload: reductions then gemv problems."""

    red_kind: list = field(default_factory=list)   # "dot" or "asum"
    red_len: list = field(default_factory=list)
    gemv_mn: list = field(default_factory=list)    # (m, n)


def batch_shapes(n_red: int = BATCH_NRED, n_gemv: int = BATCH_NGEMV,
                 lo_exp: float = 8.0, hi_exp: float = 20.0,
                 mn_lo: int = 64, mn_hi: int = 4096, seed: int = 4) -> BatchSpec:
    """Reduction lengths floor(2^U(lo, hi)) (log-uniform), kinds alternating
    dot (even index) / asum (odd index); gemv M, N uniform in [mn_lo, mn_hi]."""
    g = gen(seed)
    u = torch.rand(n_red, generator=g, dtype=torch.float64) * (hi_exp - lo_exp) + lo_exp
    lens = [int(math.floor(2.0 ** float(e))) for e in u]
    kinds = ["dot" if i % 2 == 0 else "asum" for i in range(n_red)]
    mn = torch.randint(mn_lo, mn_hi + 1, (n_gemv, 2), generator=g)
    return BatchSpec(kinds, lens, [(int(a), int(b)) for a, b in mn])


def batch_values(spec: BatchSpec, storage: str = "f32", seed: int = 5):
    """Values for a batch: reductions uniform, gemv normal (A, x, y per problem)."""
    g = gen(seed)
    reds = []
    for kind, n in zip(spec.red_kind, spec.red_len):
        x = uniform(n, g, storage)
        y = uniform(n, g, storage) if kind == "dot" else None
        reds.append((kind, x, y))
    gemvs = []
    for m, n in spec.gemv_mn:
        A = normal((m, n), g, storage)
        x = normal(n, g)
        y = normal(m, g)
        gemvs.append((A, x, y))
    return reds, gemvs


def blackscholes_prices(n: int = BS_N, seed: int = 6):
    """Stock prices ~ U[5, 30) in fp32 (around the strike of 20: in, at and
    out of the money), seed 6; returns the prices and (strike, rate,
    volatility, years)."""
    g = gen(seed)
    s = torch.rand(n, generator=g, dtype=torch.float32) * 25 + 5
    return s, (BS_STRIKE, BS_RATE, BS_VOLATILITY, BS_YEARS)


def md_system(box=MD_BOX, slots: int = MD_SLOTS, spacing: float = 1.0, jitter: float = 0.1,
              rlist: float = 2.8, seed: int = 7, shuffle: bool = True):
    """Particles on a jittered cubic lattice (box = lattice points per axis,
    spacing 1, jitter U(-0.1, 0.1) per coordinate) with neighbour lists of
    every lattice point within rlist (a skin beyond the 2.5 cutoff), nearest
    first, padded with -1 to `slots`; particles at the faces have shorter
    lists.  With ``shuffle`` the particle order is a random permutation, so
    the gathers of neighbour positions are irregular.  Returns positions
    (n, 4) float32 (x, y, z, 0), neighbour indices (n, slots) int32 and
    (cutoff, epsilon, sigma)."""
    import numpy as np

    rng = np.random.default_rng(seed)
    nx, ny, nz = box
    n = nx * ny * nz
    c = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"), -1).reshape(-1, 3)
    r = int(math.ceil(rlist / spacing))
    o = np.stack(np.meshgrid(*[np.arange(-r, r + 1)] * 3, indexing="ij"), -1).reshape(-1, 3)
    d2 = (o * o).sum(1) * spacing * spacing
    keep = (d2 > 0) & (d2 <= rlist * rlist)
    o, d2 = o[keep], d2[keep]
    o = o[np.lexsort((o[:, 2], o[:, 1], o[:, 0], d2))][:slots]
    pos = np.zeros((n, 4), np.float32)
    pos[:, :3] = (c * spacing + rng.uniform(-jitter, jitter, (n, 3))).astype(np.float32)
    perm = rng.permutation(n).astype(np.int32) if shuffle else np.arange(n, dtype=np.int32)
    inv = np.empty(n, np.int64)                # perm: new index of old particle i
    inv[perm] = np.arange(n)
    cx, cy, cz = (c[inv, a].astype(np.int32) for a in range(3))   # lattice coords in the new order
    nbr = np.full((n, slots), -1, np.int32)
    for j, (ox, oy, oz) in enumerate(o):
        qx, qy, qz = cx + ox, cy + oy, cz + oz
        ok = (qx >= 0) & (qx < nx) & (qy >= 0) & (qy < ny) & (qz >= 0) & (qz < nz)
        old = (qx * ny + qy) * nz + qz
        nbr[:, j] = np.where(ok, perm[np.where(ok, old, 0)], -1)
    pos = pos[inv]
    return torch.from_numpy(np.ascontiguousarray(pos)), torch.from_numpy(np.ascontiguousarray(nbr)), \
        (MD_CUTOFF, MD_EPSILON, MD_SIGMA)
