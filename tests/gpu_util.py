"""Helpers for the GPU parity tests: CPU tensors -> oracle inputs, error
measures with the tolerances the tests state, and a case banner printed
before each GPU step so a failing run names its case."""
import sys

import numpy as np
import torch

import oracle


def banner(*parts):
    print("[case]", *parts, file=sys.stderr, flush=True)


def np_of(t: torch.Tensor):
    """numpy view of a CPU tensor and the oracle dtype tag (bf16 as bits)."""
    t = t.contiguous()
    if t.dtype == torch.bfloat16:
        return t.view(torch.int16).numpy().view(np.uint16), "bf16"
    return t.numpy(), None


def o_asum(x: torch.Tensor) -> float:
    a, dt = np_of(x)
    return oracle.asum(a, dtype=dt)


def o_dot(x: torch.Tensor, y: torch.Tensor):
    a, dt = np_of(x)
    b, _ = np_of(y)
    return oracle.dot(a, b, dtype=dt), oracle.dot_absmass(a, b, dtype=dt)


def o_gemv(alpha, A: torch.Tensor, x: torch.Tensor, beta, y: torch.Tensor, n=None):
    a, dt = np_of(A)
    xs = x.numpy()[: n if n is not None else x.numel()].copy()
    yy = y.numpy()
    out = oracle.gemv(alpha, a, xs, beta, yy, adtype=dt, lda=A.shape[1])
    mass = oracle.gemv_absmass(alpha, a, xs, beta, yy, adtype=dt, lda=A.shape[1])
    return out, mass


def rel(g: float, r: float) -> float:
    return abs(g - r) / abs(r) if r != 0 else abs(g)
