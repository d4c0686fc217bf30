"""Helpers shared by the GPU tests: seeded device inputs and bit views."""

import numpy as np
import torch

import bsgen

SEED = bsgen.DEFAULT_SEED
F64 = torch.float64


def dev_uniform(n, stream, seed=SEED, lo=-1.0, dtype=F64, pad=0, offset=0):
    """Device vector of n seeded values (optionally inside a larger buffer,
    starting `offset` elements in, to test unaligned pointers)."""
    buf = torch.zeros(n + pad + offset, dtype=dtype, device="cuda")
    t = buf[offset:offset + n]
    if n:
        bsgen.device_uniform(t, seed, stream, lo=lo)
    return t


def host_uniform(n, stream, seed=SEED, lo=-1.0):
    return bsgen.uniform(seed, stream, n, lo=lo)


def bits(a):
    a = np.ascontiguousarray(a)
    return a.view(np.uint64) if a.dtype == np.float64 else a.view(np.uint32 if a.itemsize == 4 else np.uint16)


def to_host(t):
    torch.cuda.synchronize()
    if t.dtype == torch.bfloat16:
        return t.view(torch.int16).cpu().numpy().view(np.uint16)
    return t.cpu().numpy()


def scalar_out():
    return torch.full((1,), float("nan"), dtype=F64, device="cuda")


def rel_err(got, ref):
    if ref == 0.0:
        return abs(got)
    return abs(got - ref) / abs(ref)
