"""Helpers for the GPU parity tests (test code only)."""
import sys

import numpy as np
import pytest


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    return torch


def to_dev(a: np.ndarray):
    import torch
    return torch.from_numpy(np.array(a, copy=True, order="C")).to("cuda")


def bits(t):
    """uint64 bit patterns of a float64 array/tensor as numpy."""
    if not isinstance(t, np.ndarray):
        t = t.cpu().numpy()
    return np.ascontiguousarray(t).view(np.uint64)


def announce(*parts):
    sys.stdout.write("CASE " + " ".join(str(p) for p in parts) + "\n")
    sys.stdout.flush()


def multiset_hash_dev(t):
    """Order-independent hash of a device tensor's 8-byte elements: wrapping
    sums of two different mixes of each element's bits (torch on the device)."""
    import torch
    z = t.contiguous().view(torch.int64)
    h1 = z * -7046029254386353131          # 0x9E3779B97F4A7C15 as int64
    h1 = h1 ^ ((h1 >> 29) & ((1 << 35) - 1))
    h2 = (z ^ 0x5DEECE66D) * -4658895280553007687   # 0xBF58476D1CE4E5B9 as int64
    h2 = h2 ^ ((h2 >> 31) & ((1 << 33) - 1))
    return int(h1.sum().item()), int(h2.sum().item())
