"""Shared helpers for the GPU tests: moving column-major matrices between numpy and the device."""
import sys

import numpy as np


def torch():
    import torch as t

    return t


def to_gpu(a):
    """numpy (any order) -> column-major float64 CUDA tensor with the same values."""
    t = torch()
    a = np.asfortranarray(np.asarray(a, dtype=np.float64))
    rows, cols = a.shape
    host = t.from_numpy(np.ascontiguousarray(a.T))  # (cols, rows) row-major == column-major (rows, cols)
    return host.to("cuda").t()


def to_np(x):
    """column-major (or any) CUDA tensor -> numpy float64 Fortran array."""
    return np.asfortranarray(x.detach().to("cpu").double().numpy())


def announce(*parts):
    """Name the case on stdout before a GPU step (a fault then names its case)."""
    print("[gpu-case]", *parts, flush=True)
    sys.stdout.flush()
