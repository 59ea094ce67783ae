"""Shared helpers of the GPU tests: seeded inputs on the device and the
matching host copies for the oracle."""
import numpy as np
import torch

import oracle
import seeded_inputs as si

TOL = {torch.float64: 1e-13, torch.float32: 1e-5}


def dev_matrix(seed, stream, rows, cols, dtype, dev, ld=None, dist="uniform", r=8):
    return si.matrix(seed, stream, rows, cols, ld=ld, dtype=dtype, device=dev, dist=dist, r=r)


def host_matrix(seed, stream, rows, cols, dtype, dist="uniform", r=8):
    """The same values as dev_matrix, on the CPU as float64 numpy (values
    rounded to `dtype` first)."""
    t = si.matrix(seed, stream, rows, cols, dtype=dtype, dist=dist, r=r)
    return t.to(torch.float64).numpy()


def host_rows(seed, stream, rows, cols, idx, dtype, dist="uniform"):
    t = si.matrix_rows(seed, stream, rows, cols, idx, dtype=dtype, dist=dist)
    return t.to(torch.float64).numpy()


def sample_rows(m, count=48, seed=0):
    rng = np.random.default_rng(seed)
    head = list(range(min(m, 8)))
    tail = list(range(max(0, m - 8), m))
    mid = rng.integers(0, m, size=max(0, count - 16)).tolist()
    return sorted(set(head + tail + mid))


def to_np(t):
    return t.detach().to(torch.float64).cpu().numpy()


def err(C, C_ref):
    return oracle.normwise_error(C, C_ref)
