"""The straight-line paths that keep the next chunk's loads in flight (float
TSM2R and dB for n > 16, the 16-bit TSM2R and dB): they add the same
products in the same order as the general loops, so the results are equal
bit for bit with the path switched off (the TSM2X_*_PF and TSM2X_LP_RS
measurement overrides, read at call time), and they match the FP64 oracle.
Shapes are chosen so that most wavefronts take the straight-line path (full
tiles, k ranges a whole number of chunks) and a ragged tail takes the other."""
import numpy as np
import pytest
import torch

import oracle
import paper_2002_03258_amd as tsm
import seeded_inputs as si

from helpers import TOL, dev_matrix, err, host_matrix, to_np

pytestmark = pytest.mark.gpu

DTYPES = [torch.float64, torch.float32]


def _both(monkeypatch, var, values, fn):
    out = []
    for v in values:
        monkeypatch.setenv(var, str(v))
        out.append(fn().clone())
        torch.cuda.synchronize()
    monkeypatch.delenv(var)
    return out


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("m,k,n", [(4096, 8192, 32), (4096, 8192, 24), (2048, 16384, 4),
                                   (4100, 8200, 32)])
def test_tsm2r_in_flight_path(dev, monkeypatch, dtype, m, k, n):
    seed = 700 + n
    A = dev_matrix(seed, si.STREAM_A, m, k, dtype, dev)
    B = dev_matrix(seed, si.STREAM_B, k, n, dtype, dev)
    off, on = _both(monkeypatch, "TSM2X_NN_PF", (0, 1), lambda: tsm.tsm2r(A, B))
    assert torch.equal(off, on)
    ref = oracle.matmul(host_matrix(seed, si.STREAM_A, m, k, dtype),
                        host_matrix(seed, si.STREAM_B, k, n, dtype))
    assert err(to_np(on), ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
def test_tsm2r_in_flight_integer_exact(dev, monkeypatch, dtype):
    m, k, n = 4096, 4096, 32
    A = dev_matrix(5, si.STREAM_A, m, k, dtype, dev, dist="int", r=8)
    B = dev_matrix(5, si.STREAM_B, k, n, dtype, dev, dist="int", r=8)
    monkeypatch.setenv("TSM2X_NN_PF", "1")
    C = tsm.tsm2r(A, B)
    ref = oracle.matmul(host_matrix(5, si.STREAM_A, m, k, dtype, dist="int"),
                        host_matrix(5, si.STREAM_B, k, n, dtype, dist="int"))
    assert np.array_equal(to_np(C), ref)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("m,k,n", [(8192, 4096, 32), (8192, 4096, 17), (8200, 1000, 32)])
def test_grad_b_in_flight_path(dev, monkeypatch, dtype, m, k, n):
    """dB = A^T dC (A m x k, dC m x n): the reduction runs along m."""
    seed = 800 + n
    A = dev_matrix(seed, si.STREAM_A, m, k, dtype, dev)
    dC = dev_matrix(seed, si.STREAM_DC, m, n, dtype, dev)
    off, on = _both(monkeypatch, "TSM2X_TN_PF", (0, 1), lambda: tsm.grad_b(A, dC))
    assert torch.equal(off, on)
    ref = oracle.matmul(host_matrix(seed, si.STREAM_A, m, k, dtype).T,
                        host_matrix(seed, si.STREAM_DC, m, n, dtype))
    assert err(to_np(on), ref) <= TOL[dtype]


CODES = {"bf16": oracle.BF16, "f16": oracle.F16}


def _stored(A_np, fmt, lo):
    """hi (+ lo) of the oracle's split of A (float64 host values of a float32
    matrix): the values the 16-bit kernels multiply."""
    hi, lo_plane = oracle.split(np.asfortranarray(A_np.astype(np.float32)), CODES[fmt])
    v = oracle.decode_plane(hi, CODES[fmt])
    if lo:
        v = v + oracle.decode_plane(lo_plane, CODES[fmt])
    return v


@pytest.mark.parametrize("fmt", ["bf16", "f16"])
@pytest.mark.parametrize("lo", [False, True])
@pytest.mark.parametrize("m,k,n", [(4096, 8192, 8), (4096, 8192, 32), (4100, 8200, 16)])
def test_lowp_tsm2r_in_flight_path(dev, monkeypatch, fmt, lo, m, k, n):
    """The row-split kernel with and without the prefetch (same slices):
    equal bit for bit; against the oracle on the stored values."""
    seed = 900 + n
    A = dev_matrix(seed, si.STREAM_A, m, k, torch.float32, dev)
    B = dev_matrix(seed, si.STREAM_B, k, n, torch.float32, dev)
    S = tsm.split(A, fmt, lo=lo)
    monkeypatch.setenv("TSM2X_LP_S", "3")
    off, on = _both(monkeypatch, "TSM2X_LP_RS", (1, 2), lambda: tsm.tsm2r(S, B))
    assert torch.equal(off, on)
    monkeypatch.delenv("TSM2X_LP_S")
    Ah = host_matrix(seed, si.STREAM_A, m, k, torch.float32)
    ref = oracle.matmul(_stored(Ah, fmt, lo), host_matrix(seed, si.STREAM_B, k, n, torch.float32))
    assert err(to_np(on), ref) <= 3e-6


@pytest.mark.parametrize("lo", [False, True])
@pytest.mark.parametrize("m,k,n", [(8192, 4096, 8), (8192, 4096, 32), (8200, 1000, 24),
                                   (8200, 1000, 16)])
def test_lowp_grad_b_in_flight_path(dev, monkeypatch, lo, m, k, n):
    """The 16-bit matrix-core dB: one or two steps in flight (single form),
    four tiles per workgroup for n <= 16; (8200, 1000) leaves ragged rows and
    a ragged last column group to the bounds-checked step."""
    seed = 950 + n
    A = dev_matrix(seed, si.STREAM_A, m, k, torch.float32, dev)
    dC = dev_matrix(seed, si.STREAM_DC, m, n, torch.float32, dev)
    S = tsm.split(A, "bf16", lo=lo)
    off, on = _both(monkeypatch, "TSM2X_TN_PF", (0, 1), lambda: tsm.grad_b(S, dC))
    assert torch.equal(off, on)
    Ah = host_matrix(seed, si.STREAM_A, m, k, torch.float32)
    ref = oracle.matmul(_stored(Ah, "bf16", lo).T, host_matrix(seed, si.STREAM_DC, m, n, torch.float32))
    assert err(to_np(on), ref) <= 3e-6


def test_split_planes_of_wide_matrices_are_padded(dev):
    """Planes of a wide matrix whose column stride would be a multiple of
    1 KiB get 128 bytes more per column; the products on them are unchanged."""
    m, k, n = 2048, 2048, 8
    A = dev_matrix(3, si.STREAM_A, m, k, torch.float32, dev)
    S = tsm.split(A, "bf16", lo=True)
    assert S.ld == tsm.plane_ld(m, k) == m + 64
    assert S.hi.stride() == (1, m + 64)
    B = dev_matrix(3, si.STREAM_B, k, n, torch.float32, dev)
    Ah = host_matrix(3, si.STREAM_A, m, k, torch.float32)
    ref = oracle.matmul(_stored(Ah, "bf16", True), host_matrix(3, si.STREAM_B, k, n, torch.float32))
    assert err(to_np(tsm.tsm2r(S, B)), ref) <= 3e-6
