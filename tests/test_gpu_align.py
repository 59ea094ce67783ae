"""Operands and outputs whose base pointer is not 16-byte aligned (views that
start one element into their storage): every kernel family then takes its
element-wise load and store paths, which must give the same results."""
import numpy as np
import pytest
import torch

import oracle
import paper_2002_03258_amd as tsm
import seeded_inputs as si

from helpers import TOL, dev_matrix, err, host_matrix, to_np

pytestmark = pytest.mark.gpu

DTYPES = [torch.float64, torch.float32]


def shifted(rows, cols, dtype, dev, src=None):
    """A column-major rows x cols view starting one element into its storage
    (base pointer 4 or 8 bytes past a 16-byte boundary), holding `src`."""
    store = torch.full((cols, rows + 3), float("nan"), dtype=dtype, device=dev)
    view = store[:, 1:rows + 1].t()
    assert view.data_ptr() % 16 != 0
    if src is not None:
        view.copy_(src)
    return view


def _mat(seed, stream, rows, cols, dtype, dev, dist="uniform"):
    return shifted(rows, cols, dtype, dev, dev_matrix(seed, stream, rows, cols, dtype, dev, dist=dist))


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("fn,m,k,n", [("tsm2r", 3001, 2500, 16), ("tsm2r", 777, 9000, 5),
                                      ("tsm2l", 50001, 16, 16), ("tsm2l", 4099, 9, 30),
                                      ("gemm", 2000, 40, 33)])
def test_products_misaligned(dev, dtype, fn, m, k, n):
    seed = 2000 + m + k + n
    A = _mat(seed, si.STREAM_A, m, k, dtype, dev)
    B = _mat(seed, si.STREAM_B, k, n, dtype, dev)
    C = shifted(m, n, dtype, dev)
    getattr(tsm, fn)(A, B, out=C)
    ref = oracle.matmul(host_matrix(seed, si.STREAM_A, m, k, dtype),
                        host_matrix(seed, si.STREAM_B, k, n, dtype))
    assert err(to_np(C), ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
def test_rowmajor_a_misaligned(dev, dtype):
    m, k, n = 1500, 3000, 8
    src = dev_matrix(7, si.STREAM_A, m, k, dtype, dev)
    store = torch.empty((m, k + 2), dtype=dtype, device=dev)
    A = store[:, 1:k + 1]                       # row-major, misaligned
    A.copy_(src)
    B = _mat(7, si.STREAM_B, k, n, dtype, dev)
    C = tsm.tsm2r(A, B)
    ref = oracle.matmul(host_matrix(7, si.STREAM_A, m, k, dtype),
                        host_matrix(7, si.STREAM_B, k, n, dtype))
    assert err(to_np(C), ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("m,k,n", [(3001, 3000, 8), (40001, 16, 16), (5000, 33, 20)])
def test_gradients_misaligned(dev, dtype, m, k, n):
    seed = 2100 + m + k + n
    A = _mat(seed, si.STREAM_A, m, k, dtype, dev)
    B = _mat(seed, si.STREAM_B, k, n, dtype, dev)
    dC = _mat(seed, si.STREAM_DC, m, n, dtype, dev, dist="normal")
    dA = shifted(m, k, dtype, dev)
    dB = shifted(k, n, dtype, dev)
    tsm.grad_a(dC, B, out=dA)
    tsm.grad_b(A, dC, out=dB)
    rA, rB = oracle.grad(host_matrix(seed, si.STREAM_A, m, k, dtype),
                         host_matrix(seed, si.STREAM_B, k, n, dtype),
                         host_matrix(seed, si.STREAM_DC, m, n, dtype, dist="normal"))
    assert err(to_np(dA), rA) <= TOL[dtype]
    assert err(to_np(dB), rB) <= TOL[dtype]
    if k <= 32 and n <= 32:
        fA, fB = tsm.tsm2l_backward(A, B, dC)
        assert err(to_np(fA), rA) <= TOL[dtype]
        assert err(to_np(fB), rB) <= TOL[dtype]


@pytest.mark.parametrize("fn,m,k,n", [("tsm2r", 3001, 2500, 16), ("tsm2l", 50001, 16, 16)])
def test_lowp_misaligned_b_and_c(dev, fn, m, k, n):
    seed = 2200 + m + k + n
    A = dev_matrix(seed, si.STREAM_A, m, k, torch.float32, dev)
    S = tsm.split(A, "bf16", lo=True)
    B = _mat(seed, si.STREAM_B, k, n, torch.float32, dev)
    C = shifted(m, n, torch.float32, dev)
    getattr(tsm, fn)(S, B, out=C)
    hi, lo = oracle.split(np.asfortranarray(host_matrix(seed, si.STREAM_A, m, k,
                                                        torch.float32).astype(np.float32)),
                          oracle.BF16)
    stored = oracle.decode_plane(hi, oracle.BF16) + oracle.decode_plane(lo, oracle.BF16)
    ref = oracle.matmul(stored, host_matrix(seed, si.STREAM_B, k, n, torch.float32))
    assert err(to_np(C), ref) <= 1e-5
