"""Parity of the HIP kernels with the FP64 oracle, through the C ABI.

Small shapes are compared in full (several tiles plus ragged tails, padded
leading dimensions filled with NaN, integer inputs bit-exact); the full-size
workloads are compared on sampled rows the oracle computes one by one."""
import numpy as np
import pytest
import torch

import oracle
import paper_2002_03258_amd as tsm
import seeded_inputs as si

from helpers import TOL, dev_matrix, err, host_matrix, host_rows, sample_rows, to_np

pytestmark = pytest.mark.gpu

DTYPES = [torch.float64, torch.float32]

SMALL_R = [(1, 1, 1), (7, 5, 3), (129, 257, 2), (300, 1000, 16), (1000, 3000, 32),
           (4133, 2500, 8), (255, 4097, 17), (64, 64, 4), (513, 9000, 1), (2048, 777, 12)]


def test_device_generator_matches_host(dev):
    for dist in ("uniform", "normal", "int"):
        d = si.matrix(9, si.STREAM_A, 1000, 37, device=dev, dist=dist).cpu()
        h = si.matrix(9, si.STREAM_A, 1000, 37, dist=dist)
        assert torch.equal(d, h)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("m,k,n", SMALL_R)
def test_tsm2r_small(dev, dtype, m, k, n):
    seed = 100 + m + k + n
    A = dev_matrix(seed, si.STREAM_A, m, k, dtype, dev)
    B = dev_matrix(seed, si.STREAM_B, k, n, dtype, dev)
    C = tsm.tsm2r(A, B)
    ref = oracle.matmul(host_matrix(seed, si.STREAM_A, m, k, dtype),
                        host_matrix(seed, si.STREAM_B, k, n, dtype))
    assert err(to_np(C), ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
def test_tsm2r_padded_ld_and_nan_padding(dev, dtype):
    m, k, n = 1000, 1500, 8
    A = dev_matrix(3, si.STREAM_A, m, k, dtype, dev, ld=1037)   # padding rows are NaN
    B = dev_matrix(3, si.STREAM_B, k, n, dtype, dev, ld=1501)
    Cs = torch.full((n, 1100), float("nan"), dtype=dtype, device=dev)
    C = Cs.t()[:m]
    tsm.tsm2r(A, B, out=C)
    ref = oracle.matmul(host_matrix(3, si.STREAM_A, m, k, dtype),
                        host_matrix(3, si.STREAM_B, k, n, dtype))
    assert err(to_np(C), ref) <= TOL[dtype]
    assert torch.isnan(Cs[:, m:]).all()          # rows past m untouched


@pytest.mark.parametrize("dtype", DTYPES)
def test_tsm2r_integer_inputs_bit_exact(dev, dtype):
    m, k, n = 3000, 1024, 16
    A = dev_matrix(4, si.STREAM_A, m, k, dtype, dev, dist="int", r=8)
    B = dev_matrix(4, si.STREAM_B, k, n, dtype, dev, dist="int", r=8)
    C = to_np(tsm.tsm2r(A, B))
    ref = oracle.matmul(host_matrix(4, si.STREAM_A, m, k, dtype, dist="int"),
                        host_matrix(4, si.STREAM_B, k, n, dtype, dist="int"))
    assert np.array_equal(C, ref)


@pytest.mark.parametrize("dtype", DTYPES)
def test_tsm2r_deterministic(dev, dtype):
    A = dev_matrix(5, si.STREAM_A, 5000, 20000, dtype, dev)
    B = dev_matrix(5, si.STREAM_B, 20000, 16, dtype, dev)
    C1 = tsm.tsm2r(A, B).clone()
    C2 = tsm.tsm2r(A, B)
    assert torch.equal(C1, C2)


@pytest.mark.parametrize("dtype", DTYPES)
def test_tsm2r_k_zero_and_closed_forms(dev, dtype):
    A = dev_matrix(6, si.STREAM_A, 300, 0, dtype, dev) if False else \
        torch.empty((0, 300), dtype=dtype, device=dev).t()
    B = torch.empty((4, 0), dtype=dtype, device=dev).t()
    C = tsm.tsm2r(A, B)
    assert torch.all(C == 0)
    # B = e_j picks column j exactly; B = ones gives row sums
    m, k = 777, 3000
    A = dev_matrix(6, si.STREAM_A, m, k, dtype, dev)
    E = torch.zeros((k, 4), dtype=dtype, device=dev)
    for p, j in enumerate([0, 5, 1234, k - 1]):
        E[j, p] = 1
    C = tsm.tsm2r(A, tsm.colmajor(E))
    assert torch.equal(C, A[:, [0, 5, 1234, k - 1]])


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("m,k,n", [(9, 70, 3), (33, 33, 17), (70, 9, 4), (1000, 777, 32)])
def test_tsm2r_rowmajor_small(dev, dtype, m, k, n):
    Arm = si.row_major(11, si.STREAM_A, m, k, dtype=dtype, device=dev)
    B = dev_matrix(11, si.STREAM_B, k, n, dtype, dev)
    C = tsm.tsm2r(Arm, B)
    ref = oracle.matmul(si.row_major(11, si.STREAM_A, m, k).to(dtype).double().numpy(),
                        host_matrix(11, si.STREAM_B, k, n, dtype))
    assert err(to_np(C), ref) <= TOL[dtype]


def test_tsm2r_rowmajor_config(dev):
    """A 1024 x 1024 row-major FP64 matrix times B 1024 x 4, checked in full."""
    seed = si.config_seed(0)
    m = k = 1024
    Arm = si.row_major(seed, si.STREAM_A, m, k, device=dev)
    B = dev_matrix(seed, si.STREAM_B, k, 4, torch.float64, dev)
    C = tsm.tsm2r(Arm, B)
    Ah = si.row_major(seed, si.STREAM_A, m, k).numpy()
    ref = oracle.matmul(Ah, host_matrix(seed, si.STREAM_B, k, 4, torch.float64))
    assert err(to_np(C), ref) <= 1e-13


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("m", [10240, 20480, 30720])
def test_tsm2r_full_size_sampled(dev, dtype, m):
    """Square A (m = k), n in {2, 4, 8, 16}: sampled rows against the oracle."""
    seed = si.config_seed(1)
    k = m
    A = dev_matrix(seed, si.STREAM_A, m, k, dtype, dev)
    rows = sample_rows(m, 40, seed=m)
    Arows = host_rows(seed, si.STREAM_A, m, k, rows, dtype)
    for n in (2, 4, 8, 16):
        B = dev_matrix(seed + n, si.STREAM_B, k, n, dtype, dev)
        C = tsm.tsm2r(A, B)
        Cs = to_np(C[rows])
        ref = oracle.matmul(Arows, host_matrix(seed + n, si.STREAM_B, k, n, dtype))
        e = err(Cs, ref)
        print("tsm2r", dtype, m, n, "err", e)
        assert e <= TOL[dtype], (m, n, e)
        del C, B
    del A
    torch.cuda.empty_cache()


# ------------------------------------------------------------------- TSM2L
SMALL_L = [(1, 1, 1), (100, 3, 5), (1000, 8, 8), (4099, 16, 16), (2500, 32, 32),
           (70000, 17, 9), (66000, 32, 1), (257, 1, 32)]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("m,k,n", SMALL_L)
def test_tsm2l_small(dev, dtype, m, k, n):
    seed = 200 + m + k + n
    A = dev_matrix(seed, si.STREAM_A, m, k, dtype, dev)
    B = dev_matrix(seed, si.STREAM_B, k, n, dtype, dev)
    C = tsm.tsm2l(A, B)
    ref = oracle.matmul(host_matrix(seed, si.STREAM_A, m, k, dtype),
                        host_matrix(seed, si.STREAM_B, k, n, dtype))
    assert err(to_np(C), ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
def test_tsm2l_identity_and_permutation_exact(dev, dtype):
    m, k = 100003, 16
    A = dev_matrix(7, si.STREAM_A, m, k, dtype, dev)
    I = torch.eye(k, dtype=dtype, device=dev)
    assert torch.equal(tsm.tsm2l(A, I), A)
    perm = torch.randperm(k, generator=torch.Generator().manual_seed(1))
    P = I[:, perm.to(dev)].contiguous()
    assert torch.equal(tsm.tsm2l(A, tsm.colmajor(P)), A[:, perm.to(dev)])
    assert torch.equal(tsm.tsm2l(A, tsm.colmajor(4 * I)), 4 * A)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("m", [1 << 20, 1 << 22, 1 << 24])
def test_tsm2l_full_size_sampled(dev, dtype, m):
    seed = si.config_seed(2)
    rows = sample_rows(m, 48, seed=m)
    for k in (8, 16, 32):
        A = dev_matrix(seed + k, si.STREAM_A, m, k, dtype, dev)
        B = dev_matrix(seed + k, si.STREAM_B, k, k, dtype, dev)
        C = tsm.tsm2l(A, B)
        ref = oracle.matmul(host_rows(seed + k, si.STREAM_A, m, k, rows, dtype),
                            host_matrix(seed + k, si.STREAM_B, k, k, dtype))
        e = err(to_np(C[rows]), ref)
        print("tsm2l", dtype, m, k, "err", e)
        assert e <= TOL[dtype], (m, k, e)
        del A, B, C
    torch.cuda.empty_cache()


# --------------------------------------------------------------- gradients
SMALL_G = [(1, 1, 1), (1000, 16, 16), (3000, 700, 8), (4097, 33, 5), (257, 2000, 32),
           (70001, 16, 16), (9, 70, 3), (9, 70, 17), (33, 33, 17), (15, 64, 1)]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("m,k,n", SMALL_G)
def test_grads_small(dev, dtype, m, k, n):
    seed = 300 + m + k + n
    A = dev_matrix(seed, si.STREAM_A, m, k, dtype, dev)
    B = dev_matrix(seed, si.STREAM_B, k, n, dtype, dev)
    dC = dev_matrix(seed, si.STREAM_DC, m, n, dtype, dev, dist="normal")
    dA = tsm.grad_a(dC, B)
    dB = tsm.grad_b(A, dC)
    rA, rB = oracle.grad(host_matrix(seed, si.STREAM_A, m, k, dtype),
                         host_matrix(seed, si.STREAM_B, k, n, dtype),
                         host_matrix(seed, si.STREAM_DC, m, n, dtype, dist="normal"))
    assert err(to_np(dA), rA) <= TOL[dtype]
    assert err(to_np(dB), rB) <= TOL[dtype]


# dA of TSM2R shapes (many output columns): column ranges split across
# workgroups, ragged rows and column ranges, padded (unaligned) leading
# dimensions
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("m,k,n,pad", [(1000, 300, 16, 0), (777, 129, 1, 0), (4099, 1000, 9, 3),
                                       (65, 65, 8, 1), (2048, 4096, 16, 0), (3, 700, 2, 0)])
def test_grad_a_rank_update(dev, dtype, m, k, n, pad):
    seed = 600 + m + k + n
    B = dev_matrix(seed, si.STREAM_B, k, n, dtype, dev, ld=k + pad)
    dC = dev_matrix(seed, si.STREAM_DC, m, n, dtype, dev, ld=m + pad, dist="normal")
    dA = tsm.grad_a(dC, B)
    rA = oracle.matmul(host_matrix(seed, si.STREAM_DC, m, n, dtype, dist="normal"),
                       host_matrix(seed, si.STREAM_B, k, n, dtype).T)
    assert err(to_np(dA), rA) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
def test_grad_a_rank_update_integer_exact(dev, dtype):
    m, k, n = 5000, 3000, 16
    B = dev_matrix(61, si.STREAM_B, k, n, dtype, dev, dist="int", r=8)
    dC = dev_matrix(61, si.STREAM_DC, m, n, dtype, dev, dist="int", r=8)
    ref = oracle.matmul(host_matrix(61, si.STREAM_DC, m, n, dtype, dist="int", r=8),
                        host_matrix(61, si.STREAM_B, k, n, dtype, dist="int", r=8).T)
    assert np.array_equal(to_np(tsm.grad_a(dC, B)), ref)


@pytest.mark.parametrize("dtype", DTYPES)
def test_shared_workspace_across_shapes(dev, dtype):
    """Calls of different shapes share the library workspace: a call with few
    row tiles followed by calls with more tiles (and a reduction along m) must
    all be right."""
    seq = [(600, 20000, 16), (5000, 20000, 16), (20000, 6000, 2), (1000, 30000, 4),
           (12000, 12000, 8)]
    for i, (m, k, n) in enumerate(seq):
        A = dev_matrix(40 + i, si.STREAM_A, m, k, dtype, dev)
        B = dev_matrix(40 + i, si.STREAM_B, k, n, dtype, dev)
        C = tsm.tsm2r(A, B)
        rows = sample_rows(m, 24, seed=i)
        ref = oracle.matmul(host_rows(40 + i, si.STREAM_A, m, k, rows, dtype),
                            host_matrix(40 + i, si.STREAM_B, k, n, dtype))
        assert err(to_np(C[rows]), ref) <= TOL[dtype], (m, k, n)
        dC = dev_matrix(40 + i, si.STREAM_DC, m, n, dtype, dev, dist="normal")
        dB = tsm.grad_b(A, dC)
        cols = sample_rows(k, 16, seed=i)
        Acols = si.matrix_cols(40 + i, si.STREAM_A, m, k, cols, dtype=dtype).double().numpy()
        dBref = oracle.matmul(Acols.T, host_matrix(40 + i, si.STREAM_DC, m, n, dtype,
                                                   dist="normal"))
        assert err(to_np(dB[cols]), dBref) <= TOL[dtype], ("grad_b", m, k, n)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("m,k,n", [(1, 1, 1), (1000, 16, 16), (70001, 16, 16), (4097, 33 - 1, 5),
                                   (2500, 7, 29), (66000, 32, 32), (300, 17, 3)])
def test_tsm2l_backward_fused(dev, dtype, m, k, n):
    seed = 600 + m + k + n
    A = dev_matrix(seed, si.STREAM_A, m, k, dtype, dev)
    B = dev_matrix(seed, si.STREAM_B, k, n, dtype, dev)
    dC = dev_matrix(seed, si.STREAM_DC, m, n, dtype, dev, dist="normal")
    dA, dB = tsm.tsm2l_backward(A, B, dC)
    rA, rB = oracle.grad(host_matrix(seed, si.STREAM_A, m, k, dtype),
                         host_matrix(seed, si.STREAM_B, k, n, dtype),
                         host_matrix(seed, si.STREAM_DC, m, n, dtype, dist="normal"))
    assert err(to_np(dA), rA) <= TOL[dtype]
    assert err(to_np(dB), rB) <= TOL[dtype]
    # same dA bits as the separate kernel (same products in the same order)
    assert torch.equal(dA, tsm.grad_a(dC, B))
    dA2, dB2 = tsm.tsm2l_backward(A, B, dC)
    assert torch.equal(dA, dA2) and torch.equal(dB, dB2)
