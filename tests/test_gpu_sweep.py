"""A seeded sweep over random shapes and storage layouts of every entry point
against the FP64 oracle: products (tsm2r, tsm2l, gemm with transposed
operands and beta), the gradients and the fused backward, the 16-bit forms,
TSMTTSM and the K-means assignment.  The draws are fixed (one seed per case),
sized so the oracle finishes in well under a second per case."""
import numpy as np
import pytest
import torch

import oracle
import paper_2002_03258_amd as tsm
from paper_2002_03258_amd import kmeans
import seeded_inputs as si

from helpers import TOL, dev_matrix, err, host_matrix, to_np

pytestmark = pytest.mark.gpu

DT = [torch.float64, torch.float32]


def _shape(rng, kind):
    """(m, k, n) of a problem class: 'r' large k, 'l' small k, 'any'."""
    if kind == "r":
        return int(rng.integers(1, 3000)), int(rng.integers(33, 4000)), int(rng.integers(1, 80))
    if kind == "l":
        return int(rng.integers(1, 60000)), int(rng.integers(1, 33)), int(rng.integers(1, 40))
    return int(rng.integers(1, 5000)), int(rng.integers(1, 300)), int(rng.integers(1, 50))


def _maybe_rowmajor(x, flag):
    return x.contiguous() if flag else x


@pytest.mark.parametrize("case", range(60))
def test_products(dev, case):
    rng = np.random.default_rng(9000 + case)
    dtype = DT[case % 2]
    fn = ("tsm2r", "tsm2l", "gemm")[case % 3]
    m, k, n = _shape(rng, ("r", "l", "any")[(case // 3) % 3])
    rowA, rowB = bool(rng.integers(0, 2)), bool(rng.integers(0, 2))
    beta = float(rng.choice([0.0, 1.0, -0.5]))
    seed = 9100 + case
    A = _maybe_rowmajor(dev_matrix(seed, si.STREAM_A, m, k, dtype, dev), rowA)
    B = _maybe_rowmajor(dev_matrix(seed, si.STREAM_B, k, n, dtype, dev), rowB)
    C0 = dev_matrix(seed, si.STREAM_V, m, n, dtype, dev)
    C = getattr(tsm, fn)(A, B, out=C0.clone(), beta=beta)
    ref = oracle.matmul(host_matrix(seed, si.STREAM_A, m, k, dtype),
                        host_matrix(seed, si.STREAM_B, k, n, dtype))
    if beta != 0:
        ref = ref + beta * host_matrix(seed, si.STREAM_V, m, n, dtype)
    assert err(to_np(C), ref) <= TOL[dtype], (fn, m, k, n, rowA, rowB, beta)


@pytest.mark.parametrize("case", range(30))
def test_gradients(dev, case):
    rng = np.random.default_rng(9300 + case)
    dtype = DT[case % 2]
    m, k, n = _shape(rng, ("r", "l", "any")[(case // 2) % 3])
    n = min(n, 32)
    seed = 9400 + case
    A = dev_matrix(seed, si.STREAM_A, m, k, dtype, dev)
    B = dev_matrix(seed, si.STREAM_B, k, n, dtype, dev)
    dC = dev_matrix(seed, si.STREAM_DC, m, n, dtype, dev, dist="normal")
    rA, rB = oracle.grad(host_matrix(seed, si.STREAM_A, m, k, dtype),
                         host_matrix(seed, si.STREAM_B, k, n, dtype),
                         host_matrix(seed, si.STREAM_DC, m, n, dtype, dist="normal"))
    assert err(to_np(tsm.grad_a(dC, B)), rA) <= TOL[dtype], (m, k, n)
    assert err(to_np(tsm.grad_b(A, dC)), rB) <= TOL[dtype], (m, k, n)
    if k <= 32:
        fA, fB = tsm.tsm2l_backward(A, B, dC)
        assert err(to_np(fA), rA) <= TOL[dtype] and err(to_np(fB), rB) <= TOL[dtype], (m, k, n)


@pytest.mark.parametrize("case", range(30))
def test_lowp_forms(dev, case):
    rng = np.random.default_rng(9500 + case)
    fmt = ("bf16", "f16")[case % 2]
    code = oracle.BF16 if fmt == "bf16" else oracle.F16
    lo = bool((case // 2) % 2)
    fn = ("tsm2r", "tsm2l", "grad_b")[(case // 4) % 3]
    m, k, n = _shape(rng, ("r", "l", "any")[(case // 4) % 3])
    n = min(n, 32)
    seed = 9600 + case
    A = dev_matrix(seed, si.STREAM_A, m, k, torch.float32, dev)
    S = tsm.split(A, fmt, lo=lo)
    hi, lo_ = oracle.split(np.asfortranarray(host_matrix(seed, si.STREAM_A, m, k,
                                                         torch.float32).astype(np.float32)), code)
    stored = oracle.decode_plane(hi, code) + (oracle.decode_plane(lo_, code) if lo else 0)
    if fn == "grad_b":
        dC = dev_matrix(seed, si.STREAM_DC, m, n, torch.float32, dev, dist="normal")
        got = tsm.grad_b(S, dC)
        ref = oracle.matmul(stored.T, host_matrix(seed, si.STREAM_DC, m, n, torch.float32,
                                                  dist="normal"))
    else:
        B = dev_matrix(seed, si.STREAM_B, k, n, torch.float32, dev)
        got = getattr(tsm, fn)(S, B)
        ref = oracle.matmul(stored, host_matrix(seed, si.STREAM_B, k, n, torch.float32))
    assert err(to_np(got), ref) <= 1e-5, (fn, fmt, lo, m, k, n)


@pytest.mark.parametrize("case", range(16))
def test_tsmttsm_and_kmeans(dev, case):
    rng = np.random.default_rng(9700 + case)
    dtype = DT[case % 2]
    m = int(rng.integers(1, 200000))
    k, n = int(rng.integers(1, 70)), int(rng.integers(1, 70))
    seed = 9800 + case
    X = dev_matrix(seed, si.STREAM_A, m, k, dtype, dev, dist="int", r=4)
    Y = dev_matrix(seed, si.STREAM_B, m, n, dtype, dev, dist="int", r=4)
    Xh = host_matrix(seed, si.STREAM_A, m, k, dtype, dist="int", r=4)
    Yh = host_matrix(seed, si.STREAM_B, m, n, dtype, dist="int", r=4)
    if dtype == torch.float64 or m * 16 < (1 << 24):       # float sums stay exact
        assert np.array_equal(to_np(tsm.tsmttsm(X, Y)), oracle.matmul(np.ascontiguousarray(Xh.T), Yh))
    Mu = dev_matrix(seed, si.STREAM_V, k, n, dtype, dev, dist="int", r=4)
    Muh = host_matrix(seed, si.STREAM_V, k, n, dtype, dist="int", r=4)
    Xv = X.contiguous() if case % 4 >= 2 else X
    lab, dist = kmeans.assign(Xv, Mu.t())
    rlab, rdist = oracle.kmeans_assign(Xh, Muh)
    assert np.array_equal(lab.cpu().numpy(), rlab), (m, k, n)
    assert np.array_equal(dist.double().cpu().numpy(), rdist), (m, k, n)
