"""ABFT checksums (the checksum-encoding use of TSM2R named in the paper's
introduction) on the library's kernels: encoding against the FP64 oracle,
no false alarm on a correct product, detection, location and correction of
planted single-element errors."""
import numpy as np
import pytest
import torch

import oracle
import paper_2002_03258_amd as tsm
from paper_2002_03258_amd import abft
import seeded_inputs as si

from helpers import dev_matrix, host_matrix, to_np

pytestmark = pytest.mark.gpu

DTYPES = [torch.float64, torch.float32]


@pytest.mark.parametrize("dtype", DTYPES)
def test_encode_integer_exact(dev, dtype):
    X = dev_matrix(31, si.STREAM_A, 5000, 3000, dtype, dev, dist="int", r=8)
    Xh = host_matrix(31, si.STREAM_A, 5000, 3000, dtype, dist="int", r=8)
    W = np.stack([np.ones(3000), np.arange(1, 3001)], axis=1)
    assert np.array_equal(to_np(abft.encode(X)), oracle.matmul(Xh, W))


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("m,k,n", [(4000, 3000, 16), (200000, 16, 16), (3000, 5000, 40)])
def test_clean_product_passes(dev, dtype, m, k, n):
    A = dev_matrix(32, si.STREAM_A, m, k, dtype, dev)
    B = dev_matrix(32, si.STREAM_B, k, n, dtype, dev)
    C = tsm.gemm(A, B)
    bad, res, tol = abft.verify(A, B, C)
    assert bad.numel() == 0
    assert (res.abs() <= tol).all()


@pytest.mark.parametrize("dtype", DTYPES)
def test_planted_errors_located_and_corrected(dev, dtype):
    m, k, n = 6000, 4000, 16
    A = dev_matrix(33, si.STREAM_A, m, k, dtype, dev)
    B = dev_matrix(33, si.STREAM_B, k, n, dtype, dev)
    C = tsm.gemm(A, B)
    C0 = C.clone()
    _, _, tol = abft.verify(A, B, C)
    plants = [(17, 3, 1000.0), (2999, 0, -300.0), (5990, 15, 50.0)]   # in units of tol
    for i, p, f in plants:
        C[i, p] += f * tol[i, 0].item()
    bad, _, _ = abft.verify(A, B, C)
    assert sorted(bad.tolist()) == [17, 2999, 5990]
    fixed = abft.correct(A, B, C)
    assert sorted((i, p) for i, p, _ in fixed) == [(17, 3), (2999, 0), (5990, 15)]
    assert abft.verify(A, B, C)[0].numel() == 0
    # the corrected elements are back within the checksum tolerance
    for i, p, _ in plants:
        assert abs(C[i, p].item() - C0[i, p].item()) <= 2 * tol[i, 0].item()
    others = torch.ones_like(C, dtype=torch.bool)
    for i, p, _ in plants:
        others[i, p] = False
    assert torch.equal(C[others], C0[others])
