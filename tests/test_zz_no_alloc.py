"""The allocation-free fused TSM2L backward (tsm2l_backward_noalloc): same
results as tsm2l_backward, bit for bit (same kernels, same grid, the dB
partials in the library's static scratch instead of a workspace), on two
calls in a row, the second smaller, and against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_2002_03258_amd as tsm
from paper_2002_03258_amd import _lib
import seeded_inputs as si

from helpers import dev_matrix, host_rows, sample_rows, to_np

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-13, torch.float32: 1e-5}


def _noalloc(A, B, dC, code, out_dt):
    m, k = A.shape
    n = B.shape[1]
    dA = tsm.empty_colmajor(m, k, out_dt, A.device)
    dB = tsm.empty_colmajor(k, n, out_dt, A.device)
    L = _lib.lib()
    rc = L.tsm2l_backward_noalloc(m, k, n, A.data_ptr(), max(1, A.stride(1)), B.data_ptr(), max(1, B.stride(1)),
            dC.data_ptr(), max(1, dC.stride(1)), dA.data_ptr(), max(1, dA.stride(1)),
            dB.data_ptr(), max(1, dB.stride(1)), code, torch.cuda.current_stream().cuda_stream)
    assert rc == 0, (rc, L.tsm2x_last_hip_error())
    return dA, dB


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_noalloc_backward_matches_the_workspace_form(dev, dt):
    seed = 0x5EED0042
    code = tsm.F64 if dt == torch.float64 else tsm.F32
    for m, k, n in ((3_000_001, 16, 16), (40_961, 32, 8)):       # the second call smaller
        A = dev_matrix(seed, si.STREAM_A, m, k, dt, dev)
        B = dev_matrix(seed, si.STREAM_B, k, n, dt, dev)
        dC = dev_matrix(seed, si.STREAM_DC, m, n, dt, dev, dist="normal")
        dA, dB = _noalloc(A, B, dC, code, dt)
        rA, rB = tsm.tsm2l_backward(A, B, dC)
        torch.cuda.synchronize()
        assert torch.equal(dA, rA) and torch.equal(dB, rB)
        rows = sample_rows(m, 24, seed=m)
        Ar = host_rows(seed, si.STREAM_A, m, k, rows, dt)
        Bh = to_np(B)
        dCr = host_rows(seed, si.STREAM_DC, m, n, rows, dt, dist="normal")
        assert oracle.normwise_error(to_np(dA[rows]), oracle.matmul(dCr, Bh.T)) <= TOL[dt]
        ref_b = oracle.matmul(np.ascontiguousarray(to_np(A).T), to_np(dC))
        assert oracle.normwise_error(to_np(dB), ref_b) <= TOL[dt]
        del A, B, dC, dA, dB, rA, rB
    torch.cuda.empty_cache()


def test_noalloc_backward_split_form(dev):
    seed = 0x5EED0043
    for m, k, n in ((1_000_003, 16, 16), (5_000, 8, 4)):
        A = dev_matrix(seed, si.STREAM_A, m, k, torch.float32, dev)
        S = tsm.split(A, "bf16", lo=True)
        B = dev_matrix(seed, si.STREAM_B, k, n, torch.float32, dev)
        dC = dev_matrix(seed, si.STREAM_DC, m, n, torch.float32, dev, dist="normal")
        planes = torch.as_strided(S.planes, (m, k), (1, S.ld))
        dA, dB = _noalloc(planes, B, dC, tsm.BF16_SPLIT, torch.float32)
        rA, rB = tsm.tsm2l_backward(S, B, dC)
        torch.cuda.synchronize()
        assert torch.equal(dA, rA) and torch.equal(dB, rB)


def test_noalloc_backward_argument_checks(dev):
    fn = _lib.lib().tsm2l_backward_noalloc
    assert fn(-1, 4, 4, None, 1, None, 4, None, 1, None, 1, None, 4, 0, None) == -1
    assert fn(10, 4, 4, 1, 5, 1, 4, 1, 10, 1, 10, 1, 4, 0, None) == -5
    # k > 32 is outside the kernel's range
    x = torch.zeros(64, dtype=torch.float64, device=dev)
    p = x.data_ptr()
    assert fn(1, 33, 1, p, 1, p, 33, p, 1, p, 1, p, 33, 0, None) == 1
