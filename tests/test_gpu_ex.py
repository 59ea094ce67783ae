"""The extended product forms C := beta*C + op(A)*op(B): beta, A and B given
transposed (row-major tensors), n > 32 in panels, TSM2L shapes with k > 32
and the shape-class dispatch of tsm2x_gemm, against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_2002_03258_amd as tsm
import seeded_inputs as si

from helpers import TOL, dev_matrix, err, host_matrix, to_np

pytestmark = pytest.mark.gpu

DTYPES = [torch.float64, torch.float32]
STREAM_C0 = si.STREAM_V


def _rowmajor(seed, stream, rows, cols, dtype, dev, dist="uniform", r=8):
    """The same values as dev_matrix, stored row-major (a contiguous tensor)."""
    return dev_matrix(seed, stream, rows, cols, dtype, dev, dist=dist, r=r).contiguous()


def _ref(Ah, Bh, C0h, beta):
    ref = oracle.matmul(Ah, Bh)
    return ref + beta * C0h.astype(np.float64) if beta != 0 else ref


CASES = [(1000, 3000, 16), (4097, 700, 5), (300, 20000, 8), (9, 70, 3), (2000, 16, 16),
         (70001, 8, 8), (129, 33, 32)]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("fn", ["tsm2r", "tsm2l", "gemm"])
@pytest.mark.parametrize("m,k,n", CASES)
@pytest.mark.parametrize("beta", [1.0, -0.5])
def test_beta_accumulates(dev, dtype, fn, m, k, n, beta):
    seed = 1100 + m + k + n
    A = dev_matrix(seed, si.STREAM_A, m, k, dtype, dev)
    B = dev_matrix(seed, si.STREAM_B, k, n, dtype, dev)
    C = dev_matrix(seed, STREAM_C0, m, n, dtype, dev)
    getattr(tsm, fn)(A, B, out=C, beta=beta)
    ref = _ref(host_matrix(seed, si.STREAM_A, m, k, dtype), host_matrix(seed, si.STREAM_B, k, n, dtype),
               host_matrix(seed, STREAM_C0, m, n, dtype), beta)
    assert err(to_np(C), ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("fn", ["tsm2r", "tsm2l"])
def test_beta_zero_does_not_read_c(dev, dtype, fn):
    m, k, n = 3000, 16, 16
    A = dev_matrix(5, si.STREAM_A, m, k, dtype, dev)
    B = dev_matrix(5, si.STREAM_B, k, n, dtype, dev)
    C = tsm.empty_colmajor(m, n, dtype, dev)
    C.fill_(float("nan"))
    getattr(tsm, fn)(A, B, out=C, beta=0.0)
    assert torch.isfinite(C).all()


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("fn", ["tsm2r", "tsm2l", "gemm"])
def test_beta_integer_bit_exact(dev, dtype, fn):
    for (m, k, n) in [(3000, 5000, 16), (5000, 16, 16)]:
        A = dev_matrix(9, si.STREAM_A, m, k, dtype, dev, dist="int", r=8)
        B = dev_matrix(9, si.STREAM_B, k, n, dtype, dev, dist="int", r=8)
        C = dev_matrix(9, STREAM_C0, m, n, dtype, dev, dist="int", r=64)
        getattr(tsm, fn)(A, B, out=C, beta=-2.0)
        ref = _ref(host_matrix(9, si.STREAM_A, m, k, dtype, dist="int", r=8),
                   host_matrix(9, si.STREAM_B, k, n, dtype, dist="int", r=8),
                   host_matrix(9, STREAM_C0, m, n, dtype, dist="int", r=64), -2.0)
        assert np.array_equal(to_np(C), ref)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("fn", ["tsm2r", "tsm2l", "gemm"])
@pytest.mark.parametrize("m,k,n", [(1000, 3000, 16), (4097, 700, 5), (2000, 16, 16), (65, 9, 31),
                                   (129, 33, 32)])
@pytest.mark.parametrize("rowA", [False, True])
def test_transposed_operands(dev, dtype, fn, m, k, n, rowA):
    """B (and A) as row-major tensors: passed as the transposes they store."""
    seed = 1300 + m + k + n
    A = _rowmajor(seed, si.STREAM_A, m, k, dtype, dev) if rowA else \
        dev_matrix(seed, si.STREAM_A, m, k, dtype, dev)
    B = _rowmajor(seed, si.STREAM_B, k, n, dtype, dev)
    C = getattr(tsm, fn)(A, B)
    ref = oracle.matmul(host_matrix(seed, si.STREAM_A, m, k, dtype),
                        host_matrix(seed, si.STREAM_B, k, n, dtype))
    assert err(to_np(C), ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("fn", ["tsm2r", "tsm2l", "gemm"])
@pytest.mark.parametrize("m,k,n", [(1000, 3000, 33), (300, 5000, 70), (20000, 16, 40),
                                   (777, 40, 64), (5000, 100, 3)])
def test_wide_b_and_deep_tsm2l(dev, dtype, fn, m, k, n):
    """n > 32 in panels of 32; TSM2L shapes with k > 32 on the TSM2R kernels."""
    seed = 1500 + m + k + n
    A = dev_matrix(seed, si.STREAM_A, m, k, dtype, dev)
    B = dev_matrix(seed, si.STREAM_B, k, n, dtype, dev)
    C = dev_matrix(seed, STREAM_C0, m, n, dtype, dev)
    getattr(tsm, fn)(A, B, out=C, beta=1.0)
    ref = _ref(host_matrix(seed, si.STREAM_A, m, k, dtype), host_matrix(seed, si.STREAM_B, k, n, dtype),
               host_matrix(seed, STREAM_C0, m, n, dtype), 1.0)
    assert err(to_np(C), ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
def test_empty_k_scales_c(dev, dtype):
    C = dev_matrix(3, STREAM_C0, 500, 7, dtype, dev)
    C0 = to_np(C).copy()
    A = torch.empty((500, 0), dtype=dtype, device=dev)
    B = torch.empty((0, 7), dtype=dtype, device=dev)
    tsm.tsm2r(A, B, out=C, beta=3.0)
    nd = np.float64 if dtype == torch.float64 else np.float32
    assert np.array_equal(to_np(C), (nd(3.0) * C0.astype(nd)).astype(np.float64))
    tsm.tsm2l(A, B, out=C, beta=0.0)
    assert not to_np(C).any()


@pytest.mark.parametrize("dtype", DTYPES)
def test_caller_workspace_transposed_b(dev, dtype):
    m, k, n = 3000, 20000, 16
    A = dev_matrix(21, si.STREAM_A, m, k, dtype, dev)
    B = _rowmajor(21, si.STREAM_B, k, n, dtype, dev)
    code = tsm.F64 if dtype == torch.float64 else tsm.F32
    nb = tsm.workspace_size(tsm.OP_TSM2R, m, k, n, code)
    assert nb > 0
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    C = tsm.tsm2r(A, B, workspace=ws)
    ref = oracle.matmul(host_matrix(21, si.STREAM_A, m, k, dtype),
                        host_matrix(21, si.STREAM_B, k, n, dtype))
    assert err(to_np(C), ref) <= TOL[dtype]
    # the size covers every plan of the shape: also that of an A whose
    # leading dimension rules out 16-byte loads (a different grid)
    A1 = dev_matrix(21, si.STREAM_A, m, k, dtype, dev, ld=m + 1)
    assert err(to_np(tsm.tsm2r(A1, B, workspace=ws)), ref) <= TOL[dtype]
    with pytest.raises(tsm.TSMError):
        tsm.tsm2r(A, B, workspace=ws[:256])


# the precision form: beta, a transposed B, TSM2L with k > 32, panels
TOL_LP = 1e-5


def _stored(Ah, code, lo):
    hi, lo_ = oracle.split(np.asfortranarray(Ah.astype(np.float32)), code)
    v = oracle.decode_plane(hi, code)
    return v + oracle.decode_plane(lo_, code) if lo else v


@pytest.mark.parametrize("fn", ["tsm2r", "tsm2l", "gemm"])
@pytest.mark.parametrize("m,k,n", [(2000, 3000, 16), (5000, 16, 16), (1000, 48, 40), (129, 8, 33)])
@pytest.mark.parametrize("lo", [False, True])
def test_lowp_beta_and_transposed_b(dev, fn, m, k, n, lo):
    seed = 1700 + m + k + n
    A = dev_matrix(seed, si.STREAM_A, m, k, torch.float32, dev)
    S = tsm.split(A, "bf16", lo=lo)
    B = _rowmajor(seed, si.STREAM_B, k, n, torch.float32, dev)
    C = dev_matrix(seed, STREAM_C0, m, n, torch.float32, dev)
    getattr(tsm, fn)(S, B, out=C, beta=0.75)
    Ah = host_matrix(seed, si.STREAM_A, m, k, torch.float32)
    ref = _ref(_stored(Ah, oracle.BF16, lo), host_matrix(seed, si.STREAM_B, k, n, torch.float32),
               host_matrix(seed, STREAM_C0, m, n, torch.float32), 0.75)
    assert err(to_np(C), ref) <= TOL_LP


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("m,k,n", [(1 << 20, 16, 16), (300001, 8, 40), (100003, 64, 8),
                                   (4097, 3, 1), (77, 20, 33)])
@pytest.mark.parametrize("beta", [0.0, 1.0])
def test_tsmttsm(dev, dtype, m, k, n, beta):
    seed = 2300 + m % 1000 + k + n
    A = dev_matrix(seed, si.STREAM_A, m, k, dtype, dev)
    B = dev_matrix(seed, si.STREAM_B, m, n, dtype, dev, dist="normal")
    C0 = dev_matrix(seed, STREAM_C0, k, n, dtype, dev)
    C = tsm.tsmttsm(A, B, out=C0.clone(), beta=beta)
    Ah = host_matrix(seed, si.STREAM_A, m, k, dtype)
    Bh = host_matrix(seed, si.STREAM_B, m, n, dtype, dist="normal")
    ref = _ref(np.ascontiguousarray(Ah.T), Bh, host_matrix(seed, STREAM_C0, k, n, dtype), beta)
    assert err(to_np(C), ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
def test_tsmttsm_integer_bit_exact_and_deterministic(dev, dtype):
    m, k, n = 500001, 16, 24
    A = dev_matrix(71, si.STREAM_A, m, k, dtype, dev, dist="int", r=2)
    B = dev_matrix(71, si.STREAM_B, m, n, dtype, dev, dist="int", r=2)
    C = tsm.tsmttsm(A, B)
    ref = oracle.matmul(np.ascontiguousarray(host_matrix(71, si.STREAM_A, m, k, dtype, dist="int",
                                                         r=2).T),
                        host_matrix(71, si.STREAM_B, m, n, dtype, dist="int", r=2))
    assert np.array_equal(to_np(C), ref)
    assert torch.equal(C, tsm.tsmttsm(A, B))


def test_tsmttsm_shape_check(dev):
    A = torch.zeros(10, 3, dtype=torch.float64, device=dev)
    with pytest.raises(ValueError):
        tsm.tsmttsm(A, torch.zeros(11, 2, dtype=torch.float64, device=dev))


def test_workspace_errors_leave_outputs_untouched(dev):
    """A caller workspace that is too small or not 256-byte aligned is refused
    (TSM_ERR_WORKSPACE = 3) before anything is launched."""
    from paper_2002_03258_amd import _lib
    L = _lib.lib()
    m, k, n = 2000, 8000, 16
    A = dev_matrix(81, si.STREAM_A, m, k, torch.float64, dev)
    B = dev_matrix(81, si.STREAM_B, k, n, torch.float64, dev)
    # the query covers a transposed B too; the split partials alone are
    # megabytes here (S > 1), so 256 bytes is too small for any form
    assert tsm.tsm2r_plan(m, k, n, tsm.F64)["slices"] > 1
    need = tsm.workspace_size(tsm.OP_TSM2R, m, k, n, tsm.F64)
    ws = torch.empty(need + 512, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream().cuda_stream
    for ptr, nbytes in ((ws.data_ptr(), 256), (ws.data_ptr() + 16, need)):
        C = torch.full((n, m), float("nan"), dtype=torch.float64, device=dev).t()
        rc = L.tsm2r_ex(0, 0, m, k, n, A.data_ptr(), m, B.data_ptr(), k, 0.0, C.data_ptr(), m,
                        tsm.F64, ptr, nbytes, stream)
        assert rc == 3
        torch.cuda.synchronize()
        assert torch.isnan(C).all()
    # dB and the K-means assignment likewise
    dC = dev_matrix(82, si.STREAM_DC, 100000, 8, torch.float64, dev)
    Ag = dev_matrix(82, si.STREAM_A, 100000, 3000, torch.float64, dev)
    gneed = tsm.workspace_size(tsm.OP_GRAD_B, 100000, 3000, 8, tsm.F64)
    dB = torch.full((8, 3000), float("nan"), dtype=torch.float64, device=dev).t()
    if gneed > 0:
        rc = L.tsm_grad_b(100000, 3000, 8, Ag.data_ptr(), 100000, dC.data_ptr(), 100000,
                          dB.data_ptr(), 3000, tsm.F64, ws.data_ptr() + 16, gneed, stream)
        assert rc == 3
    X = dev_matrix(83, si.STREAM_A, 1000, 16, torch.float64, dev)
    lab = torch.full((1000,), -7, dtype=torch.int32, device=dev)
    rc = L.tsm_kmeans_assign(1000, 16, 16, X.data_ptr(), 1000, 0, B.data_ptr(), k,
                             lab.data_ptr(), None, tsm.F64, ws.data_ptr() + 16, 4096, stream)
    assert rc == 3
    torch.cuda.synchronize()
    assert torch.isnan(dB).all() and (lab == -7).all()


@pytest.mark.parametrize("lo", [False, True])
@pytest.mark.parametrize("rowB", [False, True])
def test_caller_workspace_precision_form(dev, lo, rowB):
    """The precision form's workspace holds the split partials and B's packed
    terms; tsm2x_workspace_size covers both, with B in either order, and a
    workspace too small for them is refused before any launch."""
    m, k, n = 3000, 20000, 24
    A = dev_matrix(23, si.STREAM_A, m, k, torch.float32, dev)
    B = _rowmajor(23, si.STREAM_B, k, n, torch.float32, dev) if rowB else \
        dev_matrix(23, si.STREAM_B, k, n, torch.float32, dev)
    S = tsm.split(A, "bf16", lo=lo)
    nb = tsm.workspace_size(tsm.OP_TSM2R, m, k, n, S.dtype_code)
    assert nb > 0
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    C = tsm.tsm2r(S, B, workspace=ws)
    assert torch.equal(C, tsm.tsm2r(S, B))
    C2 = tsm.empty_colmajor(m, n, torch.float32, dev).fill_(7.0)
    with pytest.raises(tsm.TSMError):
        tsm.tsm2r(S, B, out=C2, workspace=ws[:256])
    torch.cuda.synchronize()
    assert bool((C2 == 7.0).all())


@pytest.mark.parametrize("lo", [False, True])
@pytest.mark.parametrize("n", [8, 24])
def test_caller_workspace_precision_form_grad_b(dev, lo, n):
    """dB on bfloat16 planes: for n > 16 the workspace holds dC's packed bf16
    terms after the slice partials; tsm2x_workspace_size covers them, the
    result with the caller's (256-byte aligned) workspace equals the library
    buffer's bit for bit, and a workspace too small is refused before any
    launch."""
    m, k = 8192, 4096
    A = dev_matrix(29, si.STREAM_A, m, k, torch.float32, dev)
    dC = dev_matrix(29, si.STREAM_DC, m, n, torch.float32, dev)
    S = tsm.split(A, "bf16", lo=lo)
    nb = tsm.workspace_size(tsm.OP_GRAD_B, m, k, n, S.dtype_code)
    if n > 16:
        assert nb >= (m // 32) * 2 * 3 * 64 * 16        # dC's packed terms
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev)
    dB = tsm.grad_b(S, dC, workspace=ws)
    assert torch.equal(dB, tsm.grad_b(S, dC))
    if nb > 0:
        dB2 = tsm.empty_colmajor(k, n, torch.float32, dev).fill_(7.0)
        with pytest.raises(tsm.TSMError):
            tsm.grad_b(S, dC, out=dB2, workspace=ws[:nb - 1])
        torch.cuda.synchronize()
        assert bool((dB2 == 7.0).all())
