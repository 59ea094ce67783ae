"""The C-ABI library loads, exports every function tsm2x.h declares, and
rejects invalid arguments on the host (no GPU calls are made)."""
import ctypes
import os
import re

import pytest

import paper_2002_03258_amd as tsm
from paper_2002_03258_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\**\s+\**([a-z_0-9]+)\s*\(",
                                    src, flags=re.M))
    return names


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    names = declared_functions()
    assert {"tsm2r", "tsm2l", "tsm2r_ex", "tsm_grad_a", "tsm_grad_b"} <= names
    for nme in names:
        assert hasattr(L, nme), nme
    assert set(_lib.EXPORTS) <= names


def test_version_and_error_strings():
    L = _lib.lib()
    assert L.tsm2x_version() >= 100
    for code in (0, 1, 2, 3, 4, -5, 99):
        assert len(L.tsm2x_error_string(code)) > 0


NULL = None
P = 4096  # a non-null dummy address: never dereferenced, validation fails first


@pytest.mark.parametrize("args,expect", [
    ((-1, 4, 4, P, 4, P, 4, P, 4, 0, NULL), -1),
    ((4, -1, 4, P, 4, P, 4, P, 4, 0, NULL), -2),
    ((4, 4, -1, P, 4, P, 4, P, 4, 0, NULL), -3),
    ((4, 4, 4, NULL, 4, P, 4, P, 4, 0, NULL), -4),
    ((4, 4, 4, P, 3, P, 4, P, 4, 0, NULL), -5),
    ((4, 4, 4, P, 4, NULL, 4, P, 4, 0, NULL), -6),
    ((4, 4, 4, P, 4, P, 3, P, 4, 0, NULL), -7),
    ((4, 4, 4, P, 4, P, 4, NULL, 4, 0, NULL), -8),
    ((4, 4, 4, P, 4, P, 4, P, 3, 0, NULL), -9),
    ((4, 4, 4, P, 4, P, 4, P, 4, 9, NULL), -10),
])
def test_tsm2r_argument_checks(args, expect):
    assert _lib.lib().tsm2r(*args) == expect


def test_tsm2l_checks():
    L = _lib.lib()
    assert L.tsm2l(8, 4, 4, P, 7, P, 4, P, 8, 0, NULL) == -5
    assert L.tsm2l(8, 4, 4, P, 8, P, 3, P, 8, 0, NULL) == -7


# extended forms: 1 transA, 2 transB, 3 m, 4 k, 5 n, 6 A, 7 lda, 8 B, 9 ldb,
# 10 beta, 11 C, 12 ldc, 13 dtype, 14 ws, 15 ws_bytes, 16 stream
EX_OK = [0, 0, 8, 16, 4, P, 8, P, 16, 0.0, P, 8, 0, NULL, 0, NULL]


@pytest.mark.parametrize("fn", ["tsm2r_ex", "tsm2l_ex", "tsm2x_gemm"])
@pytest.mark.parametrize("pos,bad,expect", [
    (0, 2, -1), (1, -1, -2), (2, -1, -3), (3, -1, -4), (4, -1, -5), (5, NULL, -6),
    (6, 7, -7), (7, NULL, -8), (8, 15, -9), (10, NULL, -11), (11, 7, -12), (12, 9, -13),
])
def test_extended_argument_checks(fn, pos, bad, expect):
    args = list(EX_OK)
    args[pos] = bad
    assert getattr(_lib.lib(), fn)(*args) == expect


@pytest.mark.parametrize("fn", ["tsm2r_ex", "tsm2l_ex", "tsm2x_gemm"])
def test_extended_transposed_leading_dimensions(fn):
    L = getattr(_lib.lib(), fn)
    # transA = 1: A is k x m, lda >= k; transB = 1: B is n x k, ldb >= n
    assert L(1, 0, 8, 16, 4, P, 15, P, 16, 0.0, P, 8, 0, NULL, 0, NULL) == -7
    assert L(0, 1, 8, 16, 4, P, 8, P, 3, 0.0, P, 8, 0, NULL, 0, NULL) == -9
    # a 16-bit form of A must not be transposed (valid arguments otherwise)
    assert L(1, 0, 8, 16, 4, P, 16, P, 16, 0.0, P, 8, 2, NULL, 0, NULL) == 1
    # empty products: no work, no GPU needed
    assert L(0, 0, 0, 16, 4, NULL, 1, P, 16, 1.0, NULL, 1, 0, NULL, 0, NULL) == 0
    assert L(0, 1, 8, 16, 0, P, 8, NULL, 1, 0.0, NULL, 8, 1, NULL, 0, NULL) == 0


def test_grad_argument_checks():
    L = _lib.lib()
    assert L.tsm_grad_a(8, 4, 4, P, 7, P, 4, P, 8, 0, NULL) == -5
    assert L.tsm_grad_a(8, 4, 4, P, 8, P, 3, P, 8, 0, NULL) == -7
    assert L.tsm_grad_b(8, 4, 4, P, 8, P, 8, P, 3, 0, NULL, 0, NULL) == -9
    assert L.tsm_grad_b(8, 4, 40, P, 8, P, 8, P, 4, 0, NULL, 0, NULL) == 1


def test_empty_problems_are_noops_without_gpu():
    L = _lib.lib()
    assert L.tsm2r(0, 4, 4, NULL, 1, P, 4, NULL, 1, 0, NULL) == 0
    assert L.tsm2r(4, 4, 0, P, 4, NULL, 4, NULL, 4, 0, NULL) == 0
    assert L.tsm2l(0, 4, 4, NULL, 1, P, 4, NULL, 1, 1, NULL) == 0
    assert L.tsm_grad_b(8, 0, 4, P, 8, P, 8, NULL, 1, 0, NULL, 0, NULL) == 0


def test_binding_refuses_cpu_tensors():
    import torch
    with pytest.raises(ValueError):
        tsm.tsm2r(torch.zeros(4, 4, dtype=torch.float64), torch.zeros(4, 2, dtype=torch.float64))


def test_fused_backward_argument_checks():
    L = _lib.lib()
    # m k n A lda B ldb dC lddc dA ldda dB lddb dtype ws wsb stream
    ok = [8, 4, 4, P, 8, P, 4, P, 8, P, 8, P, 4, 0, NULL, 0, NULL]
    for pos, bad in [(0, -1), (4, 7), (6, 3), (8, 7), (10, 7), (12, 3), (13, 9)]:
        args = list(ok)
        args[pos] = bad
        assert L.tsm2l_backward(*args) == -(pos + 1), pos
    args = list(ok)
    args[1] = 33
    args[6] = 33
    args[12] = 33
    assert L.tsm2l_backward(*args) == 1          # k > 32 unsupported
    args = list(ok)
    args[1] = 0
    assert L.tsm2l_backward(*args) == 0          # empty dA and dB: no-op


def test_split_argument_checks():
    L = _lib.lib()
    assert L.tsm2x_split(-1, 4, P, 4, P, P, 4, 0, NULL) == -1
    assert L.tsm2x_split(4, 4, P, 3, P, P, 4, 0, NULL) == -4
    assert L.tsm2x_split(4, 4, P, 4, P, P, 3, 0, NULL) == -7
    assert L.tsm2x_split(4, 4, P, 4, P, P, 4, 2, NULL) == -8
    assert L.tsm2x_split(0, 4, NULL, 1, NULL, NULL, 1, 0, NULL) == 0


def test_plane_leading_dimension():
    # 16-byte columns; 128 bytes more for wide matrices whose column stride
    # would be a multiple of 1 KiB; tall TSM2L-class planes are not padded
    assert tsm.plane_ld(16384, 16384) == 16384 + 64
    assert tsm.plane_ld(32768, 100) == 32768 + 64
    assert tsm.plane_ld(1 << 23, 16) == 1 << 23
    assert tsm.plane_ld(1 << 23, 32) == 1 << 23
    assert tsm.plane_ld(1000, 4096) == 1000
    assert tsm.plane_ld(1001, 4096) == 1008
    assert tsm.plane_ld(1, 64) == 8
    for m in (1, 7, 511, 512, 513, 30720, 32768):
        for k in (8, 33, 1024):
            ld = tsm.plane_ld(m, k)
            assert ld >= m and ld % 8 == 0 and ld - m < 8 + 64


def test_workspace_size_is_zero_without_split():
    L = _lib.lib()
    # no reduction split for tiny problems; an op outside the table needs none
    assert L.tsm2x_workspace_size(1, 1000, 16, 16, 0) == 0
    assert L.tsm2x_workspace_size(99, 1000, 1000, 16, 0) == 0


def test_kernel_name_query():
    import paper_2002_03258_amd as tsm
    for dt, tname in ((tsm.F64, "double"), (tsm.F32, "float")):
        for n in (1, 16, 17, 32):
            name = tsm.kernel_name(tsm.OP_TSM2R, 4096, 4096, n, dt)
            assert name.startswith("tsm2r_nn_kernel<%s, %d, " % (tname, 1 if n <= 16 else 2)), name
    assert tsm.kernel_name(tsm.OP_TSM2R, 4096, 4096, 33, tsm.F64) is None
    assert tsm.kernel_name(tsm.OP_TSM2R, 0, 4096, 8, tsm.F64) is None
    assert tsm.kernel_name(tsm.OP_TSM2L, 4096, 8, 8, tsm.F64) is None
    assert tsm.kernel_name(tsm.OP_TSM2R, 4096, 4096, 8, tsm.BF16) is None


@pytest.mark.parametrize("args,expect", [
    ((0, 100, 8, 0, 1, 0), -1), ((100, 0, 8, 0, 1, 0), -2), ((100, 100, 0, 0, 1, 0), -3),
    ((100, 100, 33, 0, 1, 0), -3), ((100, 100, 8, 2, 1, 0), -4), ((100, 100, 8, 9, 1, 0), -4),
    ((100, 100, 8, 0, -1, 0), -5), ((100, 100, 8, 0, 101, 0), -5), ((100, 100, 8, 0, 1, 2), -6),
    ((100, 100, 8, 0, 1, -2), -6)])
def test_tsm2r_pin_argument_checks(args, expect):
    assert _lib.lib().tsm2x_tsm2r_pin(*args) == expect


def test_tsm2r_pin_and_unpin_on_host():
    L = _lib.lib()
    assert L.tsm2x_tsm2r_pin(1000, 2000, 8, 0, 3, 1) == 0
    assert L.tsm2x_tsm2r_pin(1000, 2000, 8, 0, 0, -1) == 0      # removes it
    assert L.tsm2x_tsm2r_pin(1000, 2000, 8, 0, 0, -1) == 0      # removing twice is fine


@pytest.mark.parametrize("args,expect", [
    ((0, 100, 8, 0), -1), ((100, 0, 8, 0), -2), ((100, 100, 0, 0), -3), ((100, 100, 40, 0), -3),
    ((100, 100, 8, 4), -4)])
def test_tsm2r_plan_argument_checks(args, expect):
    n = None
    assert _lib.lib().tsm2x_tsm2r_plan(*args, n, n, n, n, n, n) == expect


def test_kmeans_argument_checks():
    L = _lib.lib()
    p = 4096                                    # never dereferenced: the checks come first
    ok = [1000, 16, 8, p, 1000, 0, p, 16, p, None, 0, None, 0, None]
    for pos, bad in [(1, -1), (2, 0), (3, 0), (4, None), (5, 999), (6, 2), (7, None), (8, 15),
                     (9, None), (11, 2)]:
        args = list(ok)
        args[pos - 1] = bad
        assert L.tsm_kmeans_assign(*args) == -pos, pos
    rowm = list(ok)
    rowm[5], rowm[4] = 1, 15                    # row-major: ldx >= k
    assert L.tsm_kmeans_assign(*rowm) == -5
    empty = list(ok)
    empty[0] = 0
    assert L.tsm_kmeans_assign(*empty) == 0     # no points: nothing to do, no GPU call


def test_kmeans_workspace_size():
    assert tsm.workspace_size(tsm.OP_KMEANS, 1000, 16, 8, tsm.F64) == 256
    assert tsm.workspace_size(tsm.OP_KMEANS, 1000, 16, 100, tsm.F32) == 512
    assert tsm.workspace_size(tsm.OP_KMEANS, 1000, 16, 8, tsm.BF16) == 0
