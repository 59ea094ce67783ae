"""MI355X (gfx950) tall-and-skinny matrix products of TSM2X.

Thin torch binding of libtsm2x.so.  Torch supplies device memory and the
current stream; the products themselves run in the library's HIP kernels.
Matrices are column-major: a torch tensor ``X`` of shape (rows, cols) with
``X.stride(0) == 1`` and ``X.stride(1) = ld >= rows`` (e.g. ``Y.t()`` for a
row-major ``Y``).  Outputs are allocated column-major.
"""
from __future__ import annotations

import torch

from . import _lib
from ._lib import (BF16, BF16_SPLIT, COL_MAJOR, F16, F16_SPLIT, F32, F64,
                   ROW_MAJOR, TSMError)

__all__ = ["tsm2r", "tsm2l", "grad_a", "grad_b", "colmajor", "empty_colmajor",
           "workspace_size", "TSMError", "F64", "F32", "BF16", "F16",
           "BF16_SPLIT", "F16_SPLIT"]

_DT = {torch.float64: F64, torch.float32: F32}


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def is_colmajor(x: torch.Tensor) -> bool:
    return x.dim() == 2 and (x.stride(0) == 1 or x.size(0) <= 1) and \
        x.stride(1) >= max(1, x.size(0))


def colmajor(x: torch.Tensor) -> torch.Tensor:
    """``x`` itself if column-major, else a column-major copy."""
    if is_colmajor(x):
        return x
    return x.t().contiguous().t()


def empty_colmajor(rows: int, cols: int, dtype, device) -> torch.Tensor:
    return torch.empty((cols, rows), dtype=dtype, device=device).t()


def _ld(x: torch.Tensor) -> int:
    return max(1, x.stride(1)) if x.size(1) > 1 else max(1, x.size(0))


def _check_device(*ts):
    for t in ts:
        if not t.is_cuda:
            raise ValueError("tensors must be on a GPU device")


def tsm2r(A: torch.Tensor, B: torch.Tensor, out: torch.Tensor | None = None,
          workspace: torch.Tensor | None = None) -> torch.Tensor:
    """C = A*B for a large A (m x k, column- or row-major) and a skinny B
    (k x n, n <= 32) -- TSM2R."""
    _check_device(A, B)
    dt = _DT[A.dtype]
    m, k = A.shape
    n = B.shape[1]
    B = colmajor(B)
    C = out if out is not None else empty_colmajor(m, n, A.dtype, A.device)
    rowA = (not is_colmajor(A)) and A.stride(1) == 1 and k > 1
    if not rowA:
        A = colmajor(A)
        lda = _ld(A)
    else:
        lda = max(1, A.stride(0))
    ws, wsb = (workspace.data_ptr(), workspace.numel() * workspace.element_size()) \
        if workspace is not None else (None, 0)
    _lib.call("tsm2r_ex", ROW_MAJOR if rowA else COL_MAJOR, m, k, n, A.data_ptr(), lda,
              B.data_ptr(), _ld(B), C.data_ptr(), _ld(C), dt, ws, wsb, _stream())
    return C


def tsm2l(A: torch.Tensor, B: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """C = A*B for a tall-and-skinny A (m x k, k <= 32) and a small B
    (k x n, n <= 32) -- TSM2L."""
    _check_device(A, B)
    dt = _DT[A.dtype]
    A = colmajor(A)
    B = colmajor(B)
    m, k = A.shape
    n = B.shape[1]
    C = out if out is not None else empty_colmajor(m, n, A.dtype, A.device)
    _lib.call("tsm2l", m, k, n, A.data_ptr(), _ld(A), B.data_ptr(), _ld(B),
              C.data_ptr(), _ld(C), dt, _stream())
    return C


def grad_a(dC: torch.Tensor, B: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """dA = dC*B^T (dC m x n, B k x n, n <= 32)."""
    _check_device(dC, B)
    dt = _DT[dC.dtype]
    dC = colmajor(dC)
    B = colmajor(B)
    m, n = dC.shape
    k = B.shape[0]
    dA = out if out is not None else empty_colmajor(m, k, dC.dtype, dC.device)
    _lib.call("tsm_grad_a", m, k, n, dC.data_ptr(), _ld(dC), B.data_ptr(), _ld(B),
              dA.data_ptr(), _ld(dA), dt, _stream())
    return dA


def grad_b(A: torch.Tensor, dC: torch.Tensor, out: torch.Tensor | None = None,
           workspace: torch.Tensor | None = None) -> torch.Tensor:
    """dB = A^T*dC (A m x k, dC m x n, n <= 32)."""
    _check_device(A, dC)
    dt = _DT[A.dtype]
    A = colmajor(A)
    dC = colmajor(dC)
    m, k = A.shape
    n = dC.shape[1]
    dB = out if out is not None else empty_colmajor(k, n, A.dtype, A.device)
    ws, wsb = (workspace.data_ptr(), workspace.numel() * workspace.element_size()) \
        if workspace is not None else (None, 0)
    _lib.call("tsm_grad_b", m, k, n, A.data_ptr(), _ld(A), dC.data_ptr(), _ld(dC),
              dB.data_ptr(), _ld(dB), dt, ws, wsb, _stream())
    return dB


def workspace_size(op: int, m: int, k: int, n: int, dtype: int) -> int:
    return int(_lib.lib().tsm2x_workspace_size(op, m, k, n, dtype))
