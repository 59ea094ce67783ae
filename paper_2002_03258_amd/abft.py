"""Algorithm-based fault tolerance (ABFT) checksums on the library's kernels.

Encoding checksums for ABFT multiplies a matrix by a tall-and-skinny weight
matrix (Introduction of the TSM2X paper), which is a TSM2R product: here the
row checksums of X (m x n) are X*W with W = [1, w] (n x 2, w_p = p + 1).

For C = A*B (A m x k, B k x n) the row checksums satisfy C*W = A*(B*W), the
checksum relation for matrix products (Huang and Abraham, IEEE Trans. Comput.
1984).  ``verify`` evaluates both sides with the library's products and flags
the rows whose residual exceeds the rounding bound of the two evaluations; a
single corrupted element in a row changes its residual by (d, d*(p + 1)), so
``correct`` locates column p from the ratio of the two residuals and
subtracts d.
"""
from __future__ import annotations

import torch

from . import empty_colmajor, gemm


def weights(n: int, dtype, device) -> torch.Tensor:
    """W = [1, w] (n x 2, column-major) with w_p = p + 1."""
    W = empty_colmajor(n, 2, dtype, device)
    W[:, 0] = 1
    W[:, 1] = torch.arange(1, n + 1, dtype=dtype, device=device)
    return W


def encode(X: torch.Tensor) -> torch.Tensor:
    """Row checksums X*W (m x 2) of X (m x n)."""
    return gemm(X, weights(X.shape[1], X.dtype, X.device))


def verify(A: torch.Tensor, B: torch.Tensor, C: torch.Tensor, c: float = 4.0):
    """Check C against A*B through their row checksums.

    Returns (rows, residual, tol): the indices of rows whose checksum residual
    C*W - A*(B*W) exceeds tol, the m x 2 residual and the m x 2 tolerance.
    Each side (and C itself) is a sum of at most k + n rounded products; with
    random signs their rounding errors grow like sqrt(k + n) u |A| (|B| W)
    (W >= 0), and tol = c sqrt(k + n + 2) u |A| (|B| W).  This is an estimate,
    as ABFT thresholds usually are: the worst-case bound gamma_{k+n} is about
    sqrt(k + n) times larger and would let much larger corruptions through.
    """
    m, k = A.shape
    n = B.shape[1]
    W = weights(n, C.dtype, C.device)
    got = gemm(C, W)                          # C*W, m x 2
    ref = gemm(A, gemm(B, W))                 # A*(B*W), m x 2
    scale = gemm(A.abs(), gemm(B.abs(), W))   # |A| (|B| W)
    u = torch.finfo(C.dtype).eps / 2
    tol = c * (k + n + 2) ** 0.5 * u * scale
    res = got - ref
    bad = (res.abs() > tol).any(dim=1).nonzero().flatten()
    return bad, res, tol


def correct(A: torch.Tensor, B: torch.Tensor, C: torch.Tensor) -> list:
    """Locate and fix one corrupted element in each flagged row of C (in
    place).  Returns [(row, column, correction)]; a row whose two residuals do
    not point at a single column is left unchanged and reported with column -1."""
    bad, res, _ = verify(A, B, C)
    n = C.shape[1]
    fixed = []
    for i in bad.tolist():
        d, dw = res[i, 0].item(), res[i, 1].item()
        ratio = dw / d if d != 0 else float("nan")
        p = round(ratio) - 1 if ratio == ratio else -1
        if 0 <= p < n and abs(ratio - (p + 1)) < 0.25:
            C[i, p] -= d
            fixed.append((i, p, d))
        else:
            fixed.append((i, -1, 0.0))
    return fixed
