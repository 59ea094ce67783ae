"""K-means assignment step on the library's fused kernel.

K-means is the first application the TSM2X paper gives for tall-and-skinny
GEMM (Introduction): the distance computation multiplies the m-by-k points by
the k-by-n centroids with n far below m.  ``assign`` runs that product and the
nearest-centroid choice in one kernel (``tsm_kmeans_assign``): the points are
read once, and only the labels and distances are written.
"""
from __future__ import annotations

import torch

from . import _check_device, _DT, _ld, _lib, _stream, _ws, colmajor, is_colmajor


def assign(X: torch.Tensor, centroids: torch.Tensor, with_dist: bool = True,
           workspace: torch.Tensor | None = None):
    """Nearest centroid of every point.

    X: m x k points (one per row), row-major (each point's coordinates
    contiguous) or column-major (feature-major); another layout is copied
    first.  centroids: n x k (one per row).  F64 or F32.  Returns (labels, dist): int32 labels[i], the
    smallest c with the smallest squared distance, and dist[i], that distance
    (None unless with_dist)."""
    _check_device(X, centroids)
    if X.dtype != centroids.dtype or X.dtype not in _DT:
        raise ValueError("X and centroids: the same dtype, float64 or float32")
    m, k = X.shape
    n, k2 = centroids.shape
    if k2 != k:
        raise ValueError("centroids have %d coordinates, points %d" % (k2, k))
    if X.stride(1) == 1 and X.stride(0) >= k:
        rowmajor, ldx = 1, X.stride(0)
    else:
        if not is_colmajor(X):
            X = colmajor(X)
        rowmajor, ldx = 0, _ld(X)
    Mu = centroids.contiguous()              # n x k row-major = k x n column-major, ld k
    labels = torch.empty(m, dtype=torch.int32, device=X.device)
    dist = torch.empty(m, dtype=X.dtype, device=X.device) if with_dist else None
    ws, wsb = _ws(workspace)
    _lib.call("tsm_kmeans_assign", m, k, n, X.data_ptr(), ldx, rowmajor, Mu.data_ptr(), k,
              labels.data_ptr(), dist.data_ptr() if dist is not None else None, _DT[X.dtype],
              ws, wsb, _stream())
    return labels, dist
