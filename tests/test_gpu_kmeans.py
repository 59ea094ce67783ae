"""The fused K-means assignment kernel against the FP64 oracle: bit-exact
labels and distances on integer data (every sum exact, ties to the smaller
index on both sides), and on random data labels whose distance is within the
rounding bound of the true minimum."""
import numpy as np
import pytest
import torch

import oracle
import paper_2002_03258_amd as tsm
from paper_2002_03258_amd import kmeans
import seeded_inputs as si

from helpers import dev_matrix, host_matrix, to_np

pytestmark = pytest.mark.gpu

DTYPES = [torch.float64, torch.float32]
SHAPES = [(1 << 20, 16, 16), (300001, 8, 5), (4097, 32, 32), (100003, 3, 40), (20000, 100, 10),
          (77, 1, 1), (5, 20, 33), (1000, 33, 17), (129, 9, 70)]


def _data(seed, m, k, n, dtype, dev, dist="uniform", r=8):
    X = dev_matrix(seed, si.STREAM_A, m, k, dtype, dev, dist=dist, r=r)
    Mu = dev_matrix(seed, si.STREAM_B, k, n, dtype, dev, dist=dist, r=r)
    Xh = host_matrix(seed, si.STREAM_A, m, k, dtype, dist=dist, r=r)
    Muh = host_matrix(seed, si.STREAM_B, k, n, dtype, dist=dist, r=r)
    return X, Mu, Xh, Muh


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("m,k,n", SHAPES)
def test_integer_points_bit_exact(dev, dtype, m, k, n):
    seed = 2400 + m % 997 + k + n
    X, Mu, Xh, Muh = _data(seed, m, k, n, dtype, dev, dist="int", r=6)
    lab, dist = kmeans.assign(X, Mu.t())
    rlab, rdist = oracle.kmeans_assign(Xh, Muh)
    assert np.array_equal(lab.cpu().numpy(), rlab)
    assert np.array_equal(dist.double().cpu().numpy(), rdist)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("m,k,n", SHAPES)
@pytest.mark.parametrize("pad", [0, 3])
def test_rowmajor_points_bit_exact(dev, dtype, m, k, n, pad):
    """Row-major points (each point's k values contiguous, ld = k + pad): the
    contiguous-stream path, staged through LDS."""
    seed = 2450 + m % 997 + k + n
    X, Mu, Xh, Muh = _data(seed, m, k, n, dtype, dev, dist="int", r=6)
    store = torch.empty((m, k + pad), dtype=dtype, device=dev)
    Xr = store[:, :k]
    Xr.copy_(X)
    assert Xr.stride() == (k + pad, 1)
    lab, dist = kmeans.assign(Xr, Mu.t())
    rlab, rdist = oracle.kmeans_assign(Xh, Muh)
    assert np.array_equal(lab.cpu().numpy(), rlab)
    assert np.array_equal(dist.double().cpu().numpy(), rdist)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("m,k,n", [(200003, 16, 16), (3001, 100, 40)])
def test_rowmajor_random_points_within_rounding(dev, dtype, m, k, n):
    seed = 2550 + m % 997 + k + n
    X, Mu, Xh, Muh = _data(seed, m, k, n, dtype, dev)
    lab, dist = kmeans.assign(X.contiguous(), Mu.t())
    _check_valid(lab, dist, Xh, Muh, torch.finfo(dtype).eps / 2)


def _check_valid(lab, dist, Xh, Muh, u):
    """Each label's oracle distance is within the rounding bound of the
    minimum, and the returned distance within that bound of the label's."""
    lab = lab.cpu().numpy()
    dist = dist.double().cpu().numpy()
    m = Xh.shape[0]
    D = ((Xh[:, :, None] - Muh[None, :, :]) ** 2).sum(axis=1)
    xn = np.sqrt((Xh ** 2).sum(axis=1))
    mn = np.sqrt((Muh ** 2).sum(axis=0))
    k = Xh.shape[1]
    tol = 4 * (k + 2) * u * (xn[:, None] + mn[None, :]).max(axis=1) ** 2
    Dl = D[np.arange(m), lab]
    assert np.all(Dl <= D.min(axis=1) + tol)
    assert np.all(np.abs(dist - Dl) <= tol)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("m,k,n", [(200003, 16, 16), (5000, 32, 32), (3001, 100, 40), (999, 5, 3)])
def test_random_points_within_rounding(dev, dtype, m, k, n):
    seed = 2500 + m % 997 + k + n
    X, Mu, Xh, Muh = _data(seed, m, k, n, dtype, dev)
    lab, dist = kmeans.assign(X, Mu.t())
    _check_valid(lab, dist, Xh, Muh, torch.finfo(dtype).eps / 2)
    rlab, _ = oracle.kmeans_assign(Xh, Muh)
    assert (lab.cpu().numpy() == rlab).mean() > 0.999     # only near-ties may differ


@pytest.mark.parametrize("dtype", DTYPES)
def test_labels_only_and_deterministic(dev, dtype):
    X, Mu, _, _ = _data(2601, 100003, 16, 16, dtype, dev)
    lab, dist = kmeans.assign(X, Mu.t())
    lab2, none = kmeans.assign(X, Mu.t(), with_dist=False)
    assert none is None and torch.equal(lab, lab2)
    lab3, dist3 = kmeans.assign(X, Mu.t())
    assert torch.equal(lab, lab3) and torch.equal(dist, dist3)


@pytest.mark.parametrize("dtype", DTYPES)
def test_ties_points_on_centroids_and_nan(dev, dtype):
    m, k, n = 5003, 12, 20
    X, Mu, Xh, Muh = _data(2602, m, k, n, dtype, dev)
    Mu[:, 13] = Mu[:, 4]                       # duplicate centroid: never chosen over 4
    X[:n] = Mu.t()                             # point c sits on centroid c
    X[7, 3] = float("nan")
    lab, dist = kmeans.assign(X, Mu.t())
    lab = lab.cpu().numpy()
    dist = dist.double().cpu().numpy()
    assert not np.any(lab == 13)
    want = [c if c != 13 else 4 for c in range(n)]
    ok = [c for c in range(n) if c != 7]
    assert np.array_equal(lab[ok], np.array(want)[ok])
    assert np.all(np.abs(dist[ok]) <= 1e-4 if dtype == torch.float32 else np.abs(dist[ok]) <= 1e-12)
    assert lab[7] == 0 and np.isnan(dist[7])


@pytest.mark.parametrize("dtype", DTYPES)
def test_misaligned_and_rowmajor_points(dev, dtype):
    m, k, n = 40001, 16, 8
    X, Mu, Xh, Muh = _data(2603, m, k, n, dtype, dev, dist="int", r=5)
    store = torch.empty((k, m + 3), dtype=dtype, device=dev)
    Xs = store[:, 1:m + 1].t()                 # column-major, base not 16-byte aligned
    Xs.copy_(X)
    rstore = torch.empty((m, k + 1), dtype=dtype, device=dev)
    Xrs = rstore[:, 1:]                        # row-major, base not 16-byte aligned
    Xrs.copy_(X)
    rlab, rdist = oracle.kmeans_assign(Xh, Muh)
    for Xv in (Xs, X.contiguous(), Xrs):
        lab, dist = kmeans.assign(Xv, Mu.t())
        assert np.array_equal(lab.cpu().numpy(), rlab)
        assert np.array_equal(dist.double().cpu().numpy(), rdist)


def test_caller_workspace(dev):
    X, Mu, Xh, Muh = _data(2604, 10000, 16, 16, torch.float64, dev, dist="int", r=5)
    w = tsm.workspace_size(tsm.OP_KMEANS, 10000, 16, 16, tsm.F64)
    ws = torch.empty(w, dtype=torch.uint8, device=dev)
    lab, dist = kmeans.assign(X, Mu.t(), workspace=ws)
    rlab, rdist = oracle.kmeans_assign(Xh, Muh)
    assert np.array_equal(lab.cpu().numpy(), rlab) and np.array_equal(to_np(dist), rdist)
