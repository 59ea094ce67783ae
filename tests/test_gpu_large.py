"""More than 2^31 rows: every row index, tile counter and stride of the
kernels is 64-bit, and these checks run the TSM2L, TSM2R, dB (reduction over
m) and K-means kernels at m = 2^31 + 257.  The data are small integers given
by closed forms (exact in float), so the results are checked exactly against
the same closed forms.  Needs about 60 GB of device memory at a time."""
import pytest
import torch

import paper_2002_03258_amd as tsm
from paper_2002_03258_amd import kmeans

pytestmark = pytest.mark.gpu

M = (1 << 31) + 257


@pytest.fixture(scope="module")
def big(dev):
    if torch.cuda.get_device_properties(dev).total_memory < (120 << 30):
        pytest.skip("needs a GPU with at least 120 GB")
    yield
    torch.cuda.empty_cache()


def _col(j, dev, dtype=torch.float32):
    """Column j of the test matrix: ((i + 3 j) mod 7) - 3, i < M."""
    i = torch.arange(M, device=dev, dtype=torch.int64)
    return ((i + 3 * j) % 7 - 3).to(dtype)


def _sum_col(j):
    """Exact sum over i < M of ((i + 3 j) mod 7) - 3."""
    full, rem = divmod(M, 7)
    return sum(((r + 3 * j) % 7 - 3) for r in range(rem))    # full periods sum to 0


def test_tsm2l_and_grad_b_beyond_2_31_rows(dev, big):
    k, n = 2, 3
    A = tsm.empty_colmajor(M, k, torch.float32, dev)
    for j in range(k):
        A[:, j] = _col(j, dev)
    B = torch.tensor([[1.0, 2.0, -1.0], [3.0, -1.0, 2.0]], device=dev)
    C = tsm.tsm2l(A, B)
    for p in range(n):
        want = A[:, 0] * B[0, p] + A[:, 1] * B[1, p]       # exact small integers
        assert torch.equal(C[:, p], want), p
    del C
    # dB = A^T dC with dC = 1: column sums over all M rows, exact in the
    # double reduction, rounded once to float
    dC = torch.ones((n, M), device=dev).t()
    dB = tsm.grad_b(A, dC)
    for j in range(k):
        assert dB[j].tolist() == [float(torch.tensor(float(_sum_col(j)), dtype=torch.float32))] * n
    del A, dC, dB


def test_tsm2r_beyond_2_31_rows(dev, big):
    k, n = 5, 2
    A = tsm.empty_colmajor(M, k, torch.float32, dev)
    for j in range(k):
        A[:, j] = _col(j, dev)
    B = torch.arange(1, k * n + 1, device=dev, dtype=torch.float32).reshape(k, n)
    C = tsm.tsm2r(A, B)
    for p in range(n):
        want = sum(A[:, j] * B[j, p] for j in range(k))
        assert torch.equal(C[:, p], want), p
    del A, C


def test_kmeans_beyond_2_31_points(dev, big):
    k, n = 2, 3
    X = torch.empty((M, k), device=dev)                    # row-major points
    for j in range(k):
        X[:, j] = _col(j, dev)
    cents = [(-3, -3), (0, 0), (3, 2)]
    cent = torch.tensor(cents, dtype=torch.float32, device=dev)
    lab, dist = kmeans.assign(X, cent)
    # the points repeat with period 7 in i: the expected label and distance
    # of each residue class, by the definition (point (-3, 0) ties between
    # centroids 0 and 1: the smaller index)
    lut_l, lut_d = [], []
    for r in range(7):
        pt = ((r % 7) - 3, ((r + 3) % 7) - 3)
        d = [(pt[0] - c[0]) ** 2 + (pt[1] - c[1]) ** 2 for c in cents]
        lut_l.append(d.index(min(d)))
        lut_d.append(float(min(d)))
    res = torch.arange(M, device=dev, dtype=torch.int64) % 7
    assert torch.equal(lab, torch.tensor(lut_l, dtype=torch.int32, device=dev)[res])
    assert torch.equal(dist, torch.tensor(lut_d, dtype=torch.float32, device=dev)[res])


def test_lowp_beyond_2_31_rows(dev, big):
    """The bf16 storage form (small integers are exact in bf16; lo = 0):
    split, TSM2L on the planes, and dB over all M rows."""
    k, n = 2, 3
    A = tsm.empty_colmajor(M, k, torch.float32, dev)
    for j in range(k):
        A[:, j] = _col(j, dev)
    S = tsm.split(A, "bf16", lo=True)
    B = torch.tensor([[1.0, 2.0, -1.0], [3.0, -1.0, 2.0]], device=dev)
    C = tsm.tsm2l(S, B)
    for p in range(n):
        assert torch.equal(C[:, p], A[:, 0] * B[0, p] + A[:, 1] * B[1, p]), p
    del C
    dC = torch.ones((n, M), device=dev).t()
    dB = tsm.grad_b(S, dC)
    for j in range(k):
        assert dB[j].tolist() == [float(_sum_col(j))] * n
    del A, S, dC, dB
