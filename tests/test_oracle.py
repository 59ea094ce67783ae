"""Pins of the oracle against facts that do not come from the oracle itself:
exact rational arithmetic, integer exactness, closed forms, transpose
identities, the bilinearity of the gradient, library rounding routines and the
paper's printed performance-model values."""
import json
import math
import os
import random
from fractions import Fraction

import numpy as np
import pytest
import torch

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _exact_matmul(A, B):
    m, k = A.shape
    n = B.shape[1]
    return [[sum((Fraction(float(A[i, j])) * Fraction(float(B[j, p]))
                  for j in range(k)), Fraction(0)) for p in range(n)]
            for i in range(m)]


# --------------------------------------------------------------- brute force
@pytest.mark.parametrize("seed", range(6))
def test_brute_force_matches_exact_rationals(seed):
    """Every (m,k,n) in 1..5 plus random larger shapes: the oracle's double
    result is within the sequential-summation bound of the exact rational
    result (|C - C_exact| <= gamma_k * (|A||B|), Higham, Accuracy and
    Stability of Numerical Algorithms, eq. 3.13)."""
    rng = np.random.default_rng(seed)
    shapes = [(m, k, n) for m in range(1, 6) for k in range(1, 6)
              for n in range(1, 6)] if seed == 0 else \
        [tuple(int(x) for x in rng.integers(1, 20, 3)) for _ in range(40)]
    u = 2.0 ** -53
    for (m, k, n) in shapes:
        A = rng.uniform(-1, 1, (m, k))
        B = rng.uniform(-1, 1, (k, n))
        C = oracle.matmul(np.asfortranarray(A), np.asfortranarray(B))
        E = _exact_matmul(A, B)
        absAB = np.abs(A) @ np.abs(B)
        gamma = k * u / (1 - k * u)
        for i in range(m):
            for p in range(n):
                err = abs(Fraction(float(C[i, p])) - E[i][p])
                assert err <= Fraction(gamma * absAB[i, p] * 1.0000001), (m, k, n, i, p)


def test_dropped_term_would_be_caught():
    """A sanity check of the pin itself: leaving out one product moves the
    result far outside the rounding bound."""
    rng = np.random.default_rng(11)
    A = rng.uniform(-1, 1, (4, 7))
    B = rng.uniform(-1, 1, (7, 3))
    C = oracle.matmul(A, B)
    C_bad = oracle.matmul(A[:, :6], B[:6, :])
    E = np.array([[float(x) for x in row] for row in _exact_matmul(A, B)])
    assert np.abs(C - E).max() < 1e-14
    assert np.abs(C_bad - E).max() > 1e-6


# ---------------------------------------------------------------- integers
@pytest.mark.parametrize("m,k,n", [(33, 70, 5), (1, 1, 1), (64, 257, 16), (7, 1, 32)])
def test_integer_inputs_bit_exact(m, k, n):
    """Integer-valued inputs with |a|,|b| <= 2^10 keep every partial sum below
    2^53, so the double result equals the integer result exactly."""
    rng = np.random.default_rng(m * 1000 + k)
    Ai = rng.integers(-1024, 1025, (m, k))
    Bi = rng.integers(-1024, 1025, (k, n))
    C = oracle.matmul(np.asfortranarray(Ai.astype(np.float64)),
                      np.asfortranarray(Bi.astype(np.float64)))
    ref = [[sum(int(Ai[i, j]) * int(Bi[j, p]) for j in range(k)) for p in range(n)]
           for i in range(m)]
    assert np.array_equal(C, np.array(ref, dtype=np.float64))


# ------------------------------------------------------------- closed forms
def test_ones_column_gives_row_sums():
    rng = np.random.default_rng(3)
    m, k = 50, 301
    A = np.asfortranarray(rng.uniform(-1, 1, (m, k)))
    C = oracle.matmul(A, np.ones((k, 1)))
    for i in range(m):
        exact = math.fsum(A[i, :])
        assert abs(C[i, 0] - exact) <= k * 2.0 ** -53 * np.abs(A[i, :]).sum()


def test_unit_vectors_identity_permutation_scaling_zero():
    rng = np.random.default_rng(4)
    m, k = 37, 9
    A = np.asfortranarray(rng.uniform(-1, 1, (m, k)))
    for j in range(k):
        e = np.zeros((k, 1))
        e[j, 0] = 1.0
        assert np.array_equal(oracle.matmul(A, e)[:, 0], A[:, j])
    assert np.array_equal(oracle.matmul(A, np.eye(k)), A)
    perm = rng.permutation(k)
    P = np.eye(k)[:, perm]
    assert np.array_equal(oracle.matmul(A, P), A[:, perm])
    assert np.array_equal(oracle.matmul(A, 8.0 * np.eye(k)), 8.0 * A)
    assert np.array_equal(oracle.matmul(np.zeros((m, k)), rng.uniform(-1, 1, (k, 4))),
                          np.zeros((m, 4)))


def test_empty_inner_dimension_gives_zeros():
    C = oracle.matmul(np.zeros((5, 0)), np.zeros((0, 3)))
    assert C.shape == (5, 3) and np.all(C == 0)


def test_linearity_in_B():
    rng = np.random.default_rng(5)
    A = rng.uniform(-1, 1, (20, 40))
    B1 = rng.uniform(-1, 1, (40, 3))
    B2 = rng.uniform(-1, 1, (40, 3))
    lhs = oracle.matmul(A, B1 + B2)
    rhs = oracle.matmul(A, B1) + oracle.matmul(A, B2)
    assert np.abs(lhs - rhs).max() < 1e-13


# --------------------------------------------------------------- transposes
def test_memory_order_and_transpose_identity():
    """Row-major and column-major storage give identical bits, and
    (A*B)^T = B^T*A^T with the same products in the same order."""
    rng = np.random.default_rng(6)
    A = rng.uniform(-1, 1, (31, 45))
    B = rng.uniform(-1, 1, (45, 7))
    C_f = oracle.matmul(np.asfortranarray(A), np.asfortranarray(B))
    C_c = oracle.matmul(np.ascontiguousarray(A), np.ascontiguousarray(B))
    assert np.array_equal(C_f, C_c)
    Ct = oracle.matmul(B.T, A.T)
    assert np.array_equal(Ct, C_f.T)


# ---------------------------------------------------------------- gradients
def test_grad_against_exact_rationals():
    rng = np.random.default_rng(7)
    m, k, n = 6, 5, 4
    A = rng.uniform(-1, 1, (m, k))
    B = rng.uniform(-1, 1, (k, n))
    dC = rng.normal(size=(m, n))
    dA, dB = oracle.grad(A, B, dC)
    for i in range(m):
        for j in range(k):
            e = sum(Fraction(float(dC[i, p])) * Fraction(float(B[j, p])) for p in range(n))
            assert abs(Fraction(float(dA[i, j])) - e) < Fraction(1, 10 ** 14)
    for j in range(k):
        for p in range(n):
            e = sum(Fraction(float(A[i, j])) * Fraction(float(dC[i, p])) for i in range(m))
            assert abs(Fraction(float(dB[j, p])) - e) < Fraction(1, 10 ** 14)


def test_grad_directional_derivative():
    """L(A,B) = <dC, A*B> is bilinear, so the central difference
    (L(A+eV) - L(A-eV)) / 2e equals <dA, V> up to rounding; likewise in B.
    L is evaluated with numpy, independently of the oracle."""
    rng = np.random.default_rng(8)
    m, k, n = 300, 24, 16
    A = rng.uniform(-1, 1, (m, k))
    B = rng.uniform(-1, 1, (k, n))
    dC = rng.normal(size=(m, n))
    dA, dB = oracle.grad(A, B, dC)

    def L(A_, B_):
        return float(np.sum(dC * (A_ @ B_)))

    V = rng.normal(size=(m, k))
    W = rng.normal(size=(k, n))
    eps = 0.5
    fdA = (L(A + eps * V, B) - L(A - eps * V, B)) / (2 * eps)
    fdB = (L(A, B + eps * W) - L(A, B - eps * W)) / (2 * eps)
    assert abs(fdA - np.sum(dA * V)) <= 1e-10 * (1 + abs(fdA))
    assert abs(fdB - np.sum(dB * W)) <= 1e-10 * (1 + abs(fdB))


# ----------------------------------------------------------------- rounding
def _special_values():
    vals = [0.0, -0.0, 1.0, -1.0, 3.0e38, -3.0e38, 1e-40, -1e-40, 65504.0,
            65519.99, 65520.0, 2.0 ** -24, 2.0 ** -25, 3 * 2.0 ** -26, 2.0 ** -14,
            1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -11, 1.0 + 3 * 2.0 ** -11,
            float("inf"), float("-inf"), 2.0 ** -133, 2.0 ** -134, 3 * 2.0 ** -135]
    return np.array(vals, dtype=np.float32)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(9)
    x = np.concatenate([
        rng.uniform(-1, 1, 20000).astype(np.float32),
        (rng.standard_normal(20000) * 10.0 ** rng.integers(-40, 38, 20000)).astype(np.float32),
        _special_values()])
    ours = oracle.round_fmt(x.astype(np.float64), oracle.BF16)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(ours, ref)


def test_f16_rounding_matches_numpy():
    rng = np.random.default_rng(10)
    x = np.concatenate([
        rng.uniform(-1, 1, 20000).astype(np.float32),
        (rng.standard_normal(20000) * 10.0 ** rng.integers(-9, 6, 20000)).astype(np.float32),
        _special_values()])
    ours = oracle.round_fmt(x.astype(np.float64), oracle.F16)
    ref = x.astype(np.float16).astype(np.float64)
    assert np.array_equal(ours, ref)


@pytest.mark.parametrize("fmt", [oracle.BF16, oracle.F16])
def test_encode_decode_all_patterns(fmt):
    """decode is checked against the library's reinterpretation of all 2^16
    patterns; encode(decode(h)) == h for every non-NaN pattern."""
    pats = np.arange(65536, dtype=np.uint16)
    dec = oracle.decode_plane(pats, fmt)
    if fmt == oracle.BF16:
        ref = torch.from_numpy(pats.view(np.int16)).view(torch.bfloat16).to(torch.float64).numpy()
    else:
        ref = pats.view(np.float16).astype(np.float64)
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(dec), nan)
    assert np.array_equal(dec[~nan], ref[~nan])
    for h in range(0, 65536, 7):
        if not nan[h]:
            assert oracle.encode(dec[h], fmt) == h


def test_split_bf16_error_and_hi():
    rng = np.random.default_rng(12)
    a = rng.uniform(-1, 1, 50000).astype(np.float32)
    hi, lo = oracle.split(a, oracle.BF16)
    ref_hi = torch.from_numpy(a).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(hi, ref_hi)
    v = oracle.decode_plane(hi, 0) + oracle.decode_plane(lo, 0)
    assert np.all(np.abs(a.astype(np.float64) - v) <= 2.0 ** -16 * np.abs(a))
    # the single form alone is within half a bfloat16 ulp
    assert np.all(np.abs(a - oracle.decode_plane(hi, 0)) <= 2.0 ** -8 * np.abs(a))


def test_split_f16_error_normal_range():
    rng = np.random.default_rng(13)
    a = rng.uniform(0.125, 1, 50000).astype(np.float32) * rng.choice([-1, 1], 50000).astype(np.float32)
    hi, lo = oracle.split(a, oracle.F16)
    assert np.array_equal(hi, a.astype(np.float16).view(np.uint16))
    v = oracle.decode_plane(hi, 1) + oracle.decode_plane(lo, 1)
    assert np.all(np.abs(a.astype(np.float64) - v) <= 2.0 ** -22 * np.abs(a))


def test_split_integer_values_have_zero_lo():
    a = np.arange(-256, 257, dtype=np.float32)
    hi, lo = oracle.split(a, oracle.BF16)
    assert np.all(oracle.decode_plane(lo, 0) == 0)
    assert np.array_equal(oracle.decode_plane(hi, 0), a)


# ------------------------------------------------------------ perf model
def test_t2_threshold_reproduces_paper_values():
    g = json.load(open(os.path.join(GOLDEN, "t2_threshold.json")))
    bpe = g["bytes_per_element"]
    by_name = {}
    for row in g["gpus"]:
        t2 = oracle.t2_threshold(row["peak_fp64_gflops"], row["peak_bw_gbs"], bpe)
        by_name[row["gpu"]] = t2
        assert abs(t2 - row["paper_t2_threshold"]) <= 0.1 * row["paper_t2_threshold"], row
    for claim in g["regime_claims"]:
        bound = "memory" if claim["n"] <= by_name[claim["gpu"]] else "compute"
        assert bound == claim["bound"], claim


def test_mi355x_ridge_is_far_above_32():
    # 78.6 TFLOP/s FP64 vector, 8 TB/s HBM3E: every n <= 32 is memory-bound.
    assert oracle.t2_threshold(78600, 8000, 8) > 32
    assert oracle.t2_threshold(78600, 8000, 4) > 32   # FP32 FMA without packing


def test_normwise_error():
    assert oracle.normwise_error([[3.0, 4.0]], [[0.0, 0.0]]) == 5.0
    assert oracle.normwise_error([[1.0, 1.0]], [[1.0, 1.0]]) == 0.0
    assert abs(oracle.normwise_error([[1.1]], [[1.0]]) - 0.1) < 1e-12


def test_componentwise_error_closed_forms():
    # A = [1, -1], B = [1; 1]: C = 0 exactly and (|A||B|) = 2, so an error of
    # 1e-3 in C is 5e-4 of the componentwise scale, however small C is
    A = np.array([[1.0, -1.0], [2.0, 0.0]])
    B = np.array([[1.0], [1.0]])
    ref = oracle.matmul(A, B)
    assert ref[0, 0] == 0.0 and ref[1, 0] == 2.0
    assert oracle.componentwise_error(ref, ref, A, B) == 0.0
    assert oracle.componentwise_error(ref + [[1e-3], [0.0]], ref, A, B) == pytest.approx(5e-4)
    assert oracle.componentwise_error(ref + [[0.0], [1e-3]], ref, A, B) == pytest.approx(5e-4)
    # a zero scale: exact entries count 0, anything else infinity
    Z = np.zeros((1, 2))
    assert oracle.componentwise_error([[0.0]], [[0.0]], Z, B) == 0.0
    assert oracle.componentwise_error([[1e-300]], [[0.0]], Z, B) == math.inf
    assert oracle.componentwise_error(np.zeros((0, 1)), np.zeros((0, 1)), np.zeros((0, 2)), B) == 0.0


@pytest.mark.parametrize("seed", [3, 4])
def test_componentwise_error_bounds_the_sequential_sum(seed):
    """The oracle's own double sums, against exact rational sums, stay within
    gamma_k = k u / (1 - k u) of |A||B| componentwise (Higham, eq. 3.13),
    and a single perturbation larger than that is seen."""
    rng = random.Random(seed)
    m, k, n = 6, 40, 3
    A = np.array([[rng.uniform(-1, 1) for _ in range(k)] for _ in range(m)])
    B = np.array([[rng.uniform(-1, 1) for _ in range(n)] for _ in range(k)])
    exact = np.array([[float(sum(Fraction(A[i, j]) * Fraction(B[j, p]) for j in range(k)))
                       for p in range(n)] for i in range(m)])
    u = 2.0 ** -53
    gamma = k * u / (1 - k * u)
    C = oracle.matmul(A, B)
    e = oracle.componentwise_error(C, exact, A, B)
    assert e <= gamma
    scale = np.abs(A) @ np.abs(B)
    bad = C.copy()
    bad[2, 1] += 4 * gamma * scale[2, 1]
    assert oracle.componentwise_error(bad, exact, A, B) > gamma


# ------------------------------------------------------------ k-means assignment
def _kmeans_brute(X, Mu):
    """Exact rational distances, first index among equal minima."""
    from fractions import Fraction
    m, k = X.shape
    n = Mu.shape[1]
    labels, dists = [], []
    for i in range(m):
        best, bd = None, None
        for c in range(n):
            d = sum((Fraction(X[i, j]) - Fraction(Mu[j, c])) ** 2 for j in range(k))
            if bd is None or d < bd:
                best, bd = c, d
        labels.append(best)
        dists.append(bd)
    return np.array(labels), dists


@pytest.mark.parametrize("m,k,n,seed", [(7, 3, 4, 1), (9, 1, 5, 2), (5, 6, 1, 3), (12, 4, 9, 4),
                                        (3, 9, 2, 5)])
def test_kmeans_oracle_against_exact_brute_force(m, k, n, seed):
    rng = np.random.default_rng(seed)
    X = rng.integers(-32, 33, (m, k)) / 8.0          # dyadic: every distance exact in double
    Mu = rng.integers(-32, 33, (k, n)) / 8.0
    lab, dist = oracle.kmeans_assign(X, Mu)
    blab, bdist = _kmeans_brute(X, Mu)
    assert np.array_equal(lab, blab)
    assert [float(d) for d in bdist] == dist.tolist()


def test_kmeans_oracle_one_dimension_matches_sorted_search():
    rng = np.random.default_rng(11)
    cents = np.sort(rng.choice(np.arange(-1000, 1000), 40, replace=False)).astype(np.float64)
    pts = rng.integers(-1100, 1100, 5000) + 0.25        # never on a midpoint of integers
    lab, dist = oracle.kmeans_assign(pts[:, None], cents[None, :])
    pos = np.clip(np.searchsorted(cents, pts), 1, len(cents) - 1)
    left, right = cents[pos - 1], cents[pos]
    want = np.where(pts - left <= right - pts, pos - 1, pos)
    want[pts < cents[0]] = 0
    want[pts > cents[-1]] = len(cents) - 1
    assert np.array_equal(lab, want)
    assert np.array_equal(dist, (pts - cents[want]) ** 2)


def test_kmeans_oracle_points_on_centroids_and_ties():
    rng = np.random.default_rng(12)
    Mu = rng.standard_normal((5, 6))
    Mu[:, 4] = Mu[:, 1]                               # a duplicate centroid: ties go to 1
    X = np.ascontiguousarray(Mu.T)                     # point c sits on centroid c
    lab, dist = oracle.kmeans_assign(X, Mu)
    assert lab.tolist() == [0, 1, 2, 3, 1, 5]
    assert np.all(dist == 0)


def test_kmeans_oracle_permutation_and_translation():
    rng = np.random.default_rng(13)
    X = rng.integers(-8, 9, (400, 7)).astype(np.float64)
    Mu = rng.integers(-8, 9, (7, 10)).astype(np.float64) + 0.5
    lab, dist = oracle.kmeans_assign(X, Mu)
    perm = rng.permutation(10)
    lab_p, dist_p = oracle.kmeans_assign(X, Mu[:, perm])
    # the distance is unique; the label is a minimiser, and the same centroid
    # wherever the minimiser is unique
    assert np.array_equal(dist_p, dist)
    D = ((X[:, :, None] - Mu[None, :, :]) ** 2).sum(axis=1)
    assert np.all(D[np.arange(400), perm[lab_p]] == dist)
    unique = (D == dist[:, None]).sum(axis=1) == 1
    assert unique.sum() > 200
    assert np.array_equal(perm[lab_p][unique], lab[unique])
    v = rng.integers(-50, 50, 7).astype(np.float64)
    lab_t, dist_t = oracle.kmeans_assign(X + v, Mu + v[:, None])
    assert np.array_equal(lab_t, lab) and np.array_equal(dist_t, dist)


def test_kmeans_oracle_nan_handling():
    X = np.array([[0.0, 0.0], [np.nan, 1.0], [5.0, 5.0]])
    Mu = np.array([[np.nan, 1.0, 4.0], [0.0, 1.0, 4.0]])    # centroid 0 has a NaN coordinate
    lab, dist = oracle.kmeans_assign(X, Mu)
    assert lab.tolist() == [1, 0, 2]                   # row 1: every distance NaN -> label 0
    assert dist[0] == 2.0 and np.isnan(dist[1]) and dist[2] == 2.0


# ------------------------------------------------------------ Dot2 oracle
def _exact_dot(x, y):
    from fractions import Fraction
    return sum((Fraction(float(a)) * Fraction(float(b)) for a, b in zip(x, y)), Fraction(0))


def _illcond_vectors(n, rng):
    """Dot products with heavy cancellation: large terms that cancel in pairs
    around a small true value (exponents spread over 2^0 .. 2^60)."""
    x = rng.standard_normal(n) * 2.0 ** rng.integers(0, 60, n)
    y = rng.standard_normal(n)
    half = n // 2
    x[half:2 * half] = -x[:half]
    y[half:2 * half] = y[:half] * (1 + 2.0 ** -40 * rng.standard_normal(half))
    return x, y


@pytest.mark.parametrize("n,seed", [(10, 1), (64, 2), (200, 3), (501, 4)])
def test_dot2_within_its_error_bound_on_cancelling_sums(n, seed):
    rng = np.random.default_rng(seed)
    x, y = _illcond_vectors(n, rng)
    exact = float(_exact_dot(x, y))
    got = oracle.matmul_dot2(x[None, :], y[:, None])[0, 0]
    plain = oracle.matmul(x[None, :], y[:, None])[0, 0]
    u = 2.0 ** -53
    gam = n * u / (1 - n * u)
    bound = u * abs(exact) + gam ** 2 * float(np.sum(np.abs(x * y)))
    assert abs(got - exact) <= bound
    # the sequential sum is far off on these: the check has teeth
    if n >= 64:
        assert abs(plain - exact) > 1e3 * max(abs(got - exact), bound)


def test_dot2_equals_plain_on_exact_sums():
    rng = np.random.default_rng(5)
    A = rng.integers(-8, 9, (37, 300)).astype(np.float64)
    B = rng.integers(-8, 9, (300, 5)).astype(np.float64)
    assert np.array_equal(oracle.matmul_dot2(A, B), oracle.matmul(A, B))
    assert np.array_equal(oracle.matmul_dot2(A, B), A @ B)


def test_plain_oracle_error_at_full_size_is_far_below_the_fp64_bar():
    # rows of the largest TSM2R product (k = 30720, uniform[-1, 1)): the
    # sequential oracle differs from Dot2 by about 6e-15 normwise (u sqrt(k/2)
    # is 1.4e-14), well below the FP64 tolerance of the parity tests
    import seeded_inputs as si
    m = k = 30720
    rows = [0, 12345, m - 1]
    Ar = si.matrix_rows(7, si.STREAM_A, m, k, rows, dtype=torch.float64).numpy()
    B = si.matrix(8, si.STREAM_B, k, 16, dtype=torch.float64).numpy()
    plain = oracle.matmul(Ar, B)
    dd = oracle.matmul_dot2(Ar, B)
    assert oracle.normwise_error(plain, dd) < 1e-14
