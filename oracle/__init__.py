"""Oracle for TSM2X tall-and-skinny products: TEST INFRASTRUCTURE ONLY.

Only tests/, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The library in
``paper_2002_03258_amd`` never imports it, and it imports nothing from there.

It wraps the plain C routines of ``tsm_oracle.c`` (double precision,
unblocked, sequential sums) with numpy marshalling:

- :func:`matmul` -- C = A*B, the problem statement of the paper (Background,
  "Tall-and-Skinny Input for GEMM"), with the sum over j in increasing order
  as in the per-thread loop of the outer-product design (Algorithm 2).
- :func:`grad` -- dA = dC*B^T and dB = A^T*dC, the gradients of
  L = <dC, A*B>.
- :func:`round_fmt`, :func:`split` -- round-to-nearest-even into bfloat16 /
  binary16 and the hi+lo storage form of A.
- :func:`t2_threshold` -- the paper's boundary between the memory-bound and
  compute-bound regimes (Design of TSM2R, "Determine compute-bound or
  memory-bound"): t2 = PeakPerf / PeakBand * bytes_per_element.
- :func:`normwise_error` -- ||C - C_ref||_F / ||C_ref||_F, and
  :func:`componentwise_error` -- max |C - C_ref| / (|A||B|), elementwise.
- :func:`matmul_dot2` -- the same product with every sum taken by Dot2
  (Ogita, Rump, Oishi 2005), as accurate as a sum in twice double precision:
  it measures the rounding error of :func:`matmul` itself at full size.
- :func:`kmeans_assign` -- the K-means assignment step named in the paper's
  Introduction: nearest centroid by squared Euclidean distance, from its
  definition.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tsm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

BF16 = 0
F16 = 1


def build(force: bool = False) -> str:
    """Compile tsm_oracle.c into liboracle.so with gcc (-O2, OpenMP, no
    floating-point contraction, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c11",
               "-ffp-contract=off", "-fno-fast-math", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB_PATH)
            i64, dp = ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
            lib.tsm_oracle_matmul.argtypes = [i64, i64, i64, dp, i64, i64,
                                              dp, i64, i64, dp, i64, i64]
            lib.tsm_oracle_matmul.restype = None
            lib.tsm_oracle_grad.argtypes = [i64, i64, i64, dp, i64, dp, i64,
                                            dp, i64, ctypes.c_void_p, i64,
                                            ctypes.c_void_p, i64]
            lib.tsm_oracle_grad.restype = None
            lib.tsm_oracle_round.argtypes = [ctypes.c_double, ctypes.c_int,
                                             ctypes.c_int, ctypes.c_double]
            lib.tsm_oracle_round.restype = ctypes.c_double
            lib.tsm_oracle_round_fmt.argtypes = [ctypes.c_double, ctypes.c_int]
            lib.tsm_oracle_round_fmt.restype = ctypes.c_double
            lib.tsm_oracle_encode.argtypes = [ctypes.c_double, ctypes.c_int]
            lib.tsm_oracle_encode.restype = ctypes.c_uint16
            lib.tsm_oracle_decode.argtypes = [ctypes.c_uint16, ctypes.c_int]
            lib.tsm_oracle_decode.restype = ctypes.c_double
            lib.tsm_oracle_split.argtypes = [ctypes.c_void_p, i64, ctypes.c_int,
                                             ctypes.c_void_p, ctypes.c_void_p]
            lib.tsm_oracle_split.restype = None
            lib.tsm_oracle_matmul_dot2.argtypes = [i64, i64, i64, dp, i64, i64,
                                                   dp, i64, i64, dp, i64, i64]
            lib.tsm_oracle_matmul_dot2.restype = None
            lib.tsm_oracle_kmeans_assign.argtypes = [i64, i64, i64, dp, i64, i64, dp, i64, i64,
                                                     ctypes.c_void_p, ctypes.c_void_p]
            lib.tsm_oracle_kmeans_assign.restype = None
            lib.tsm_oracle_threads.argtypes = []
            lib.tsm_oracle_threads.restype = ctypes.c_int
            lib.tsm_oracle_set_threads.argtypes = [ctypes.c_int]
            lib.tsm_oracle_set_threads.restype = None
            _lib = lib
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _strides(a: np.ndarray):
    assert a.dtype == np.float64 and a.ndim == 2
    return a.strides[0] // 8, a.strides[1] // 8


def matmul(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """C = A*B in double precision, any memory order of A and B.

    Inputs of another floating dtype are widened to float64 first (exact
    for every dtype this project uses)."""
    lib = _load()
    A = np.asarray(A)
    B = np.asarray(B)
    if A.dtype != np.float64:
        A = A.astype(np.float64)
    if B.dtype != np.float64:
        B = B.astype(np.float64)
    m, k = A.shape
    k2, n = B.shape
    assert k == k2, (A.shape, B.shape)
    C = np.empty((m, n), dtype=np.float64, order="F")
    ars, acs = _strides(A)
    brs, bcs = _strides(B)
    crs, ccs = _strides(C)
    lib.tsm_oracle_matmul(m, k, n, _dptr(A), ars, acs, _dptr(B), brs, bcs,
                          _dptr(C), crs, ccs)
    return C


def matmul_dot2(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """C = A*B with each entry's sum by Dot2 (error-free products and
    additions, errors summed apart): accurate to about u|C| + (k u)^2 |A||B|."""
    lib = _load()
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    m, k = A.shape
    k2, n = B.shape
    assert k == k2, (A.shape, B.shape)
    C = np.empty((m, n), dtype=np.float64, order="F")
    ars, acs = _strides(A)
    brs, bcs = _strides(B)
    crs, ccs = _strides(C)
    lib.tsm_oracle_matmul_dot2(m, k, n, _dptr(A), ars, acs, _dptr(B), brs, bcs,
                               _dptr(C), crs, ccs)
    return C


def kmeans_assign(X: np.ndarray, Mu: np.ndarray):
    """(labels, dist) for points X (m x k, one point per row) and centroids Mu
    (k x n, one centroid per column): labels[i] is the smallest c minimising
    sum_j (X[i,j] - Mu[j,c])^2 (NaN distances skipped; label 0 if all are
    NaN), dist[i] that minimum, in double precision."""
    lib = _load()
    X = np.asarray(X, dtype=np.float64)
    Mu = np.asarray(Mu, dtype=np.float64)
    m, k = X.shape
    k2, n = Mu.shape
    assert k == k2 and n >= 1, (X.shape, Mu.shape)
    labels = np.empty(m, dtype=np.int32)
    dist = np.empty(m, dtype=np.float64)
    xrs, xcs = _strides(X)
    mrs, mcs = _strides(Mu)
    lib.tsm_oracle_kmeans_assign(m, k, n, _dptr(X), xrs, xcs, _dptr(Mu), mrs, mcs,
                                 labels.ctypes.data, dist.ctypes.data)
    return labels, dist


def grad(A: np.ndarray, B: np.ndarray, dC: np.ndarray):
    """(dA, dB) = (dC*B^T, A^T*dC): gradients of L(A,B) = <dC, A*B>."""
    A = np.asfortranarray(np.asarray(A, dtype=np.float64))
    B = np.asfortranarray(np.asarray(B, dtype=np.float64))
    dC = np.asfortranarray(np.asarray(dC, dtype=np.float64))
    m, k = A.shape
    _, n = B.shape
    assert B.shape == (k, n) and dC.shape == (m, n)
    dA = np.empty((m, k), dtype=np.float64, order="F")
    dB = np.empty((k, n), dtype=np.float64, order="F")
    lib = _load()
    lib.tsm_oracle_grad(m, k, n, _dptr(A), max(m, 1), _dptr(B), max(k, 1),
                        _dptr(dC), max(m, 1), dA.ctypes.data, max(m, 1),
                        dB.ctypes.data, max(k, 1))
    return dA, dB


def round_fmt(x, fmt: int) -> np.ndarray:
    """Round each value (given as float64) to bfloat16 (fmt=0) or binary16
    (fmt=1), nearest-even; returns the rounded values as float64."""
    lib = _load()
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    fx, fo = x.reshape(-1), out.reshape(-1)
    for i in range(fx.size):
        fo[i] = lib.tsm_oracle_round_fmt(float(fx[i]), fmt)
    return out


def encode(v: float, fmt: int) -> int:
    return int(_load().tsm_oracle_encode(float(v), fmt))


def decode(h: int, fmt: int) -> float:
    return float(_load().tsm_oracle_decode(int(h), fmt))


def split(a: np.ndarray, fmt: int, with_lo: bool = True):
    """hi = round(a), lo = round(a - hi) as uint16 bit patterns (same shape
    and memory order as ``a``, which must be float32)."""
    a = np.asarray(a)
    assert a.dtype == np.float32
    flat = np.ascontiguousarray(a.reshape(-1, order="A"))
    hi = np.empty(flat.shape, dtype=np.uint16)
    lo = np.empty(flat.shape, dtype=np.uint16) if with_lo else None
    _load().tsm_oracle_split(flat.ctypes.data, flat.size, fmt, hi.ctypes.data,
                             lo.ctypes.data if with_lo else None)
    order = "F" if (a.ndim > 1 and a.flags.f_contiguous
                    and not a.flags.c_contiguous) else "C"
    hi = hi.reshape(a.shape, order=order)
    if with_lo:
        lo = lo.reshape(a.shape, order=order)
    return hi, lo


def decode_plane(h: np.ndarray, fmt: int) -> np.ndarray:
    """Values (float64) of a uint16 plane of bfloat16/binary16 patterns."""
    lib = _load()
    flat = np.asarray(h, dtype=np.uint16).reshape(-1)
    table = np.array([lib.tsm_oracle_decode(v, fmt) for v in range(65536)],
                     dtype=np.float64)
    return table[flat].reshape(np.shape(h))


def threads() -> int:
    return int(_load().tsm_oracle_threads())


def set_threads(n: int) -> None:
    """Threads the oracle's row loops use from now on (timing only)."""
    _load().tsm_oracle_set_threads(int(n))


def t2_threshold(peak_perf_gflops: float, peak_bw_gbs: float,
                 bytes_per_elem: int) -> float:
    """Ridge of the TSM2R performance model: below this many columns of C
    per pass, A-streaming is memory-bound (Design of TSM2R, "Determine
    compute-bound or memory-bound", the equation for t2^threshold)."""
    return peak_perf_gflops / peak_bw_gbs * bytes_per_elem


def componentwise_error(C, C_ref, A, B) -> float:
    """max_ij |C - C_ref|_ij / (|A| |B|)_ij for C_ref ~ A*B: the error in the
    units of the standard bound |fl(A*B) - A*B| <= gamma_k |A| |B| (Higham,
    Accuracy and Stability of Numerical Algorithms, eq. 3.13).  An entry with
    (|A||B|)_ij = 0 counts 0 if it is exact and infinity otherwise."""
    C = np.asarray(C, dtype=np.float64)
    C_ref = np.asarray(C_ref, dtype=np.float64)
    den = matmul(np.abs(np.asarray(A, dtype=np.float64)), np.abs(np.asarray(B, dtype=np.float64)))
    diff = np.abs(C - C_ref)
    if diff.size == 0:
        return 0.0
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(den > 0, diff / np.where(den > 0, den, 1.0),
                     np.where(diff > 0, np.inf, 0.0))
    return float(np.max(r))


def normwise_error(C, C_ref) -> float:
    """||C - C_ref||_F / ||C_ref||_F, absolute when ||C_ref||_F = 0."""
    C = np.asarray(C, dtype=np.float64)
    C_ref = np.asarray(C_ref, dtype=np.float64)
    den = float(np.linalg.norm(C_ref))
    num = float(np.linalg.norm(C - C_ref))
    return num / den if den > 0 else num
