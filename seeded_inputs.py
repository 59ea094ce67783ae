"""Seeded, counter-based synthetic inputs shared by the tests, the benchmark
and the smoke check.

This module holds no arithmetic of the method: it only turns
(seed, stream, logical index) into numbers, with the same bits on the CPU and
on the GPU, so that the oracle can regenerate any sampled row of a matrix that
lives only in device memory.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014).  Element ``idx`` of a stream uses the state
``base + (idx + 1) * GAMMA`` passed through the SplitMix64 finaliser, where
``base`` is the finaliser applied to ``seed * 2^8 + stream``.  All arithmetic
is on int64 tensors with two's-complement wrap-around; logical right shifts are
arithmetic shifts followed by a mask.

Distributions:
- ``uniform``: iid uniform on [-1, 1): top 53 bits u of the 64-bit output,
  value 2*u*2^-53 - 1, exact in float64.
- ``normal``: the classic sum-of-twelve-uniforms approximation of N(0, 1):
  twelve 32-bit halves of six outputs summed exactly in int64, value
  (S - 6*2^32) * 2^-32, exact in float64 (mean 0, variance 1, support
  [-6, 6)).
- ``int``: iid integers uniform in [-r, r] (``lo``/``hi`` bound), for inputs
  whose products are exact.

A matrix is generated in column-major storage: logical element (i, j) of a
rows x cols matrix has index ``j * rows + i``, independent of the leading
dimension, and padding rows (ld > rows) are filled with NaN.
"""
from __future__ import annotations

import torch

_M64 = (1 << 64) - 1


def _s64(c: int) -> int:
    c &= _M64
    return c - (1 << 64) if c >= (1 << 63) else c


GAMMA = _s64(0x9E3779B97F4A7C15)
_MUL1 = _s64(0xBF58476D1CE4E5B9)
_MUL2 = _s64(0x94D049BB133111EB)

# Fixed per-tensor streams.
STREAM_A, STREAM_B, STREAM_DC, STREAM_V, STREAM_W = 1, 2, 3, 4, 5


def _lsr(z: torch.Tensor, s: int) -> torch.Tensor:
    return (z >> s) & ((1 << (64 - s)) - 1)


def _mix(z: torch.Tensor) -> torch.Tensor:
    z = (z ^ _lsr(z, 30)) * _MUL1
    z = (z ^ _lsr(z, 27)) * _MUL2
    return z ^ _lsr(z, 31)


def _base(seed: int, stream: int) -> int:
    t = torch.tensor([_s64(((seed & 0xFFFFFFFFFF) << 8) | (stream & 0xFF))],
                     dtype=torch.int64)
    return int(_mix(t + GAMMA)[0])


def raw64(seed: int, stream: int, idx: torch.Tensor) -> torch.Tensor:
    """64-bit outputs (as int64) for the int64 counter tensor ``idx``."""
    return _mix(_base(seed, stream) + (idx + 1) * GAMMA)


def uniform(seed: int, stream: int, idx: torch.Tensor) -> torch.Tensor:
    z = raw64(seed, stream, idx)
    u = _lsr(z, 11).to(torch.float64)
    return u * (2.0 ** -52) - 1.0


def normal(seed: int, stream: int, idx: torch.Tensor) -> torch.Tensor:
    s = torch.zeros_like(idx)
    for t in range(6):
        z = raw64(seed, stream, idx * 6 + t)
        s = s + (z & 0xFFFFFFFF) + _lsr(z, 32)
    return (s - 6 * (1 << 32)).to(torch.float64) * (2.0 ** -32)


def integers(seed: int, stream: int, idx: torch.Tensor, r: int) -> torch.Tensor:
    z = _lsr(raw64(seed, stream, idx), 1)
    return (z % (2 * r + 1) - r).to(torch.float64)


def values(seed: int, stream: int, idx: torch.Tensor, dist: str = "uniform",
           r: int = 8) -> torch.Tensor:
    if dist == "uniform":
        return uniform(seed, stream, idx)
    if dist == "normal":
        return normal(seed, stream, idx)
    if dist == "int":
        return integers(seed, stream, idx, r)
    raise ValueError(dist)


_CHUNK = 1 << 24


def matrix(seed: int, stream: int, rows: int, cols: int, *, ld: int | None = None,
           dtype=torch.float64, device="cpu", dist: str = "uniform",
           r: int = 8) -> torch.Tensor:
    """Column-major rows x cols matrix, returned as the transposed view of a
    (cols, ld) storage tensor (so ``out.shape == (rows, cols)``,
    ``out.stride() == (1, ld)``).  Values are generated in float64 and
    rounded to ``dtype`` (round-to-nearest-even)."""
    ld = rows if ld is None else ld
    assert ld >= max(rows, 1)
    store = torch.empty((cols, ld), dtype=dtype, device=device)
    if ld > rows:
        store[:, rows:] = float("nan")
    total = rows * cols
    flat_rows = store[:, :rows]
    for c0 in range(0, cols, max(1, _CHUNK // max(rows, 1))):
        c1 = min(cols, c0 + max(1, _CHUNK // max(rows, 1)))
        idx = torch.arange(c0 * rows, c1 * rows, dtype=torch.int64, device=device)
        v = values(seed, stream, idx, dist, r).view(c1 - c0, rows)
        flat_rows[c0:c1] = v.to(dtype)
    del total
    return flat_rows.t()


def matrix_rows(seed: int, stream: int, rows: int, cols: int, row_idx,
                *, dtype=torch.float64, dist: str = "uniform",
                r: int = 8) -> torch.Tensor:
    """Only the listed rows of the matrix :func:`matrix` would produce, on
    the CPU: shape (len(row_idx), cols)."""
    ri = torch.as_tensor(row_idx, dtype=torch.int64).view(-1, 1)
    cj = torch.arange(cols, dtype=torch.int64).view(1, -1)
    v = values(seed, stream, cj * rows + ri, dist, r)
    return v.to(dtype)


def matrix_cols(seed: int, stream: int, rows: int, cols: int, col_idx,
                *, dtype=torch.float64, dist: str = "uniform",
                r: int = 8) -> torch.Tensor:
    """Only the listed columns of the matrix :func:`matrix` would produce, on
    the CPU: shape (rows, len(col_idx))."""
    ci = torch.as_tensor(col_idx, dtype=torch.int64).view(1, -1)
    ri = torch.arange(rows, dtype=torch.int64).view(-1, 1)
    v = values(seed, stream, ci * rows + ri, dist, r)
    return v.to(dtype)


def row_major(seed: int, stream: int, rows: int, cols: int, *,
              dtype=torch.float64, device="cpu", dist: str = "uniform"):
    """Row-major rows x cols matrix: logical (i, j) has index i * cols + j."""
    idx = torch.arange(rows * cols, dtype=torch.int64, device=device)
    return values(seed, stream, idx, dist).view(rows, cols).to(dtype)


def config_seed(index: int) -> int:
    """Seed of the index-th workload: 0x5EED0000 + index."""
    return 0x5EED0000 + index
