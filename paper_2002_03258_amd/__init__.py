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
from ._lib import (BF16, BF16_SPLIT, F16, F16_SPLIT, F32, F64, OP_GRAD_A, OP_GRAD_B, OP_KMEANS,
                   OP_TSM2L, OP_TSM2R, OP_TSM2R_ROWMAJOR, TSMError)

__all__ = ["tsm2r", "tsm2l", "gemm", "tsmttsm", "grad_a", "grad_b", "tsm2l_backward", "split", "SplitA",
           "plane_ld", "colmajor",
           "empty_colmajor", "workspace_size", "kernel_name", "tsm2r_plan", "pin_tsm2r",
           "unpin_tsm2r", "matmul", "TSMMatmul", "TSMError", "F64", "F32", "BF16", "F16",
           "BF16_SPLIT", "F16_SPLIT", "OP_TSM2R", "OP_TSM2L", "OP_GRAD_A", "OP_GRAD_B",
           "OP_TSM2R_ROWMAJOR", "timing_start", "timing_stop", "timing_tag", "timing_collect",
           "probe_stream", "probe_tiles"]

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


class SplitA:
    """Low-precision storage form of a float matrix A (m x k): a hi plane
    and optionally a lo plane of bfloat16 or binary16 values, hi + lo ~ A.
    ``planes`` is one device buffer of shape (nplanes, k, ld); plane p holds
    the column-major m x k matrix ``planes[p].t()[:m]``."""

    def __init__(self, planes: torch.Tensor, m: int, k: int, fmt: str, has_lo: bool,
                 source: torch.Tensor | None = None):
        self.planes, self.m, self.k, self.fmt, self.has_lo = planes, m, k, fmt, has_lo
        self.ld = planes.shape[2]
        # the float matrix the planes were split from (not copied), and its
        # version counter then: `matmul` differentiates with respect to it
        self.source = source
        self.source_version = source._version if source is not None else None

    def check_source(self) -> torch.Tensor:
        """The float matrix these planes were split from; raises if it was
        modified in place since (the planes would no longer hold its values)."""
        if self.source is None:
            raise ValueError("this SplitA was made without its source matrix")
        if self.source._version != self.source_version:
            raise ValueError("the source of this SplitA was modified after the split; "
                             "split it again")
        return self.source

    @property
    def hi(self) -> torch.Tensor:
        return self.planes[0].t()[: self.m]

    @property
    def lo(self) -> torch.Tensor | None:
        return self.planes[1].t()[: self.m] if self.has_lo else None

    @property
    def dtype_code(self) -> int:
        if self.fmt == "bf16":
            return BF16_SPLIT if self.has_lo else BF16
        return F16_SPLIT if self.has_lo else F16

    @property
    def shape(self):
        return (self.m, self.k)

    @property
    def device(self):
        return self.planes.device

    def nbytes(self) -> int:
        return self.m * self.k * 2 * (2 if self.has_lo else 1)


def plane_ld(m: int, k: int) -> int:
    """Leading dimension of the 16-bit planes of an m x k matrix: m rounded up
    to 8 (16-byte columns), plus 64 (128 bytes) for a wide matrix (k > 32)
    whose column stride would be a multiple of 1 KiB.  Columns a large power
    of two apart share HBM channels; the TSM2R-class kernels read many
    columns at once and measured 3-10 % faster on padded planes (A 16384^2
    and 32768^2), the TSM2L-class kernels on tall planes 2-5 % slower."""
    ld = max(8, (m + 7) // 8 * 8)
    if k > 32 and (2 * ld) % 1024 == 0:
        ld += 64
    return ld


def split(A: torch.Tensor, fmt: str = "bf16", lo: bool = True) -> SplitA:
    """hi = RNE(A), lo = RNE(A - hi) in bfloat16 ("bf16") or binary16 ("f16"),
    computed on the GPU by the library's split kernel."""
    _check_device(A)
    if A.dtype != torch.float32:
        raise ValueError("split expects a float32 matrix")
    if A.dim() != 2:
        raise ValueError("split expects a matrix")
    if fmt not in ("bf16", "f16"):
        raise ValueError("fmt must be 'bf16' or 'f16'")
    src = A
    A = colmajor(A)
    m, k = A.shape
    ld = plane_ld(m, k)
    tdt = torch.bfloat16 if fmt == "bf16" else torch.float16
    planes = torch.empty((2 if lo else 1, k, ld), dtype=tdt, device=A.device)
    lo_ptr = planes[1].data_ptr() if lo else None
    _lib.call("tsm2x_split", m, k, A.data_ptr(), _ld(A), planes[0].data_ptr(), lo_ptr, ld,
              0 if fmt == "bf16" else 1, _stream())
    return SplitA(planes, m, k, fmt, lo, source=src)


def _layout(x: torch.Tensor):
    """(trans, ld) of a 2-D tensor held column-major (trans 0) or row-major
    (trans 1: the column-major storage of its transpose); None otherwise."""
    r, c = x.shape
    if (x.stride(0) == 1 or r <= 1) and (c <= 1 or x.stride(1) >= max(1, r)):
        return 0, (x.stride(1) if c > 1 else max(1, r))
    if (x.stride(1) == 1 or c <= 1) and (r <= 1 or x.stride(0) >= max(1, c)):
        return 1, (x.stride(0) if r > 1 else max(1, c))
    return None


def _operand(x: torch.Tensor):
    """(tensor, trans, ld): x as it is when column- or row-major, else a
    column-major copy."""
    lay = _layout(x)
    if lay is None:
        x = colmajor(x)
        lay = (0, _ld(x))
    return x, lay[0], lay[1]


def _check_matrix(name: str, x: torch.Tensor, rows: int, cols: int, dtype) -> None:
    if x.dim() != 2 or tuple(x.shape) != (rows, cols):
        raise ValueError("%s must be %d x %d, got %s" % (name, rows, cols, tuple(x.shape)))
    if x.dtype != dtype:
        raise ValueError("%s must be %s, got %s" % (name, dtype, x.dtype))


def _check_out(out: torch.Tensor, rows: int, cols: int, dtype, device) -> None:
    if not is_colmajor(out) or tuple(out.shape) != (rows, cols) or out.dtype != dtype:
        raise ValueError("out must be a column-major %d x %d %s tensor" % (rows, cols, dtype))
    if out.device != device:
        raise ValueError("out must be on %s" % (device,))


def _plain_dtype(x: torch.Tensor) -> int:
    if x.dtype not in _DT:
        raise ValueError("expected a float64 or float32 tensor, got %s" % (x.dtype,))
    return _DT[x.dtype]


def _ws(workspace):
    return (workspace.data_ptr(), workspace.numel() * workspace.element_size()) \
        if workspace is not None else (None, 0)


def _product(fn: str, A, B: torch.Tensor, out, beta: float, workspace) -> torch.Tensor:
    if isinstance(A, SplitA):
        _check_device(A.planes, B)
        if B.dtype != torch.float32:
            raise ValueError("B must be float32 for the low-precision forms of A")
        m, k = A.shape
        a_ptr, ta, lda, code, cdt, dev = A.planes.data_ptr(), 0, A.ld, A.dtype_code, \
            torch.float32, A.device
    else:
        _check_device(A, B)
        if B.dtype != A.dtype:
            raise ValueError("A and B must have the same dtype")
        if A.dim() != 2 or B.dim() != 2:
            raise ValueError("A and B must be matrices")
        code, cdt, dev = _plain_dtype(A), A.dtype, A.device
        m, k = A.shape
        A, ta, lda = _operand(A)
        a_ptr = A.data_ptr()
    if B.shape[0] != k:
        raise ValueError("inner dimensions differ: A has %d columns, B %d rows" % (k, B.shape[0]))
    n = B.shape[1]
    B, tb, ldb = _operand(B)
    if out is None:
        if beta != 0:
            raise ValueError("beta != 0 accumulates into `out`, which must be given")
        out = empty_colmajor(m, n, cdt, dev)
    else:
        _check_out(out, m, n, cdt, dev)
    ws, wsb = _ws(workspace)
    _lib.call(fn, ta, tb, m, k, n, a_ptr, lda, B.data_ptr(), ldb, float(beta), out.data_ptr(),
              _ld(out), code, ws, wsb, _stream())
    return out


def tsm2r(A, B: torch.Tensor, out: torch.Tensor | None = None, beta: float = 0.0,
          workspace: torch.Tensor | None = None) -> torch.Tensor:
    """C := beta*C + A*B for a large A (m x k, column- or row-major, or a
    SplitA) and a skinny B (k x n) -- TSM2R.  For a SplitA, B and C are
    float32.  C is `out` (column-major); it is read only when beta != 0."""
    return _product("tsm2r_ex", A, B, out, beta, workspace)


def tsm2l(A, B: torch.Tensor, out: torch.Tensor | None = None, beta: float = 0.0,
          workspace: torch.Tensor | None = None) -> torch.Tensor:
    """C := beta*C + A*B for a tall-and-skinny A (m x k, k <= 32, or a SplitA)
    and a small B (k x n) -- TSM2L; other shapes run on the TSM2R kernels."""
    return _product("tsm2l_ex", A, B, out, beta, workspace)


def gemm(A, B: torch.Tensor, out: torch.Tensor | None = None, beta: float = 0.0,
         workspace: torch.Tensor | None = None) -> torch.Tensor:
    """C := beta*C + A*B, TSM2L or TSM2R chosen by the shape of A."""
    return _product("tsm2x_gemm", A, B, out, beta, workspace)


def tsmttsm(A: torch.Tensor, B: torch.Tensor, out: torch.Tensor | None = None,
            beta: float = 0.0, workspace: torch.Tensor | None = None) -> torch.Tensor:
    """C := beta*C + A^T*B for two tall matrices that share their long
    dimension (A m x k and B m x n, F64/F32, m large): the TSMTTSM form the
    paper names in its related work.  C is k x n; it runs on the reduction
    kernel of dB = A^T*dC (n in panels of 32 columns)."""
    if A.dim() != 2 or B.dim() != 2 or A.shape[0] != B.shape[0]:
        raise ValueError("tsmttsm: A (m x k) and B (m x n) must share m")
    return gemm(A.t(), B, out=out, beta=beta, workspace=workspace)


def grad_a(dC: torch.Tensor, B: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """dA = dC*B^T (dC m x n, B k x n, n <= 32, same dtype)."""
    _check_device(dC, B)
    dt = _plain_dtype(dC)
    if dC.dim() != 2 or B.dim() != 2:
        raise ValueError("dC and B must be matrices")
    m, n = dC.shape
    k = B.shape[0]
    _check_matrix("B", B, k, n, dC.dtype)
    if out is not None:
        _check_out(out, m, k, dC.dtype, dC.device)
    dC = colmajor(dC)
    B = colmajor(B)
    dA = out if out is not None else empty_colmajor(m, k, dC.dtype, dC.device)
    _lib.call("tsm_grad_a", m, k, n, dC.data_ptr(), _ld(dC), B.data_ptr(), _ld(B),
              dA.data_ptr(), _ld(dA), dt, _stream())
    return dA


def grad_b(A, dC: torch.Tensor, out: torch.Tensor | None = None,
           workspace: torch.Tensor | None = None) -> torch.Tensor:
    """dB = A^T*dC (A m x k or a SplitA, dC m x n, n <= 32; dC float32 for a
    SplitA, else of A's dtype)."""
    if isinstance(A, SplitA):
        _check_device(A.planes, dC)
        m, k = A.shape
        if dC.dim() != 2:
            raise ValueError("dC must be a matrix")
        _check_matrix("dC", dC, m, dC.shape[1], torch.float32)
        n = dC.shape[1]
        if out is not None:
            _check_out(out, k, n, torch.float32, dC.device)
        dC = colmajor(dC)
        dB = out if out is not None else empty_colmajor(k, n, torch.float32, dC.device)
        ws, wsb = (workspace.data_ptr(), workspace.numel() * workspace.element_size()) \
            if workspace is not None else (None, 0)
        _lib.call("tsm_grad_b", m, k, n, A.planes.data_ptr(), A.ld, dC.data_ptr(), _ld(dC),
                  dB.data_ptr(), _ld(dB), A.dtype_code, ws, wsb, _stream())
        return dB
    _check_device(A, dC)
    dt = _plain_dtype(A)
    if A.dim() != 2 or dC.dim() != 2:
        raise ValueError("A and dC must be matrices")
    m, k = A.shape
    n = dC.shape[1]
    _check_matrix("dC", dC, m, n, A.dtype)
    if out is not None:
        _check_out(out, k, n, A.dtype, A.device)
    A = colmajor(A)
    dC = colmajor(dC)
    dB = out if out is not None else empty_colmajor(k, n, A.dtype, A.device)
    ws, wsb = (workspace.data_ptr(), workspace.numel() * workspace.element_size()) \
        if workspace is not None else (None, 0)
    _lib.call("tsm_grad_b", m, k, n, A.data_ptr(), _ld(A), dC.data_ptr(), _ld(dC),
              dB.data_ptr(), _ld(dB), dt, ws, wsb, _stream())
    return dB


def tsm2l_backward(A, B: torch.Tensor, dC: torch.Tensor):
    """(dA, dB) = (dC*B^T, A^T*dC) for a TSM2L product (k, n <= 32) in one
    fused pass over A and dC.  A may be a SplitA (B, dC float32): dB then
    uses the stored values hi (+ lo), as the forward did."""
    if isinstance(A, SplitA):
        _check_device(A.planes, B, dC)
        if B.dtype != torch.float32 or dC.dtype != torch.float32:
            raise ValueError("B and dC must be float32 for the low-precision forms of A")
        a_ptr, lda, code, odt, dev = A.planes.data_ptr(), A.ld, A.dtype_code, torch.float32, \
            A.device
        m, k = A.shape
    else:
        _check_device(A, B, dC)
        code, odt, dev = _plain_dtype(A), A.dtype, A.device
        if A.dim() != 2:
            raise ValueError("A must be a matrix")
        A = colmajor(A)
        m, k = A.shape
        a_ptr, lda = A.data_ptr(), _ld(A)
    if B.dim() != 2 or dC.dim() != 2:
        raise ValueError("B and dC must be matrices")
    n = B.shape[1]
    _check_matrix("B", B, k, n, odt)
    _check_matrix("dC", dC, m, n, odt)
    B, dC = colmajor(B), colmajor(dC)
    dA = empty_colmajor(m, k, odt, dev)
    dB = empty_colmajor(k, n, odt, dev)
    _lib.call("tsm2l_backward", m, k, n, a_ptr, lda, B.data_ptr(), _ld(B),
              dC.data_ptr(), _ld(dC), dA.data_ptr(), _ld(dA), dB.data_ptr(), _ld(dB), code,
              None, 0, _stream())
    return dA, dB


def workspace_size(op: int, m: int, k: int, n: int, dtype: int) -> int:
    return int(_lib.lib().tsm2x_workspace_size(op, m, k, n, dtype))


def kernel_name(op: int, m: int, k: int, n: int, dtype: int):
    """Name of the main kernel the call launches (TSM2R, plain types), or None."""
    r = _lib.lib().tsm2x_kernel_name(op, m, k, n, dtype)
    return r.decode() if r else None


def tsm2r_plan(m: int, k: int, n: int, dtype: int) -> dict:
    """Launch plan of a TSM2R product on the current device (F64/F32, n <= 32):
    k split ``slices``, tile height ``tall`` (0/1), ``tiles``, ``tile_rows``,
    resident workgroups per CU ``occupancy``, ``cus`` and the kernel name."""
    import ctypes
    S, tall, rows, occ, cus = (ctypes.c_int() for _ in range(5))
    tiles = ctypes.c_int64()
    _lib.call("tsm2x_tsm2r_plan", m, k, n, dtype, ctypes.byref(S), ctypes.byref(tall),
              ctypes.byref(tiles), ctypes.byref(rows), ctypes.byref(occ), ctypes.byref(cus))
    return {"slices": S.value, "tall": tall.value, "tiles": tiles.value,
            "tile_rows": rows.value, "occupancy": occ.value, "cus": cus.value,
            "workgroups": tiles.value * S.value,
            "kernel": kernel_name(OP_TSM2R, m, k, n, dtype)}


def pin_tsm2r(m: int, k: int, n: int, dtype: int, slices: int = 0, tall: int = -1) -> None:
    """Pin the TSM2R plan of shape (m, k, n, dtype) for later calls (slices 0 /
    tall -1 leave that choice to the planner; both remove the pin)."""
    _lib.call("tsm2x_tsm2r_pin", m, k, n, dtype, slices, tall)


def unpin_tsm2r(m: int, k: int, n: int, dtype: int) -> None:
    """Remove a pinned TSM2R plan."""
    pin_tsm2r(m, k, n, dtype, 0, -1)


def timing_start() -> None:
    """Start timing every kernel launch of the library (HIP events on each
    launch's stream); earlier records are dropped."""
    _lib.call("tsm2x_timing_start")


def timing_stop() -> None:
    """Stop recording launches (the records are kept for timing_collect)."""
    _lib.call("tsm2x_timing_stop")


def timing_tag(tag: int) -> None:
    """Label later launches with ``tag`` (process-wide, all host threads)."""
    _lib.call("tsm2x_timing_tag", int(tag))


def timing_collect() -> list:
    """Wait for the recorded launches and return one dict per (kernel, tag):
    ``kernel`` (demangled, without namespace and parameters), ``tag``,
    ``launches``, ``total_ms``."""
    import ctypes
    L = _lib.lib()
    nrows = L.tsm2x_timing_collect()
    out = []
    for i in range(nrows):
        name, tag = ctypes.c_char_p(), ctypes.c_int()
        n, ms = ctypes.c_int64(), ctypes.c_double()
        if L.tsm2x_timing_row(i, ctypes.byref(name), ctypes.byref(tag), ctypes.byref(n),
                              ctypes.byref(ms)) == 0:
            out.append({"kernel": name.value.decode(), "tag": tag.value,
                        "launches": n.value, "total_ms": ms.value})
    return out


def probe_stream(kind: str, dst: torch.Tensor, src: torch.Tensor | None = None,
                 nbytes: int | None = None, blocks: int = 0) -> None:
    """Bandwidth probe (measurement support): "read" nbytes of src, "copy"
    src to dst, or "write" dst, with 16-byte non-temporal accesses."""
    kinds = {"read": 0, "copy": 1, "write": 2}
    if kind not in kinds:
        raise ValueError("kind must be read, copy or write")
    _check_device(dst)
    if src is not None:
        _check_device(src)
    if nbytes is None:
        nbytes = (src if kind == "read" else dst).numel() * \
            (src if kind == "read" else dst).element_size()
    if kind != "read" and nbytes > dst.numel() * dst.element_size():
        raise ValueError("dst is smaller than nbytes")
    if kind != "write" and (src is None or nbytes > src.numel() * src.element_size()):
        raise ValueError("src is missing or smaller than nbytes")
    if kind == "read" and dst.numel() * dst.element_size() < 16:
        raise ValueError("dst must hold at least 16 bytes")
    _lib.call("tsm2x_probe_stream", kinds[kind], src.data_ptr() if src is not None else None,
              dst.data_ptr(), int(nbytes), int(blocks), _stream())


def probe_tiles(X: torch.Tensor, O: torch.Tensor, Y: torch.Tensor | None = None,
                blocks: int = 0) -> None:
    """Bandwidth probe (measurement support): the TSM2L kernel's access
    pattern without its arithmetic, X (m x kin) read once and O (m x nout)
    written once, all column-major float64 or float32.  With Y (like X), the
    fused TSM2L backward's pattern: X and Y read, O written."""
    _check_device(X, O)
    if not (is_colmajor(X) and is_colmajor(O)) or X.shape[0] != O.shape[0] or \
            X.dtype != O.dtype:
        raise ValueError("X and O must be column-major with the same rows and dtype")
    if Y is not None:
        _check_device(Y)
        if not is_colmajor(Y) or tuple(Y.shape) != tuple(X.shape) or Y.dtype != X.dtype:
            raise ValueError("Y must be column-major with X's shape and dtype")
    _lib.call("tsm2x_probe_tiles", X.shape[0], X.shape[1], O.shape[1], X.data_ptr(), _ld(X),
              Y.data_ptr() if Y is not None else None, _ld(Y) if Y is not None else 1,
              O.data_ptr(), _ld(O), _plain_dtype(X), int(blocks), _stream())


from .autograd import TSMMatmul, matmul  # noqa: E402,F401
