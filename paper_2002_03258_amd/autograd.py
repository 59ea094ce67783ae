"""C = A*B as a torch.autograd.Function backed by the library's kernels.

Forward: TSM2R (large A) or TSM2L (tall A with k <= 32).  Backward of the
scalar loss with upstream gradient dC:  dA = dC*B^T (rowtile kernel, a TSM2L
shape) and dB = A^T*dC (tn kernel, a reduction along m split across
workgroups and finished in double).  For a TSM2L product needing both
gradients, one fused pass (tsm2l_backward) reads A and dC once.

Modes:
  "f64", "f32"            A, B, C and both gradients in that precision.
  "bf16", "bf16_split",   A is float32 and is stored for the product as
  "f16", "f16_split"      bfloat16/binary16 hi (and lo) planes, split in the
                          forward and kept for the backward; B, C, dA and dB
                          are float32.  dA = dC*B^T involves only float data
                          and runs in float.

A may also be given in its storage form, a SplitA made by ``split(A)``: the
planes are then used as they are (no split in the forward; A is read only as
its 16-bit planes) and the gradient flows to the float32 matrix they were split
from, which must not have been modified since.  This is the precision form's
intended use: A kept in HBM as its planes across calls.
"""
from __future__ import annotations

import torch

_LOWP = {"bf16": ("bf16", False), "bf16_split": ("bf16", True),
         "f16": ("f16", False), "f16_split": ("f16", True)}


def _kind(A_shape, kind: str) -> str:
    if kind in ("R", "L"):
        return kind
    m, k = A_shape
    return "L" if k <= 32 and m >= 64 * k else "R"


class TSMMatmul(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A: torch.Tensor, B: torch.Tensor, mode: str = "f32", kind: str = "auto",
                planes=None):
        from . import split, tsm2l, tsm2r
        kd = _kind(tuple(A.shape), kind)
        if mode in _LOWP:
            if A.dtype != torch.float32 or B.dtype != torch.float32:
                raise ValueError("low-precision modes take float32 A and B")
            fmt, lo = _LOWP[mode]
            if planes is not None:
                if (planes.fmt, planes.has_lo) != (fmt, lo) or planes.shape != tuple(A.shape):
                    raise ValueError("the planes do not match mode %s and A's shape" % mode)
                Aop = planes
            else:
                Aop = split(A, fmt, lo)
        elif planes is not None:
            raise ValueError("planes are only used by the low-precision modes")
        else:
            want = torch.float64 if mode == "f64" else torch.float32
            if A.dtype != want or B.dtype != want:
                raise ValueError("mode %s needs %s A and B" % (mode, want))
            Aop = A
        C = tsm2l(Aop, B) if kd == "L" else tsm2r(Aop, B)
        if mode in _LOWP:
            ctx.save_for_backward(B)
            ctx.planes = Aop     # A's stored planes (dB uses the stored values)
        else:
            ctx.save_for_backward(B, A)
            ctx.planes = None
        ctx.fused = kd == "L" and A.shape[1] <= 32 and B.shape[1] <= 32
        return C

    @staticmethod
    def backward(ctx, dC: torch.Tensor):
        from . import grad_a, grad_b, tsm2l_backward
        saved = ctx.saved_tensors
        B = saved[0]
        Aop = ctx.planes if ctx.planes is not None else saved[1]
        dA = dB = None
        dC = dC.to(B.dtype)
        if ctx.fused and ctx.needs_input_grad[0] and ctx.needs_input_grad[1]:
            # one pass over A and dC for both gradients of a TSM2L product
            dA, dB = tsm2l_backward(Aop, B, dC)
            return dA, dB, None, None, None
        if ctx.needs_input_grad[0]:
            dA = grad_a(dC, B)
        if ctx.needs_input_grad[1]:
            dB = grad_b(Aop, dC)
        return dA, dB, None, None, None


def matmul(A, B: torch.Tensor, mode: str | None = None, kind: str = "auto") -> torch.Tensor:
    """Differentiable C = A*B.  mode defaults to the dtype of A ("f64" or
    "f32"), or for a SplitA A to its storage form ("bf16_split", ...); kind
    "R" (TSM2R), "L" (TSM2L) or "auto" (by shape).  For a SplitA the gradient
    with respect to A goes to the float32 matrix it was split from."""
    from . import SplitA
    if isinstance(A, SplitA):
        own = A.fmt + ("_split" if A.has_lo else "")
        if mode is None:
            mode = own
        if mode != own:
            raise ValueError("a %s SplitA cannot run in mode %s" % (own, mode))
        return TSMMatmul.apply(A.check_source(), B, mode, kind, A)
    if mode is None:
        mode = "f64" if A.dtype == torch.float64 else "f32"
    return TSMMatmul.apply(A, B, mode, kind)
