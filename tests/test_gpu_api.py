"""Binding-level behaviour on the GPU: argument checks that must refuse a call
before any launch (dtype, shape and `out` mismatches of the gradients), the
autograd Function on a SplitA (the precision form's storage kept across
calls), the per-launch timing of the library, and the bandwidth probes."""
import numpy as np
import pytest
import torch

import oracle
import paper_2002_03258_amd as tsm
import seeded_inputs as si

from helpers import dev_matrix, to_np

pytestmark = pytest.mark.gpu


def _m(rows, cols, dt, dev, stream=si.STREAM_A, seed=11):
    return dev_matrix(seed, stream, rows, cols, dt, dev)


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_gradient_calls_refuse_mismatched_operands(dev, dt):
    other = torch.float32 if dt == torch.float64 else torch.float64
    m, k, n = 300, 12, 5
    A, B, dC = _m(m, k, dt, dev), _m(k, n, dt, dev), _m(m, n, dt, dev)
    bad = [
        lambda: tsm.grad_a(dC, _m(k, n, other, dev)),                 # dtype of B
        lambda: tsm.grad_a(dC, _m(k, n - 1, dt, dev)),                # B narrower than dC
        lambda: tsm.grad_a(dC, B, out=tsm.empty_colmajor(m - 1, k, dt, dev)),
        lambda: tsm.grad_a(dC, B, out=tsm.empty_colmajor(m, k, other, dev)),
        lambda: tsm.grad_a(dC, B, out=torch.empty(m, k, dtype=dt, device=dev)),  # row-major out
        lambda: tsm.grad_b(A, _m(m - 1, n, dt, dev)),                 # dC shorter than A
        lambda: tsm.grad_b(A, _m(m, n, other, dev)),
        lambda: tsm.grad_b(A, dC, out=tsm.empty_colmajor(k, n - 1, dt, dev)),
        lambda: tsm.tsm2l_backward(A, _m(k, n, other, dev), dC),
        lambda: tsm.tsm2l_backward(A, _m(k + 1, n, dt, dev), dC),
        lambda: tsm.tsm2l_backward(A, B, _m(m - 1, n, dt, dev)),
        lambda: tsm.tsm2l_backward(A, B, _m(m, n + 1, dt, dev)),
        lambda: tsm.tsm2r(A, B, out=tsm.empty_colmajor(m, n, other, dev)),
    ]
    for i, f in enumerate(bad):
        with pytest.raises(ValueError):
            f()
    torch.cuda.synchronize()


def test_split_form_gradient_calls_refuse_mismatched_operands(dev):
    m, k, n = 300, 12, 5
    A = _m(m, k, torch.float32, dev)
    S = tsm.split(A, "bf16", lo=True)
    dC = _m(m, n, torch.float32, dev)
    with pytest.raises(ValueError):
        tsm.grad_b(S, dC.double())
    with pytest.raises(ValueError):
        tsm.grad_b(S, _m(m + 1, n, torch.float32, dev))
    with pytest.raises(ValueError):
        tsm.grad_b(S, dC, out=tsm.empty_colmajor(k, n, torch.float64, dev))
    with pytest.raises(ValueError):
        tsm.tsm2l_backward(S, _m(k, n, torch.float32, dev), dC.double())
    with pytest.raises(ValueError):
        tsm.split(A.double())


@pytest.mark.parametrize("kind,shape", [("L", (5000, 16, 16)), ("R", (700, 1500, 8))])
def test_matmul_on_stored_planes(dev, kind, shape):
    """matmul(SplitA, B) runs on the planes as they are (no new split), equals
    the library's product of the same planes bit for bit, and sends dA to the
    float matrix the planes came from."""
    m, k, n = shape
    A = _m(m, k, torch.float32, dev).requires_grad_()
    B = _m(k, n, torch.float32, dev, stream=si.STREAM_B).requires_grad_()
    dC = dev_matrix(5, si.STREAM_DC, m, n, torch.float32, dev, dist="normal")
    S = tsm.split(A, "bf16", lo=True)
    assert S.source is A
    C = tsm.matmul(S, B, kind=kind)
    dA, dB = torch.autograd.grad(C, (A, B), dC)
    ref = tsm.tsm2l(S, B.detach()) if kind == "L" else tsm.tsm2r(S, B.detach())
    assert torch.equal(C, ref)
    # the same as the mode that splits inside the forward
    C2 = tsm.matmul(A, B, "bf16_split", kind)
    dA2, dB2 = torch.autograd.grad(C2, (A, B), dC)
    assert torch.equal(C, C2) and torch.equal(dA, dA2) and torch.equal(dB, dB2)
    # dA = dC B^T involves no stored value
    assert oracle.normwise_error(to_np(dA), to_np(dC) @ to_np(B).T) <= 1e-5
    with pytest.raises(ValueError):
        tsm.matmul(S, B, mode="bf16")
    with torch.no_grad():
        A.add_(1.0)                 # the planes no longer hold A's values
    with pytest.raises(ValueError):
        tsm.matmul(S, B)


def test_launch_timing_names_and_tags(dev):
    m, k, n = 20480, 20480, 8
    A = _m(m, k, torch.float64, dev)
    B = _m(k, n, torch.float64, dev, stream=si.STREAM_B)
    C = tsm.empty_colmajor(m, n, torch.float64, dev)
    tsm.tsm2r(A, B, out=C)
    torch.cuda.synchronize()
    tsm.timing_start()
    tsm.timing_tag(7)
    for _ in range(3):
        tsm.tsm2r(A, B, out=C)
    tsm.timing_tag(8)
    tsm.tsm2l(A[:, :16], B[:16], out=C)
    tsm.timing_tag(0)
    tsm.timing_stop()
    tsm.tsm2r(A, B, out=C)              # not recorded
    rows = tsm.timing_collect()
    name = tsm.kernel_name(tsm.OP_TSM2R, m, k, n, tsm.F64)
    main = [r for r in rows if r["kernel"] == name]
    assert len(main) == 1 and main[0]["tag"] == 7 and main[0]["launches"] == 3, (name, rows)
    # 3 x 2.7 GB in well under a second, and more than 0.1 ms each
    assert 0.3 < main[0]["total_ms"] < 1000
    assert any(r["kernel"].startswith("rowtile_kernel<double") and r["tag"] == 8 for r in rows)
    assert all(r["tag"] in (7, 8) for r in rows)
    # collecting again adds nothing; a new start clears the rows
    assert tsm.timing_collect() == rows
    tsm.timing_start()
    tsm.timing_stop()
    assert tsm.timing_collect() == []


def _tile_source_column(c, kin, es, nout):
    """The input column the tile probe stores into output column c (the
    rowtile store order: column 16 t + mrow(kk, rr) from the lane's run of
    input column 4 ((4 t + rr) % KS) + kk)."""
    KS = 2 if kin <= 8 else (4 if kin <= 16 else 8)
    t, j = divmod(c, 16)
    if es == 4:
        kk, rr = divmod(j, 4)          # mrow = 4 kk + rr
    else:
        rr, kk = divmod(j, 4)          # mrow = kk + 4 rr
    return 4 * ((4 * t + rr) % KS) + kk


@pytest.mark.parametrize("two", [False, True])
@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
@pytest.mark.parametrize("m,kin,nout", [(1000, 16, 16), (777, 8, 8), (4099, 32, 32),
                                        (513, 16, 32), (300, 5, 3)])
def test_tile_probe_moves_every_element(dev, dt, m, kin, nout, two):
    X = _m(m, kin, dt, dev)
    Y = _m(m, kin, dt, dev, stream=si.STREAM_B) if two else None
    O = tsm.empty_colmajor(m, nout, dt, dev)
    O.fill_(float("nan"))
    tsm.probe_tiles(X, O, Y=Y)
    Xh, Oh = to_np(X), to_np(O)
    if two:
        Xh = (X.cpu() + Y.cpu()).to(torch.float64).numpy()   # the add in X's own precision
    es = 8 if dt == torch.float64 else 4
    for c in range(nout):
        src = _tile_source_column(c, kin, es, nout)
        want = Xh[:, src] if src < kin else np.zeros(m)
        assert np.array_equal(Oh[:, c], want), (c, src)


def test_stream_probes(dev):
    nb = (1 << 20) + 48
    src = torch.randint(0, 255, (nb,), dtype=torch.uint8, device=dev)
    dst = torch.zeros(nb, dtype=torch.uint8, device=dev)
    tsm.probe_stream("copy", dst, src)
    assert torch.equal(dst, src)
    w = torch.zeros(nb // 4, dtype=torch.int32, device=dev)
    tsm.probe_stream("write", w)
    assert bool((w != 0).any())
    before = dst.clone()
    tsm.probe_stream("read", dst, src)
    torch.cuda.synchronize()
    assert torch.equal(dst, before) or int((dst != before).sum()) <= 16
    with pytest.raises(tsm.TSMError):
        tsm.probe_stream("copy", dst, src, nbytes=nb - 8)        # not a multiple of 16
    with pytest.raises(ValueError):
        tsm.probe_stream("copy", dst[: nb // 2], src, nbytes=nb)
