"""The autograd Function: gradcheck in double on tiny shapes, and at the
full autograd workloads (TSM2L A 8388608 x 16, B 16 x 16; TSM2R A 16384^2,
B 16384 x 8; dC ~ N(0, 1)) C, dA, dB against the FP64 oracle plus the
adjoint identity <dC, V*B> = <dA, V> and <dC, A*W> = <dB, W>, which a
finite difference of the bilinear loss reduces to."""
import numpy as np
import pytest
import torch

import oracle
import paper_2002_03258_amd as tsm
import seeded_inputs as si

from helpers import dev_matrix, err, host_matrix, host_rows, sample_rows, to_np

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind,shape", [("R", (9, 70, 3)), ("L", (300, 5, 4)), ("R", (33, 33, 17)),
                                        ("L", (257, 16, 16))])
def test_gradcheck_f64(dev, kind, shape):
    """C is linear in each input, so the central difference has no truncation
    error; eps only has to keep |C| * 2^-53 / eps well below atol."""
    m, k, n = shape
    g = torch.Generator(device="cpu").manual_seed(m + k + n)
    A = torch.rand(m, k, dtype=torch.float64, generator=g).to(dev).requires_grad_()
    B = torch.rand(k, n, dtype=torch.float64, generator=g).to(dev).requires_grad_()
    assert torch.autograd.gradcheck(lambda a, b: tsm.matmul(a, b, "f64", kind), (A, B),
                                    eps=1e-3, atol=1e-9, rtol=1e-7)


def _stored(A32, mode):
    fmt = oracle.BF16 if mode.startswith("bf16") else oracle.F16
    hi, lo = oracle.split(np.asfortranarray(A32.astype(np.float32)), fmt)
    v = oracle.decode_plane(hi, fmt)
    if mode.endswith("split"):
        v = v + oracle.decode_plane(lo, fmt)
    return v


TOL = {"f32": 1e-5, "bf16_split": 3e-6, "f64": 1e-13}
TOL_VALUE = {"f32": 1e-5, "bf16_split": 2e-5, "f64": 1e-13}
# componentwise error, max |X - X_ref| / (|P||Q|) for X_ref = P*Q: bounded by
# gamma_L for L sequential additions in the arithmetic's precision; measured
# at most 4.7e-16 (f64) and 2e-7 (float accumulation)
TOL_CW = {"f32": 1e-6, "bf16_split": 1e-6, "f64": 1e-14}


@pytest.mark.parametrize("mode", ["f32", "bf16_split", "f64"])
@pytest.mark.parametrize("kind,shape", [("L", (8388608, 16, 16)), ("R", (16384, 16384, 8))])
def test_autograd_full_size(dev, mode, kind, shape):
    m, k, n = shape
    seed = si.config_seed(4)
    dt = torch.float64 if mode == "f64" else torch.float32
    A = dev_matrix(seed, si.STREAM_A, m, k, dt, dev).requires_grad_()
    B = dev_matrix(seed, si.STREAM_B, k, n, dt, dev).requires_grad_()
    dC = dev_matrix(seed, si.STREAM_DC, m, n, dt, dev, dist="normal")
    C = tsm.matmul(A, B, mode, kind)
    C.backward(dC)
    dA, dB = A.grad, B.grad

    rows = sample_rows(m, 32, seed=kind == "L")
    Ar = host_rows(seed, si.STREAM_A, m, k, rows, dt)
    Bh = host_matrix(seed, si.STREAM_B, k, n, dt)
    dCr = host_rows(seed, si.STREAM_DC, m, n, rows, dt, dist="normal")
    Aop = _stored(Ar, mode) if mode == "bf16_split" else Ar
    e_c = err(to_np(C[rows]), oracle.matmul(Aop, Bh))
    e_cv = err(to_np(C[rows]), oracle.matmul(Ar, Bh))
    e_a = err(to_np(dA[rows]), oracle.matmul(dCr, Bh.T))
    cw_c = oracle.componentwise_error(to_np(C[rows]), oracle.matmul(Aop, Bh), Aop, Bh)
    cw_a = oracle.componentwise_error(to_np(dA[rows]), oracle.matmul(dCr, Bh.T), dCr, Bh.T)
    # dB needs every row of A and dC: the device inputs come from the same
    # counter-based generator (checked bit-identical against the host one)
    cols = sample_rows(k, 8, seed=1)
    Acols = A.detach()[:, cols].double().cpu().numpy()
    assert np.array_equal(Acols[rows], Ar[:, cols])
    if mode == "bf16_split":
        Acols = _stored(Acols.astype(np.float32), mode)
    dCh = np.ascontiguousarray(dC.double().cpu().numpy())    # row-major: one pass per row
    assert np.array_equal(dCh[rows], dCr)
    e_b = err(to_np(dB[cols]), oracle.matmul(Acols.T, dCh))
    cw_b = oracle.componentwise_error(to_np(dB[cols]), oracle.matmul(Acols.T, dCh), Acols.T, dCh)
    print(mode, kind, "err C %.2e (value %.2e) dA %.2e dB %.2e; componentwise %.2e %.2e %.2e"
          % (e_c, e_cv, e_a, e_b, cw_c, cw_a, cw_b))
    assert e_c <= TOL[mode] and e_cv <= TOL_VALUE[mode]
    assert e_a <= TOL[mode] and e_b <= TOL[mode]
    assert max(cw_c, cw_a, cw_b) <= TOL_CW[mode]

    # adjoint identities (the exact directional derivatives of the bilinear loss)
    V = dev_matrix(seed, si.STREAM_V, m, k, dt, dev, dist="normal")
    W = dev_matrix(seed, si.STREAM_W, k, n, dt, dev, dist="normal")
    with torch.no_grad():
        fdA = float((dC.double() * tsm.matmul(V, B.detach(), "f64" if mode == "f64" else "f32",
                                               kind).double()).sum())
        fdB = float((dC.double() * tsm.matmul(A.detach(), W, "f64" if mode == "f64" else "f32",
                                               kind).double()).sum())
        gA = float((dA.double() * V.double()).sum())
        gB = float((dB.double() * W.double()).sum())
    scale_a = float((dA.double().abs() * V.double().abs()).sum())
    scale_b = float((dB.double().abs() * W.double().abs()).sum())
    assert abs(fdA - gA) <= 10 * TOL[mode] * scale_a
    if mode != "bf16_split":
        assert abs(fdB - gB) <= 10 * TOL[mode] * scale_b
    del A, B, dC, C, dA, dB, V, W
    torch.cuda.empty_cache()
