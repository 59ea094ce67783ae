"""Precision form: the split kernel against the oracle's split (bit-exact),
and TSM2R on bf16/f16 hi(+lo) planes against the FP64 oracle on the stored
values (arithmetic error) and on the float values (total error)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2002_03258_amd as tsm
import seeded_inputs as si

from helpers import dev_matrix, err, host_matrix, host_rows, sample_rows, to_np

pytestmark = pytest.mark.gpu

FMTS = [("bf16", oracle.BF16), ("f16", oracle.F16)]
# normwise error bound against the oracle on the stored values hi (+ lo):
# float accumulation alone (every product of hi (+ lo) and B above 2^-24
# |a||b| is kept, each pinned exactly below).  Measured at most 1.1e-6 (A
# 32768^2, n = 32; dB over 2^23 rows); a dropped hi*B3 measured 2.3e-6.
TOL_STORED = 3e-6
# componentwise, max |C - C_ref| / (|A||B|), against the stored values: the
# float sums' error relative to the products' magnitudes; bounded by
# gamma_L = L u for L sequential float additions (L <= 32 per MFMA chain
# step); measured at most 2.3e-8 at full size
TOL_CW_STORED = 1e-6
# against the float A: the storage error of the form
TOL_VALUE = {("bf16", False): 4e-3, ("f16", False): 5e-4, ("bf16", True): 2e-5,
             ("f16", True): 2e-5}


def _planes_np(S):
    hi = S.hi.contiguous().view(torch.int16).cpu().numpy().view(np.uint16)
    lo = S.lo.contiguous().view(torch.int16).cpu().numpy().view(np.uint16) if S.has_lo else None
    return hi, lo


@pytest.mark.parametrize("fmt,code", FMTS)
@pytest.mark.parametrize("m,k", [(1, 1), (37, 5), (1000, 333), (4099, 64)])
def test_split_matches_oracle(dev, fmt, code, m, k):
    A = dev_matrix(10 + m, si.STREAM_A, m, k, torch.float32, dev)
    if m > 10:   # magnitudes from tiny to large, and specials
        A[3, 0] = float("nan")
        A[4, 0] = float("inf")
        A[5, 0] = -0.0
        A[6, 0] = 1e-30
        A[7, 0] = 3.0e4 if fmt == "f16" else 3.0e38
        A[8, 0] = 2.0 ** -20
    S = tsm.split(A, fmt, lo=True)
    hi, lo = _planes_np(S)
    Ah = A.cpu().numpy()
    rhi, rlo = oracle.split(np.asfortranarray(Ah), code)
    assert np.array_equal(hi, rhi)
    assert np.array_equal(lo, rlo)
    S1 = tsm.split(A, fmt, lo=False)
    assert S1.lo is None
    assert torch.equal(S1.hi.contiguous().view(torch.int16), S.hi.contiguous().view(torch.int16))


def _stored_value(A32_np, code, with_lo):
    hi, lo = oracle.split(np.asfortranarray(A32_np.astype(np.float32)), code)
    v = oracle.decode_plane(hi, code)
    if with_lo:
        v = v + oracle.decode_plane(lo, code)
    return v


@pytest.mark.parametrize("fmt,code", FMTS)
@pytest.mark.parametrize("with_lo", [False, True])
@pytest.mark.parametrize("m,k,n", [(1, 1, 1), (7, 5, 3), (300, 1000, 16), (1000, 3000, 32),
                                   (4133, 2500, 8), (255, 4097, 17), (2048, 777, 12)])
def test_tsm2r_lowp_small(dev, fmt, code, with_lo, m, k, n):
    seed = 500 + m + k + n
    A = dev_matrix(seed, si.STREAM_A, m, k, torch.float32, dev)
    B = dev_matrix(seed, si.STREAM_B, k, n, torch.float32, dev)
    C = tsm.tsm2r(tsm.split(A, fmt, lo=with_lo), B)
    Ah = host_matrix(seed, si.STREAM_A, m, k, torch.float32)
    Bh = host_matrix(seed, si.STREAM_B, k, n, torch.float32)
    ref_stored = oracle.matmul(_stored_value(Ah, code, with_lo), Bh)
    ref_value = oracle.matmul(Ah, Bh)
    e_s, e_v = err(to_np(C), ref_stored), err(to_np(C), ref_value)
    assert e_s <= TOL_STORED, (e_s, e_v)
    assert e_v <= TOL_VALUE[(fmt, with_lo)], (e_s, e_v)


@pytest.mark.parametrize("fmt,code", FMTS)
def test_tsm2r_lowp_integer_bit_exact(dev, fmt, code):
    """Integer A with |a| <= 64 and B with |b| <= 8 are exact in both formats
    (lo = 0, B = B1) and k*64*8 < 2^24 keeps float accumulation exact."""
    m, k, n = 2000, 4096, 16
    A = dev_matrix(7, si.STREAM_A, m, k, torch.float32, dev, dist="int", r=64)
    B = dev_matrix(7, si.STREAM_B, k, n, torch.float32, dev, dist="int", r=8)
    for with_lo in (False, True):
        C = to_np(tsm.tsm2r(tsm.split(A, fmt, lo=with_lo), B))
        ref = oracle.matmul(host_matrix(7, si.STREAM_A, m, k, torch.float32, dist="int", r=64),
                            host_matrix(7, si.STREAM_B, k, n, torch.float32, dist="int", r=8))
        assert np.array_equal(C, ref)


@pytest.mark.parametrize("fmt,code", FMTS)
def test_tsm2r_lowp_deterministic(dev, fmt, code):
    A = dev_matrix(8, si.STREAM_A, 3000, 20000, torch.float32, dev)
    B = dev_matrix(8, si.STREAM_B, 20000, 32, torch.float32, dev)
    S = tsm.split(A, fmt)
    assert torch.equal(tsm.tsm2r(S, B).clone(), tsm.tsm2r(S, B))


@pytest.mark.parametrize("fmt,code", FMTS)
def test_tsm2r_lowp_full_size_sampled(dev, fmt, code):
    """A 32768 x 32768 stored single and split, B 32768 x n, n in {8, 16, 32}."""
    seed = si.config_seed(3)
    m = k = 32768
    A = dev_matrix(seed, si.STREAM_A, m, k, torch.float32, dev)
    rows = sample_rows(m, 24, seed=3)
    Ar = host_rows(seed, si.STREAM_A, m, k, rows, torch.float32)
    for with_lo in (False, True):
        S = tsm.split(A, fmt, lo=with_lo)
        stored = _stored_value(Ar, code, with_lo)
        for n in (8, 16, 32):
            B = dev_matrix(seed + n, si.STREAM_B, k, n, torch.float32, dev)
            Bh = host_matrix(seed + n, si.STREAM_B, k, n, torch.float32)
            Cs = to_np(tsm.tsm2r(S, B)[rows])
            ref_s = oracle.matmul(stored, Bh)
            e_s = err(Cs, ref_s)
            e_v = err(Cs, oracle.matmul(Ar, Bh))
            cw = oracle.componentwise_error(Cs, ref_s, stored, Bh)
            print(fmt, "split" if with_lo else "single", n,
                  "err stored %.2e (componentwise %.2e) value %.2e" % (e_s, cw, e_v))
            assert e_s <= TOL_STORED and e_v <= TOL_VALUE[(fmt, with_lo)]
            assert cw <= TOL_CW_STORED
        del S
    del A
    torch.cuda.empty_cache()


# TSM2L and dB = A^T * dC on the planes: the planes are widened to float (hi + lo
# is exact in float) and multiplied on the float matrix cores, so the error
# against the stored values is that of float accumulation over k (TSM2L) or
# m (dB) terms.
@pytest.mark.parametrize("fmt,code", FMTS)
@pytest.mark.parametrize("with_lo", [False, True])
@pytest.mark.parametrize("m,k,n", [(1, 1, 1), (7, 5, 3), (1000, 8, 8), (4133, 16, 16),
                                   (2049, 32, 32), (300, 17, 5), (5000, 3, 29), (129, 9, 17)])
def test_tsm2l_lowp_small(dev, fmt, code, with_lo, m, k, n):
    seed = 700 + m + k + n
    A = dev_matrix(seed, si.STREAM_A, m, k, torch.float32, dev)
    B = dev_matrix(seed, si.STREAM_B, k, n, torch.float32, dev)
    C = tsm.tsm2l(tsm.split(A, fmt, lo=with_lo), B)
    Ah = host_matrix(seed, si.STREAM_A, m, k, torch.float32)
    Bh = host_matrix(seed, si.STREAM_B, k, n, torch.float32)
    e_s = err(to_np(C), oracle.matmul(_stored_value(Ah, code, with_lo), Bh))
    e_v = err(to_np(C), oracle.matmul(Ah, Bh))
    assert e_s <= TOL_STORED, (e_s, e_v)
    assert e_v <= TOL_VALUE[(fmt, with_lo)], (e_s, e_v)


@pytest.mark.parametrize("fmt,code", FMTS)
@pytest.mark.parametrize("with_lo", [False, True])
@pytest.mark.parametrize("m,k,n", [(1, 1, 1), (7, 5, 3), (1000, 16, 16), (5000, 33, 8),
                                   (3000, 17, 20), (130, 40, 32), (70001, 16, 16)])
def test_grad_b_lowp_small(dev, fmt, code, with_lo, m, k, n):
    seed = 900 + m + k + n
    A = dev_matrix(seed, si.STREAM_A, m, k, torch.float32, dev)
    dC = dev_matrix(seed, si.STREAM_DC, m, n, torch.float32, dev, dist="normal")
    dB = tsm.grad_b(tsm.split(A, fmt, lo=with_lo), dC)
    Ah = host_matrix(seed, si.STREAM_A, m, k, torch.float32)
    dCh = host_matrix(seed, si.STREAM_DC, m, n, torch.float32, dist="normal")
    e_s = err(to_np(dB), oracle.matmul(_stored_value(Ah, code, with_lo).T, dCh))
    e_v = err(to_np(dB), oracle.matmul(Ah.T, dCh))
    assert e_s <= TOL_STORED, (e_s, e_v)
    assert e_v <= TOL_VALUE[(fmt, with_lo)], (e_s, e_v)


@pytest.mark.parametrize("fmt,code", FMTS)
def test_tsm2l_grad_b_lowp_integer_bit_exact(dev, fmt, code):
    """Integer A (|a| <= 64, exact in both formats, lo = 0) and B, dC with
    |b| <= 8: every product and partial sum is an integer below 2^24."""
    m, k, n = 9000, 16, 16
    A = dev_matrix(11, si.STREAM_A, m, k, torch.float32, dev, dist="int", r=64)
    B = dev_matrix(11, si.STREAM_B, k, n, torch.float32, dev, dist="int", r=8)
    dC = dev_matrix(11, si.STREAM_DC, m, n, torch.float32, dev, dist="int", r=8)
    Ah = host_matrix(11, si.STREAM_A, m, k, torch.float32, dist="int", r=64)
    Bh = host_matrix(11, si.STREAM_B, k, n, torch.float32, dist="int", r=8)
    dCh = host_matrix(11, si.STREAM_DC, m, n, torch.float32, dist="int", r=8)
    for with_lo in (False, True):
        S = tsm.split(A, fmt, lo=with_lo)
        assert np.array_equal(to_np(tsm.tsm2l(S, B)), oracle.matmul(Ah, Bh))
        assert np.array_equal(to_np(tsm.grad_b(S, dC)), oracle.matmul(Ah.T, dCh))


@pytest.mark.parametrize("fmt,code", FMTS)
def test_tsm2l_grad_b_lowp_deterministic(dev, fmt, code):
    A = dev_matrix(12, si.STREAM_A, 300000, 16, torch.float32, dev)
    B = dev_matrix(12, si.STREAM_B, 16, 16, torch.float32, dev)
    dC = dev_matrix(12, si.STREAM_DC, 300000, 16, torch.float32, dev, dist="normal")
    S = tsm.split(A, fmt)
    assert torch.equal(tsm.tsm2l(S, B).clone(), tsm.tsm2l(S, B))
    assert torch.equal(tsm.grad_b(S, dC).clone(), tsm.grad_b(S, dC))


@pytest.mark.parametrize("fmt,code", FMTS)
@pytest.mark.parametrize("with_lo", [False, True])
@pytest.mark.parametrize("m,k,n", [(1, 1, 1), (1000, 16, 16), (4133, 9, 30), (70001, 32, 8),
                                   (300000, 16, 16)])
def test_fused_backward_lowp(dev, fmt, code, with_lo, m, k, n):
    """dA = dC*B^T and dB = planes^T*dC in one pass over the planes and dC."""
    seed = 1900 + m + k + n
    A = dev_matrix(seed, si.STREAM_A, m, k, torch.float32, dev)
    B = dev_matrix(seed, si.STREAM_B, k, n, torch.float32, dev)
    dC = dev_matrix(seed, si.STREAM_DC, m, n, torch.float32, dev, dist="normal")
    S = tsm.split(A, fmt, lo=with_lo)
    dA, dB = tsm.tsm2l_backward(S, B, dC)
    Ah = host_matrix(seed, si.STREAM_A, m, k, torch.float32)
    Bh = host_matrix(seed, si.STREAM_B, k, n, torch.float32)
    dCh = host_matrix(seed, si.STREAM_DC, m, n, torch.float32, dist="normal")
    assert err(to_np(dA), oracle.matmul(dCh, Bh.T)) <= TOL_STORED
    assert err(to_np(dB), oracle.matmul(_stored_value(Ah, code, with_lo).T, dCh)) <= TOL_STORED
    # the same as the two separate kernels
    assert err(to_np(dB), to_np(tsm.grad_b(S, dC))) <= TOL_STORED


# ------------------------------------------------------------------------
# Pins of the products the precision form keeps.  On random data a dropped
# term below ~2^-16 hides inside the float accumulation error, so each term
# is pinned by a case where it alone decides exact results: rows of A with one
# nonzero entry, so that every output is a single product and float
# accumulation adds only zeros.
# ------------------------------------------------------------------------
def _one_hot_rows(m, k, value, seed):
    """m x k float32, row i holds +-value in column i % k, zero elsewhere."""
    sign = np.where(si.values(seed, si.STREAM_V, torch.arange(m), dist="int", r=1).numpy() < 0,
                    -1.0, 1.0)
    A = np.zeros((m, k), dtype=np.float32)
    A[np.arange(m), np.arange(m) % k] = (sign * value).astype(np.float32)
    return A


def _dev(x, dev):
    return torch.from_numpy(np.asfortranarray(x)).to(dev).t().contiguous().t()


@pytest.mark.parametrize("fmt,code", FMTS)
@pytest.mark.parametrize("kind,m,k,n", [("R", 1000, 777, 16), ("R", 300, 4100, 32),
                                        ("L", 5000, 16, 16), ("L", 4133, 32, 7)])
def test_every_term_of_B_is_kept(dev, fmt, code, kind, m, k, n):
    """A one-hot with entries +-1 (hi = +-1, lo = 0) and B in [1, 2) with full
    24-bit significands, so that B needs all three 16-bit terms (bf16: 8 + 8
    + 8 bits; binary16: 11 + 11 + 2): every output must be exactly +-B[j, p]
    in both forms.  Dropping hi*B3 (or hi*B2) changes the last bits."""
    A = _one_hot_rows(m, k, 1.0, 31 + m)
    B = (1.0 + np.abs(si.matrix(37 + k, si.STREAM_B, k, n).numpy())).astype(np.float32)
    assert np.any(B != B.astype(np.float64).round(4))          # not short significands
    want = (A.astype(np.float64) @ B.astype(np.float64))
    Ad, Bd = _dev(A, dev), _dev(B, dev)
    for with_lo in (False, True):
        S = tsm.split(Ad, fmt, lo=with_lo)
        C = tsm.tsm2l(S, Bd) if kind == "L" else tsm.tsm2r(S, Bd)
        assert np.array_equal(to_np(C), want), (fmt, with_lo)


@pytest.mark.parametrize("fmt,code", FMTS)
@pytest.mark.parametrize("kind,m,k,n", [("R", 1000, 777, 16), ("R", 300, 4100, 32),
                                        ("L", 5000, 16, 16), ("L", 4133, 32, 7)])
def test_lo_plane_terms_are_kept(dev, fmt, code, kind, m, k, n):
    """A one-hot with entries +-a, a = 1 + 2^-8 (bf16) or 1 + 2^-11 (binary16):
    hi = 1 and lo = 2^-8 (2^-11).  B = 1 + r*2^-15 (1 + r*2^-12), so that B
    has two nonzero terms and a*b is exact in float.  The split form must give
    exactly +-a*b (every one of hi*B1, hi*B2, lo*B1, lo*B2 kept), the single
    form exactly +-b (its stored value is hi = 1)."""
    a, step, rmax = (1 + 2.0 ** -8, 2.0 ** -15, 1 << 14) if fmt == "bf16" else \
        (1 + 2.0 ** -11, 2.0 ** -12, 1 << 11)
    A = _one_hot_rows(m, k, a, 41 + m)
    r = si.values(43 + k, si.STREAM_B, torch.arange(k * n), dist="int", r=rmax).numpy()
    B = (1.0 + np.abs(r).reshape(n, k).T % rmax * step).astype(np.float32)
    hi, lo = oracle.split(np.asfortranarray(A), code)
    assert np.all(oracle.decode_plane(lo, code)[A != 0] != 0)
    Ad, Bd = _dev(A, dev), _dev(B, dev)
    want_split = A.astype(np.float64) @ B.astype(np.float64)
    assert np.array_equal(want_split.astype(np.float32).astype(np.float64), want_split)
    want_single = np.sign(A).astype(np.float64) @ B.astype(np.float64)
    for with_lo, want in ((True, want_split), (False, want_single)):
        S = tsm.split(Ad, fmt, lo=with_lo)
        C = tsm.tsm2l(S, Bd) if kind == "L" else tsm.tsm2r(S, Bd)
        assert np.array_equal(to_np(C), want), (fmt, with_lo)


@pytest.mark.parametrize("fmt,code", FMTS)
@pytest.mark.parametrize("m,n", [(24, 8), (64, 8), (517, 16), (2000, 32)])
def test_grad_b_keeps_the_lo_plane(dev, fmt, code, m, n):
    """dB = A^T*dC on the planes with A = diag(+-a) (m = k): dB[j, p] =
    +-a*dC[j, p] exactly for the split form, +-dC[j, p] for the single form;
    the same through the fused backward."""
    a, step, rmax = (1 + 2.0 ** -8, 2.0 ** -15, 1 << 14) if fmt == "bf16" else \
        (1 + 2.0 ** -11, 2.0 ** -12, 1 << 11)
    A = _one_hot_rows(m, m, a, 47 + m)
    r = si.values(53 + m, si.STREAM_DC, torch.arange(m * n), dist="int", r=rmax).numpy()
    dC = (1.0 + np.abs(r).reshape(n, m).T % rmax * step).astype(np.float32)
    Ad, dCd = _dev(A, dev), _dev(dC, dev)
    for with_lo in (True, False):
        want = (A if with_lo else np.sign(A)).astype(np.float64).T @ dC.astype(np.float64)
        S = tsm.split(Ad, fmt, lo=with_lo)
        assert np.array_equal(to_np(tsm.grad_b(S, dCd)), want), (fmt, with_lo, "tn")
        if m <= 32:
            B = _dev(np.ones((m, n), dtype=np.float32), dev)
            _, dB = tsm.tsm2l_backward(S, B, dCd)
            assert np.array_equal(to_np(dB), want), (fmt, with_lo, "fused")


@pytest.mark.parametrize("fmt,code", FMTS)
@pytest.mark.parametrize("m,n", [(2048, 8), (2048, 16), (2048, 32), (2000, 24), (2000, 16)])
def test_grad_b_keeps_every_term_of_dC(dev, fmt, code, m, n):
    """dB = A^T*dC with A = diag(+-1) (hi = +-1, lo = 0) and dC in [1, 2) with
    full 24-bit significands: dB[j, p] = +-dC[j, p] exactly in both forms.
    On the bf16 matrix-core path (single form; split form for n <= 16) dC
    enters as three bf16 terms (8 + 8 + 8 bits), so dropping or misplacing
    any of them changes the last bits.  m = 2048 puts every wavefront on the straight-line paths
    (four 16-column tiles per workgroup for n <= 16); m = 2000 leaves
    ragged row ranges and a ragged last column group to the bounds-checked
    step."""
    A = _one_hot_rows(m, m, 1.0, 59 + m)
    dC = (1.0 + np.abs(si.matrix(61 + n, si.STREAM_DC, m, n).numpy())).astype(np.float32)
    assert np.any(dC != dC.astype(np.float64).round(4))        # not short significands
    want = A.astype(np.float64).T @ dC.astype(np.float64)
    Ad, dCd = _dev(A, dev), _dev(dC, dev)
    for with_lo in (False, True):
        S = tsm.split(Ad, fmt, lo=with_lo)
        assert np.array_equal(to_np(tsm.grad_b(S, dCd)), want), (fmt, with_lo)
