"""The seeded counter-based generator: published SplitMix64 values,
row sampling equal to full generation, ranges and moments."""
import torch

import seeded_inputs as si


def test_splitmix64_published_vector():
    # SplitMix64 seeded with 0: the first three outputs.
    expect = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    # the states GAMMA, 2*GAMMA, 3*GAMMA, formed by wrapping int64 arithmetic
    st = torch.tensor([1, 2, 3], dtype=torch.int64) * si.GAMMA
    got = si._mix(st)
    assert [int(x) & ((1 << 64) - 1) for x in got] == expect


def test_matrix_rows_equal_full_generation():
    for dist in ("uniform", "normal", "int"):
        A = si.matrix(5, si.STREAM_A, 37, 11, dist=dist)
        rows = [0, 5, 36, 17]
        R = si.matrix_rows(5, si.STREAM_A, 37, 11, rows, dist=dist)
        assert torch.equal(A[rows, :], R)


def test_matrix_cols_equal_full_generation():
    A = si.matrix(5, si.STREAM_A, 37, 11)
    assert torch.equal(A[:, [0, 3, 10]], si.matrix_cols(5, si.STREAM_A, 37, 11, [0, 3, 10]))


def test_padding_is_nan_and_values_independent_of_ld():
    A = si.matrix(6, si.STREAM_B, 9, 4, ld=13)
    assert A.stride() == (1, 13)
    store = torch.as_strided(A, (4, 13), (13, 1))
    assert not torch.isnan(A).any()
    assert torch.isnan(store[:, 9:]).all()
    assert torch.equal(A.contiguous(), si.matrix(6, si.STREAM_B, 9, 4).contiguous())


def test_uniform_and_normal_moments():
    u = si.uniform(1, 1, torch.arange(1 << 18))
    assert u.min() >= -1 and u.max() < 1
    assert abs(float(u.mean())) < 0.01 and abs(float(u.var()) - 1 / 3) < 0.01
    z = si.normal(1, 3, torch.arange(1 << 18))
    assert abs(float(z.mean())) < 0.01 and abs(float(z.var()) - 1) < 0.02
    i = si.integers(1, 2, torch.arange(1 << 16), 4)
    assert set(i.unique().tolist()) == set(range(-4, 5))


def test_streams_and_seeds_differ():
    a = si.uniform(1, 1, torch.arange(64))
    b = si.uniform(1, 2, torch.arange(64))
    c = si.uniform(2, 1, torch.arange(64))
    assert not torch.equal(a, b) and not torch.equal(a, c)


def test_float32_rounding_of_generated_values():
    A64 = si.matrix(3, si.STREAM_A, 100, 3)
    A32 = si.matrix(3, si.STREAM_A, 100, 3, dtype=torch.float32)
    assert torch.equal(A64.to(torch.float32), A32)
