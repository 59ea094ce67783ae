"""The TSM2R plan query, per-shape pins and the autotuner: every plan the
library can launch for a shape computes the same product (bit-exact on
integer data, within tolerance on random data), pins take effect and are
removed, and the tuner pins the fastest plan it measured."""
import numpy as np
import pytest
import torch

import oracle
import paper_2002_03258_amd as tsm
from paper_2002_03258_amd import model, tune
import seeded_inputs as si

from helpers import TOL, dev_matrix, err, host_matrix, to_np

pytestmark = pytest.mark.gpu

DTYPES = [torch.float64, torch.float32]
DT = {torch.float64: tsm.F64, torch.float32: tsm.F32}


def test_plan_query_matches_kernel_name(dev):
    for m, k, n in [(30720, 30720, 16), (10240, 10240, 2), (3001, 5000, 20)]:
        p = tsm.tsm2r_plan(m, k, n, tsm.F64)
        assert p["kernel"] == tsm.kernel_name(tsm.OP_TSM2R, m, k, n, tsm.F64)
        assert p["tiles"] == -(-m // p["tile_rows"])
        assert p["slices"] >= 1 and p["occupancy"] >= 1 and p["cus"] >= 1
        assert p["workgroups"] <= p["cus"] * p["occupancy"]


@pytest.mark.parametrize("dtype", DTYPES)
def test_every_candidate_plan_gives_the_same_product(dev, dtype):
    m, k, n = 3001, 5000, 16
    dt = DT[dtype]
    cands = tune.candidates(m, k, n, dt)
    assert len({(p["tall"], p["slices"]) for p in cands}) == len(cands) >= 4
    assert {p["tall"] for p in cands} == {0, 1}
    # integer data: every plan bit-exact (all partial sums exact)
    Ai = dev_matrix(61, si.STREAM_A, m, k, dtype, dev, dist="int", r=4)
    Bi = dev_matrix(61, si.STREAM_B, k, n, dtype, dev, dist="int", r=4)
    ref_i = oracle.matmul(host_matrix(61, si.STREAM_A, m, k, dtype, dist="int", r=4),
                          host_matrix(61, si.STREAM_B, k, n, dtype, dist="int", r=4))
    A = dev_matrix(62, si.STREAM_A, m, k, dtype, dev)
    B = dev_matrix(62, si.STREAM_B, k, n, dtype, dev)
    ref = oracle.matmul(host_matrix(62, si.STREAM_A, m, k, dtype),
                        host_matrix(62, si.STREAM_B, k, n, dtype))
    try:
        for p in cands:
            tsm.pin_tsm2r(m, k, n, dt, p["slices"], p["tall"])
            q = tsm.tsm2r_plan(m, k, n, dt)
            assert (q["slices"], q["tall"]) == (p["slices"], p["tall"])
            assert np.array_equal(to_np(tsm.tsm2r(Ai, Bi)), ref_i), p
            assert err(to_np(tsm.tsm2r(A, B)), ref) <= TOL[dtype], p
    finally:
        tsm.unpin_tsm2r(m, k, n, dt)


def test_pin_applies_to_its_shape_only_and_is_removed(dev):
    m, k, n = 4000, 6000, 8
    base = tsm.tsm2r_plan(m, k, n, tsm.F64)
    other = tsm.tsm2r_plan(m, k, n + 1, tsm.F64)
    f32 = tsm.tsm2r_plan(m, k, n, tsm.F32)
    try:
        tsm.pin_tsm2r(m, k, n, tsm.F64, 1, 1 - base["tall"])
        p = tsm.tsm2r_plan(m, k, n, tsm.F64)
        assert p["slices"] == 1 and p["tall"] == 1 - base["tall"]
        assert tsm.tsm2r_plan(m, k, n + 1, tsm.F64) == other
        assert tsm.tsm2r_plan(m, k, n, tsm.F32) == f32
        # tile height left to the planner, S forced
        tsm.pin_tsm2r(m, k, n, tsm.F64, 2, -1)
        assert tsm.tsm2r_plan(m, k, n, tsm.F64)["slices"] == 2
    finally:
        tsm.unpin_tsm2r(m, k, n, tsm.F64)
    assert tsm.tsm2r_plan(m, k, n, tsm.F64) == base


def test_pinned_split_sizes_the_workspace(dev):
    m, k, n = 2000, 8000, 16
    w0 = tsm.workspace_size(tsm.OP_TSM2R, m, k, n, tsm.F64)
    try:
        tsm.pin_tsm2r(m, k, n, tsm.F64, 40, 0)
        p = tsm.tsm2r_plan(m, k, n, tsm.F64)
        w = tsm.workspace_size(tsm.OP_TSM2R, m, k, n, tsm.F64)
        assert w >= p["workgroups"] * 16 * p["tile_rows"] * 8 and w > w0
        A = dev_matrix(63, si.STREAM_A, m, k, torch.float64, dev)
        B = dev_matrix(63, si.STREAM_B, k, n, torch.float64, dev)
        ws = torch.empty(w, dtype=torch.uint8, device=dev)
        C = tsm.tsm2r(A, B, workspace=ws)
        ref = oracle.matmul(host_matrix(63, si.STREAM_A, m, k, torch.float64),
                            host_matrix(63, si.STREAM_B, k, n, torch.float64))
        assert err(to_np(C), ref) <= TOL[torch.float64]
    finally:
        tsm.unpin_tsm2r(m, k, n, tsm.F64)


@pytest.mark.parametrize("dtype", DTYPES)
def test_autotune_pins_the_fastest_measured_plan(dev, dtype):
    m, k, n = 8192, 8192, 8
    dt = DT[dtype]
    A = dev_matrix(64, si.STREAM_A, m, k, dtype, dev)
    B = dev_matrix(64, si.STREAM_B, k, n, dtype, dev)
    try:
        r = tune.autotune_tsm2r(A, B, top=4, reps=3)
        timed = [e for e in r["report"] if "gbs" in e]
        assert 4 <= len(timed) <= 5
        assert r["best"]["gbs"] == max(e["gbs"] for e in timed)
        assert r["best"]["gbs"] >= r["default"]["gbs"]
        p = tsm.tsm2r_plan(m, k, n, dt)
        assert (p["slices"], p["tall"]) == (r["best"]["slices"], r["best"]["tall"])
        # predictions are attached to every candidate and ranked
        preds = [e["pred_gbs"] for e in r["report"]]
        assert preds == sorted(preds, reverse=True) and all(x > 0 for x in preds)
        ref = oracle.matmul(host_matrix(64, si.STREAM_A, m, k, dtype),
                            host_matrix(64, si.STREAM_B, k, n, dtype))
        assert err(to_np(tsm.tsm2r(A, B)), ref) <= TOL[dtype]
    finally:
        tsm.unpin_tsm2r(m, k, n, dt)


def test_autotune_without_pin_leaves_the_planner(dev):
    m, k, n = 4096, 4096, 4
    A = dev_matrix(65, si.STREAM_A, m, k, torch.float64, dev)
    B = dev_matrix(65, si.STREAM_B, k, n, torch.float64, dev)
    before = tsm.tsm2r_plan(m, k, n, tsm.F64)
    tune.autotune_tsm2r(A, B, top=2, reps=2, pin=False)
    assert tsm.tsm2r_plan(m, k, n, tsm.F64) == before


def test_model_ranks_the_planner_choice_near_the_top(dev):
    # the model, fed the library's own plan facts, puts the planner's plan for
    # the headline shape among its best few
    m = k = 30720
    cands = tune.candidates(m, k, 16, tsm.F64)
    ranked = model.rank(m, k, 16, 8, cands)
    d = tsm.tsm2r_plan(m, k, 16, tsm.F64)
    pos = [(p["tall"], p["slices"]) for p in ranked].index((d["tall"], d["slices"]))
    assert pos < 4
