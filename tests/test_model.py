"""The TSM2R performance model (the paper's Little's-law model, counted in
bytes for gfx950): its ridge against the values the paper prints, and its
terms against their closed forms."""
import json
import os

import pytest

import oracle
from paper_2002_03258_amd import model as M

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_ridge_reproduces_paper_values():
    g = json.load(open(os.path.join(GOLDEN, "t2_threshold.json")))
    bpe = g["bytes_per_element"]
    for row in g["gpus"]:
        t2 = M.t2_threshold(row["peak_fp64_gflops"], row["peak_bw_gbs"], bpe)
        assert abs(t2 - row["paper_t2_threshold"]) <= 0.1 * row["paper_t2_threshold"], row
        # the oracle's independent statement of the same ridge
        assert t2 == pytest.approx(oracle.t2_threshold(row["peak_fp64_gflops"],
                                                       row["peak_bw_gbs"], bpe), rel=1e-12)


def test_every_library_shape_is_memory_bound_on_mi355x():
    for n in (1, 2, 4, 8, 16, 32):
        assert M.regime(n, 8) == "memory"
        assert M.regime(n, 4) == "memory"
    assert M.regime(80, 8) == "compute"


def test_littles_law_closed_forms():
    dev = M.Device(cus=100, stream_gbs=5000.0, latency_us=2.0)
    cmax = 2.0e-6 * 5000e9 / 100                   # latency x throughput per CU
    assert M.concurrent_max_mem(dev) == pytest.approx(cmax)
    assert M.util_mem(cmax / 4, dev) == pytest.approx(0.25)
    assert M.util_mem(cmax, dev) == pytest.approx(1.0)
    assert M.util_mem(3 * cmax, dev) == 1.0
    assert M.util_mem(0, dev) == 0.0


PLAIN = dict(eta=1.0, balance_exp=0.0, t0_us=0.0, round_us=0.0)


def test_single_full_round_is_bytes_over_rate():
    dev = M.Device(cus=256, stream_gbs=7000.0, latency_us=2.0, **PLAIN)
    # 512 workgroups of 32 KB in flight: 16 MB >= 2 us * 7 TB/s = 14 MB
    m, k, n, es = 512 * 64, 8192, 8, 8
    p = M.predict_tsm2r(m, k, n, es, slices=1, tiles=512, tile_rows=64, occupancy=2, dev=dev)
    t = (es * m * k + es * m * n) / 7000e9
    assert p.seconds == pytest.approx(t)
    assert p.rounds == 1 and p.tail_util == 1.0 and p.partial_bytes == 0
    assert p.gbs == pytest.approx(M.algorithmic_bytes(m, k, n, es) / t / 1e9)


def test_every_term_enters_as_stated():
    dev = M.Device(cus=256, stream_gbs=7000.0, latency_us=2.0, eta=0.9, balance_exp=0.5,
                   t0_us=10.0, round_us=4.0)
    m, k, n, es = 160 * 64, 10240, 16, 8
    # 640 workgroups on 768 slots: one round, 128 CUs hold 3 and 128 hold 2
    p = M.predict_tsm2r(m, k, n, es, slices=4, tiles=160, tile_rows=64, occupancy=3, dev=dev)
    part = 640 * 16 * 64 * 8
    assert p.partial_bytes == part and p.rounds == 1
    u = min(1.0, 640 * 4 * 8192 / 256 / M.concurrent_max_mem(dev))
    b = 2.5 / 3
    t = (10e-6 + (es * m * k + part) / (0.9 * 7000e9 * u * b ** 0.5) + 4e-6
         + (part + es * m * n) / 7000e9)
    assert p.seconds == pytest.approx(t)


def test_balance_closed_forms():
    assert M.balance(100, 256) == 1.0          # some CUs idle: no imbalance term
    assert M.balance(512, 256) == 1.0
    assert M.balance(480, 256) == pytest.approx(1.875 / 2)
    assert M.balance(640, 256) == pytest.approx(2.5 / 3)


def test_partial_last_round_is_the_slow_one():
    # 640 workgroups on 512 slots: a full round, then 128 workgroups at a
    # quarter of the concurrency the memory system needs
    dev = M.Device(latency_us=2.2, **PLAIN)
    m, k, n, es = 160 * 64, 10240, 16, 8
    p3 = M.predict_tsm2r(m, k, n, es, 3, 160, 64, 2, dev)
    p4 = M.predict_tsm2r(m, k, n, es, 4, 160, 64, 2, dev)
    p6 = M.predict_tsm2r(m, k, n, es, 6, 160, 64, 2, dev)
    assert p4.rounds == 2 and p4.tail_util < 0.3
    assert p3.seconds < p6.seconds < p4.seconds


def test_fit_recovers_known_constants():
    true = M.Device(latency_us=1.8, eta=0.9, balance_exp=0.6, t0_us=12.0, round_us=5.0)
    samples = []
    for m, es, rows in ((10240, 8, 64), (20480, 8, 128), (30720, 4, 128), (8192, 4, 256)):
        tiles = -(-m // rows)
        for S in range(1, 14):
            for occ in (2, 3):
                t = M.predict_tsm2r(m, m, 8, es, S, tiles, rows, occ, true).seconds
                samples.append(dict(m=m, k=m, n=8, es=es, slices=S, tiles=tiles,
                                    tile_rows=rows, occupancy=occ, seconds=t))
    got = M.fit(samples, M.Device())
    for f in ("latency_us", "eta", "balance_exp", "t0_us", "round_us"):
        assert getattr(got, f) == pytest.approx(getattr(true, f), rel=2e-3), f


def test_rank_orders_by_predicted_time():
    plans = [dict(slices=s, tiles=160, tile_rows=64, occupancy=3) for s in range(1, 10)]
    r = M.rank(10240, 10240, 16, 8, plans)
    # the measured optimum of this shape (480 workgroups) is the model's choice
    assert r[0]["slices"] == 3
    ts = [p["pred"].seconds for p in r]
    assert ts == sorted(ts)


def test_chunks_in_flight_follows_the_library_rule():
    # the shorter tiles hold two chunks for n > 16, FP32 with n <= 4, and a
    # grid of 7/8 to all of the CUs; the tall tiles never
    assert M.chunks_in_flight(8, 8, 0, 256, 256) == 2
    assert M.chunks_in_flight(8, 8, 0, 224, 256) == 2
    assert M.chunks_in_flight(8, 8, 0, 223, 256) == 1
    assert M.chunks_in_flight(8, 8, 0, 257, 256) == 1
    assert M.chunks_in_flight(8, 8, 0, 480, 256) == 1
    assert M.chunks_in_flight(32, 8, 0, 480, 256) == 2
    assert M.chunks_in_flight(4, 4, 0, 480, 256) == 2
    assert M.chunks_in_flight(4, 8, 0, 480, 256) == 1
    assert M.chunks_in_flight(32, 8, 1, 256, 256) == 1


def test_two_chunks_in_flight_raise_the_concurrency():
    dev = M.Device(cus=256, stream_gbs=7000.0, latency_us=2.0, **PLAIN)
    m, k, n, es = 256 * 64, 16384, 8, 8
    one = M.predict_tsm2r(m, k, n, es, 1, 256, 64, 4, dev, tall=1)
    two = M.predict_tsm2r(m, k, n, es, 1, 256, 64, 4, dev, tall=0)
    assert two.seconds < one.seconds
    assert two.tail_util == pytest.approx(min(1.0, 2 * one.tail_util))

