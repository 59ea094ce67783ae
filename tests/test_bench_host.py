"""Host logic of bench.py, without a GPU: the one-GPU refusal, the order of
the TSM2R grid's products, the algorithmic bytes of the autograd passes, the
attribution of kernels to the calls of a pass, the roofline's choice of the
dominant kernel, the ceiling each row is compared with, and the lookup of
the rocprofv3 counter summaries behind `roofline.traffic`."""
import glob
import os
import subprocess
import sys

import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_grid_order_never_repeats_A(monkeypatch):
    # small stand-ins for the workload sizes: the order, not the size, is
    # under test
    monkeypatch.setattr(bench, "R_SIZES", (64, 96, 128))
    monkeypatch.setattr(bench, "nn_kernel_name", lambda dtype, m, n: "k")
    calls = bench.make_r_inputs(torch.device("cpu"))
    assert len(calls) == len(bench.R_SIZES) * len(bench.R_NS) * len(bench.R_DTYPES)
    assert len({c["workload"] for c in calls}) == len(calls)
    for a, b in zip(calls, calls[1:]):
        assert a["A"].data_ptr() != b["A"].data_ptr(), (a["workload"], b["workload"])
    for c in calls:
        m, n = c["m"], c["n"]
        assert c["k"] == m and c["A"].shape == (m, m) and c["B"].shape == (m, n)
        assert c["A"].stride() == (1, m)                  # column-major A
        assert c["bytes"] == (m * m + 2 * m * n) * bench.es(c["dtype"])


def test_autograd_bytes():
    m, k, n = 1000, 16, 8
    # TSM2L: forward reads A and B and writes C; the fused backward reads A,
    # dC and B and writes dA and dB
    b = bench.ag_bytes("L", "f64", m, k, n)
    assert b == {"fwd": 8 * (m * k + k * n + m * n),
                 "bwd": 8 * (m * k + m * n + k * n + m * k + k * n)}
    # the split form reads A as two 2-byte planes; everything else is float32
    b = bench.ag_bytes("L", "bf16_split", m, k, n)
    assert b["fwd"] == 4 * m * k + 4 * (k * n + m * n)
    b = bench.ag_bytes("R", "bf16_split", m, k, n)
    assert b == {"fwd": 4 * m * k + 4 * (k * n + m * n), "grad_a": 4 * (m * n + k * n + m * k),
                 "grad_b": 4 * m * k + 4 * (m * n + k * n)}
    assert bench.ag_bytes("R", "bf16", m, k, n)["fwd"] == 2 * m * k + 4 * (k * n + m * n)
    assert bench.ag_bytes("R", "f32", m, k, n)["grad_b"] == 4 * (m * k + m * n + k * n)


def _case(kind, mode, index, m=4096, k=16, n=16):
    c = object.__new__(bench.AGCase)
    c.kind, c.mode, c.m, c.k, c.n = kind, mode, m, k, n
    c.tag_fwd, c.tag_bwd = 2 * index + 1, 2 * index + 2
    c.bytes = bench.ag_bytes(kind, mode, m, k, n)
    c.total_bytes = sum(c.bytes.values())
    c.name = "%s %s" % ("TSM2L" if kind == "L" else "TSM2R", mode)
    return c


def test_kernels_map_to_the_calls_of_a_pass():
    L, R = _case("L", "f64", 0), _case("R", "bf16_split", 1, 512, 512, 8)
    assert L.role(L.tag_fwd, "rowtile_kernel<double, 4, 1, 1, true, false>") == "fwd"
    assert L.role(L.tag_bwd, "tsm2l_bwd_kernel<double, 1, 1, 2, true, -1, false>") == "bwd"
    assert L.role(L.tag_bwd, "split_reduce_kernel<double, true>") is None
    assert L.role(R.tag_fwd, "rowtile_kernel<double, 4, 1, 1, true, false>") is None
    assert R.role(R.tag_fwd, "tsm2r_lp_kernel<0, 1, true, 4, true>") == "fwd"
    assert R.role(R.tag_bwd, "rowtile_kernel<float, 2, 2, 2, true, false>") == "grad_a"
    assert R.role(R.tag_bwd, "tn_lp_kernel<0, 1, true, true, true>") == "grad_b"
    assert R.role(R.tag_bwd, "split_kernel<0, true, true>") is None


def test_roofline_takes_the_longest_kernel_and_its_calls_bytes():
    L, R = _case("L", "f64", 0), _case("R", "f64", 1, 512, 512, 8)
    timing = [
        {"kernel": "rowtile_kernel<double, 4, 1, 1, true, false>", "tag": L.tag_fwd,
         "launches": 10, "total_ms": 4.0},
        {"kernel": "tsm2l_bwd_kernel<double>", "tag": L.tag_bwd, "launches": 10, "total_ms": 8.0},
        # overhead kernels never count, however long
        {"kernel": "split_reduce_kernel<double, true>", "tag": L.tag_bwd, "launches": 10,
         "total_ms": 50.0},
        {"kernel": "tn_kernel<double>", "tag": R.tag_bwd, "launches": 10, "total_ms": 6.0},
        {"kernel": "unknown_kernel", "tag": 99, "launches": 1, "total_ms": 99.0}]
    r = bench.roofline_of([L, R], timing)
    assert r["kernel"] == "tsm2l_bwd_kernel<double>"
    assert r["algorithmic_bytes_per_launch"] == L.bytes["bwd"]
    assert r["avg_launch_us"] == pytest.approx(800.0)
    assert r["achieved"] == pytest.approx(L.bytes["bwd"] / 800e-6 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)
    assert r["workload"] == "autograd:f64:L:bwd"
    assert bench.roofline_of([L, R], timing[2:3]) is None


def test_rows_take_the_ceiling_of_their_traffic_mix():
    ceil = {"read_GBps": 7000.0, "copy_GBps": 6000.0}
    rows = bench.attach_ceilings([
        {"row": "TSM2L forward (C = A*B)", "GBps": 5000.0},
        {"row": "autograd fwd+bwd", "GBps": 3000.0},
        {"row": "precision TSM2R A 32768^2", "GBps": 7000.0}], ceil)
    assert [r["measured_ceiling_GBps"] for r in rows] == [6000.0, 6000.0, 7000.0]
    assert rows[1]["frac_of_measured_ceiling"] == pytest.approx(0.5)
    assert rows[2]["frac_of_measured_ceiling"] == pytest.approx(1.0)


def test_every_headline_call_has_a_measured_ceiling():
    keys = set(bench.STREAM_CEILINGS)
    for dt, m in bench.PATTERN_SHAPES:
        keys |= {bench.pattern_key(p, dt, m) for p in ("tsm2l_pattern_", "tsm2l_bwd_pattern_")}
    for shape, kind, m, k, n in bench.AG_SHAPES:
        for mode in bench.AG_MODES:
            roles = ("fwd", "bwd") if kind == "L" else ("fwd", "grad_a", "grad_b")
            for role in roles:
                assert bench.ceiling_key(kind, mode, role, m) in keys, (kind, mode, role)
    assert bench.ceiling_key("L", "f64", "bwd", 1 << 23) == \
        "tsm2l_bwd_pattern_float64_m8388608_k16_GBps"
    assert bench.ceiling_key("R", "bf16_split", "grad_a", 16384) == "write_GBps"
    line = {"config": {"cases": [{"calls": {"bwd": {"GBps": 2000.0, "ceiling": "c"}}}]},
            "roofline": {"achieved": 3000.0, "ceiling": "c"}}
    bench.attach_call_ceilings(line, {"c": 4000.0})
    assert line["config"]["cases"][0]["calls"]["bwd"]["frac_of_measured_ceiling"] == 0.5
    assert line["roofline"]["frac_of_measured_ceiling"] == 0.75


def _summaries():
    out = []
    for path in glob.glob(os.path.join(ROOT, "profiles", "*_counters.txt")):
        info = {}
        for line in open(path):
            if "=" in line and not line.startswith("#"):
                key, val = line.split("=", 1)
                info[key.strip()] = val.strip()
        info["path"] = path
        out.append(info)
    return out


def test_counter_summaries_are_whole():
    infos = _summaries()
    assert infos
    for info in infos:
        for key in ("kernel", "workload", "kernel_source_sha256_16", "hbm_bytes_per_launch",
                    "algorithmic_bytes_per_launch", "hbm_fetch_bytes_per_launch",
                    "hbm_write_bytes_per_launch"):
            assert key in info, (info["path"], key)
        hbm = int(info["hbm_bytes_per_launch"])
        assert hbm == int(info["hbm_fetch_bytes_per_launch"]) + \
            int(info["hbm_write_bytes_per_launch"])
        # no kernel moves less than its algorithmic bytes
        assert hbm >= 0.99 * int(info["algorithmic_bytes_per_launch"]), info["path"]


def test_traffic_lookup_checks_kernel_workload_and_sources(tmp_path, monkeypatch):
    src = tmp_path / "paper_2002_03258_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "a.hip").write_text("kernel source")
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    sha = bench.sources_hash(["a.hip"])
    (tmp_path / "profiles" / "x_counters.txt").write_text(
        "# a summary\nkernel = k<double>\nworkload = autograd:f64:L:bwd\n"
        "kernel_source_sha256_16 = %s (a.hip)\nhbm_bytes_per_launch = 1234\n" % sha)
    assert bench.traffic_from_profiles("k<double>", "autograd:f64:L:bwd") == 1234.0
    assert bench.traffic_from_profiles("k<float>", "autograd:f64:L:bwd") is None
    assert bench.traffic_from_profiles("k<double>", "autograd:f64:R:fwd") is None
    (src / "a.hip").write_text("kernel source, changed")
    assert bench.traffic_from_profiles("k<double>", "autograd:f64:L:bwd") is None
