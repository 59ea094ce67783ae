"""Host logic of bench.py, without a GPU: the one-GPU refusal, the order of
the products of a step, the ceiling each row is compared with, and the
lookup of the rocprofv3 counter summaries behind `roofline.traffic`."""
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


def test_step_order_never_repeats_A(monkeypatch):
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


def test_rows_take_the_ceiling_of_their_traffic_mix():
    rows = bench.attach_ceilings([
        {"row": "TSM2L forward (C = A*B)", "GBps": 5000.0},
        {"row": "autograd fwd+bwd", "GBps": 3192.5},
        {"row": "precision TSM2R A 32768^2", "GBps": 7090.0}])
    assert [r["measured_ceiling_GBps"] for r in rows] == [bench.COPY_CEILING_GBS] * 2 + \
        [bench.READ_CEILING_GBS]
    assert rows[1]["frac_of_measured_ceiling"] == pytest.approx(0.5)
    assert rows[2]["frac_of_measured_ceiling"] == pytest.approx(1.0)


def _summaries():
    out = []
    for path in glob.glob(os.path.join(ROOT, "profiles", "tsm2r_nn_*_counters.txt")):
        info = {}
        for line in open(path):
            if "=" in line and not line.startswith("#"):
                key, val = line.split("=", 1)
                info[key.strip()] = val.strip()
        out.append(info)
    return out


def test_counter_summaries_are_whole():
    infos = _summaries()
    assert infos
    for info in infos:
        for key in ("kernel", "workload", "kernel_source_sha256_16", "hbm_bytes_per_launch",
                    "algorithmic_bytes_per_launch"):
            assert key in info, (info.get("workload"), key)
        dt, m, n = info["workload"].split(":")
        m, n, e = int(m), int(n), 8 if dt == "f64" else 4
        assert int(info["algorithmic_bytes_per_launch"]) == (m * m + 2 * m * n) * e
        hbm = int(info["hbm_bytes_per_launch"])
        assert hbm == int(info["hbm_fetch_bytes_per_launch"]) + int(info["hbm_write_bytes_per_launch"])
        # the kernel reads A once: counted traffic may exceed the
        # algorithmic bytes by little, and never falls below the bytes of A
        assert m * m * e <= hbm <= 1.02 * int(info["algorithmic_bytes_per_launch"])


def test_traffic_is_null_for_other_sources_or_missing_workloads(monkeypatch):
    infos = _summaries()
    kernel = infos[0]["kernel"]
    wls = [i["workload"] for i in infos if i["kernel"] == kernel]
    assert bench.traffic_for(kernel, ["f64:1:1"]) is None
    assert bench.traffic_for("no_such_kernel", wls) is None
    monkeypatch.setattr(bench, "src_hash", lambda: infos[0]["kernel_source_sha256_16"])
    want = {i["workload"]: int(i["hbm_bytes_per_launch"]) for i in infos if i["kernel"] == kernel}
    launches = wls + wls[:1]                    # averaged per launch, like the step
    got = bench.traffic_for(kernel, launches)
    assert got == pytest.approx(sum(want[w] for w in launches) / len(launches))
    monkeypatch.setattr(bench, "src_hash", lambda: "0" * 16)
    assert bench.traffic_for(kernel, wls) is None
