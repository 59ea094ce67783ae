"""Throughput benchmark of the TSM2R / TSM2L kernels on one MI355X.

A step is one pass over the TSM2R workload grid of square A (m = k in
{10240, 20480, 30720}) times B (k x n, n in {2, 4, 8, 16}) in FP64 and FP32:
24 products C = A*B, inputs resident in HBM, iid uniform[-1, 1] from the
seeded counter-based generator.  ``value`` is the achieved HBM throughput:
algorithmic bytes (A read once, B read once, C written once) per second over
the K timed steps.

Besides the headline line the JSON carries:
  roofline      the dominant kernel (largest total time in the step), its
                algorithmic bytes per launch over its average launch duration
                (HIP events on the stream it runs on) against 8 TB/s, and the
                HBM traffic rocprofv3 counted for it (profiles/), or null;
  cpu_baseline  the FP64 oracle timed on this host's cores on a row sample of
                the largest workload;
  rows          the other hot-path rows measured on their own workloads
                (TSM2L grid, backward of C = A*B), each with GB/s, fraction of
                8 TB/s and the normwise error of sampled outputs vs the oracle;
  check         normwise errors of sampled rows of every product of the step.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
       [--no-cpu-baseline] [--no-rows] [--profile-kernel | --profile-copy]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

import paper_2002_03258_amd as tsm  # noqa: E402
from paper_2002_03258_amd import model as perf_model  # noqa: E402
from paper_2002_03258_amd import tune  # noqa: E402
import seeded_inputs as si  # noqa: E402

PEAK_HBM_GBS = 8000.0
# streaming-read ceiling measured on MI355X with a 16-byte non-temporal
# linear-read probe (reported beside the datasheet peak)
READ_CEILING_GBS = 7090.0
# read + write ceiling measured the same way: a 1 GiB copy with 16-byte
# non-temporal loads and stores
COPY_CEILING_GBS = 6385.0


def attach_ceilings(rows):
    """Each row's fraction of the measured ceiling of its traffic mix: the
    copy ceiling for products that write about as much as they read (TSM2L,
    the backward passes), the streaming-read ceiling otherwise."""
    for r in rows:
        rw = r["row"].startswith("TSM2L forward") or r["row"].startswith("autograd")
        r["measured_ceiling_GBps"] = COPY_CEILING_GBS if rw else READ_CEILING_GBS
        r["frac_of_measured_ceiling"] = r["GBps"] / r["measured_ceiling_GBps"]
    return rows
R_SIZES = (10240, 20480, 30720)
R_NS = (2, 4, 8, 16)
R_DTYPES = (torch.float64, torch.float32)
L_MS = (1 << 20, 1 << 22, 1 << 24)
L_KS = (8, 16, 32)
TOL = {torch.float64: 1e-13, torch.float32: 1e-5}
# the TSM2R kernel's sources: counter summaries taken from another version of
# them are not used
KERNEL_SRC = [os.path.join(ROOT, "paper_2002_03258_amd", "csrc", f)
              for f in ("tsm2x_tsm2r.hip", "tsm2x_device.h")]


def es(dtype) -> int:
    return 8 if dtype == torch.float64 else 4


def nn_kernel_name(dtype, m, n) -> str:
    return tsm.kernel_name(tsm.OP_TSM2R, m, m, n, tsm.F64 if dtype == torch.float64 else tsm.F32)


def src_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SRC:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def make_r_inputs(dev):
    """The 24 products of the TSM2R grid.  Consecutive products never share
    A (the order is n, then m, per type), so no product finds part of its A
    left in the 256 MB MALL by the one before."""
    seed = si.config_seed(1)
    mats = {(dtype, m): si.matrix(seed, si.STREAM_A, m, m, dtype=dtype, device=dev)
            for dtype in R_DTYPES for m in R_SIZES}
    calls = []
    for dtype in R_DTYPES:
        for n in R_NS:
            for m in R_SIZES:
                A = mats[(dtype, m)]
                B = si.matrix(seed + n, si.STREAM_B, m, n, dtype=dtype, device=dev)
                C = tsm.empty_colmajor(m, n, dtype, dev)
                calls.append(dict(dtype=dtype, m=m, k=m, n=n, A=A, B=B, C=C, seed=seed,
                                  workload="%s:%d:%d" % ("f64" if dtype == torch.float64 else "f32", m, n),
                                  bytes=(m * m + m * n + m * n) * es(dtype),
                                  kernel=nn_kernel_name(dtype, m, n)))
    return calls


def run_step(calls, evs=None):
    for i, c in enumerate(calls):
        if evs is not None:
            evs[i][0].record()
        tsm.tsm2r(c["A"], c["B"], out=c["C"])
        if evs is not None:
            evs[i][1].record()


def gpu_clocks():
    """The GPU's current clocks as rocm-smi reports them (clocks are not
    pinned for the measurement), or None where rocm-smi is unavailable."""
    import subprocess
    try:
        r = subprocess.run(["rocm-smi", "--showclocks", "--json"], capture_output=True,
                           text=True, timeout=20)
        cards = json.loads(r.stdout)
        card = cards[sorted(cards)[0]]
        return {key: val for key, val in card.items() if "clk" in key.lower()}
    except Exception:
        return None


def _plan_prediction(c):
    p = tsm.tsm2r_plan(c["m"], c["k"], c["n"], tsm.F64 if c["dtype"] == torch.float64 else tsm.F32)
    return perf_model.predict_tsm2r(c["m"], c["k"], c["n"], es(c["dtype"]), p["slices"],
                                    p["tiles"], p["tile_rows"], p["occupancy"])


def model_summary(calls, evs, step_bytes, value):
    """The performance model's prediction for the plans the step ran, against
    the HIP-event time of each product (median over the timed steps)."""
    pred_t, errs = 0.0, []
    for i, c in enumerate(calls):
        t_pred = _plan_prediction(c).seconds
        t_meas = float(np.median([evs[s][i][0].elapsed_time(evs[s][i][1]) / 1e3
                                  for s in range(len(evs))]))
        pred_t += t_pred
        errs.append((t_pred - t_meas) / t_meas)
    dev = perf_model.MI355X
    return {"predicted_GBps": step_bytes / pred_t / 1e9, "measured_GBps": value,
            "time_rel_err_mean": float(np.mean(errs)),
            "time_rel_err_max_abs": float(np.max(np.abs(errs))),
            "latency_us": dev.latency_us, "stream_GBps": dev.stream_gbs,
            "knee_workgroups": perf_model.knee_workgroups(dev)}


def model_report(calls):
    """Every candidate plan of each workload: predicted and measured GB/s;
    then the model's constants fitted to all of them."""
    print("%-14s %4s %3s %5s %6s %9s %9s %7s" % ("workload", "tall", "S", "WGs", "rounds",
                                                 "pred GB/s", "meas GB/s", "pred/meas"))
    samples = []
    for c in calls:
        r = tune.autotune_tsm2r(c["A"], c["B"], top=1000, pin=False)
        d = r["default"]
        for e in sorted(r["report"], key=lambda e: (e["tall"], e["slices"])):
            pr = perf_model.predict_tsm2r(c["m"], c["k"], c["n"], es(c["dtype"]), e["slices"],
                                          e["tiles"], e["tile_rows"], e["occupancy"])
            mark = " planner" if (e["tall"], e["slices"]) == (d["tall"], d["slices"]) else ""
            mark += " best" if e is r["best"] else ""
            print("%-14s %4d %3d %5d %6d %9.0f %9.0f %7.2f%s" % (
                c["workload"], e["tall"], e["slices"], e["workgroups"], pr.rounds,
                e["pred_gbs"], e["gbs"], e["pred_gbs"] / e["gbs"], mark), flush=True)
            samples.append(dict(m=c["m"], k=c["k"], n=c["n"], es=es(c["dtype"]),
                                slices=e["slices"], tiles=e["tiles"], tile_rows=e["tile_rows"],
                                occupancy=e["occupancy"], seconds=e["seconds"]))

    def rms(dev):
        return float(np.sqrt(np.mean([np.log(perf_model.predict_tsm2r(
            s["m"], s["k"], s["n"], s["es"], s["slices"], s["tiles"], s["tile_rows"],
            s["occupancy"], dev).seconds / s["seconds"]) ** 2 for s in samples])))
    fitted = perf_model.fit(samples)
    print("plans %d; rms log(pred/meas) with the built-in constants %.3f, refitted %.3f: %s"
          % (len(samples), rms(perf_model.MI355X), rms(fitted), fitted), flush=True)


def check_calls(calls):
    import oracle
    worst = {}
    for c in calls:
        m, k, n, dtype = c["m"], c["k"], c["n"], c["dtype"]
        rows = sorted(set([0, 1, m - 1] + list(np.random.default_rng(m + n).integers(0, m, 13))))
        Ar = si.matrix_rows(c["seed"], si.STREAM_A, m, k, rows, dtype=dtype).double().numpy()
        B = si.matrix(c["seed"] + n, si.STREAM_B, k, n, dtype=dtype).double().numpy()
        # Dot2 reference: the sequential sum's own error (~6e-15 at k = 30720)
        # would otherwise be part of the figure
        e = oracle.normwise_error(c["C"][rows].double().cpu().numpy(), oracle.matmul_dot2(Ar, B))
        key = str(dtype).replace("torch.", "")
        worst[key] = max(worst.get(key, 0.0), e)
    return {k: {"max_normwise_err": v, "tol": TOL[getattr(torch, k)],
                "ok": v <= TOL[getattr(torch, k)]} for k, v in worst.items()}


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline():
    """The FP64 oracle on a row sample of the largest TSM2R workload, on all
    of the host's cores and on one (each sample sized for about 10 s)."""
    import oracle
    m = k = R_SIZES[-1]
    n = 16
    seed = si.config_seed(1)
    B = si.matrix(seed + n, si.STREAM_B, k, n).numpy()
    cores = oracle.threads()

    def probe_rows(target_s):
        # rows of A the oracle gets through in about target_s seconds
        Ar = si.matrix_rows(seed, si.STREAM_A, m, k, list(range(64))).numpy()
        t0 = time.perf_counter()
        oracle.matmul(Ar, B)
        return int(min(m, max(64, 64 * target_s / max(time.perf_counter() - t0, 1e-3))))

    rows_all = probe_rows(10.0)
    oracle.set_threads(1)
    rows_one = min(rows_all, probe_rows(6.0))
    oracle.set_threads(cores)
    Ar = si.matrix_rows(seed, si.STREAM_A, m, k, list(range(rows_all))).numpy()

    def rate(rows):
        t0 = time.perf_counter()
        oracle.matmul(Ar[:rows], B)
        dt = time.perf_counter() - t0
        return (rows * k + k * n + rows * n) * 8 / dt / 1e9, dt

    v_all, dt = rate(rows_all)
    oracle.set_threads(1)
    v_one, dt1 = rate(rows_one)
    oracle.set_threads(cores)
    return {"value": v_all, "unit": "GB/s", "cores": cores, "kind": "oracle", "seconds": dt,
            "single_thread_value": v_one, "single_thread_seconds": dt1, "cpu_model": _cpu_model(),
            "sample": "FP64 TSM2R C = A*B on the first %d (all cores) and %d (one core) of %d "
                      "rows of A (k = %d, n = %d); algorithmic bytes of the sample over the "
                      "oracle's time" % (rows_all, rows_one, m, k, n)}


def traffic_for(kernel: str, launches):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summaries (profiles/*_counters.txt), averaged like the launches of the
    timed step; None when a workload is missing or the summary was taken
    from another kernel source."""
    import glob
    found = {}
    for path in glob.glob(os.path.join(ROOT, "profiles", "*_counters.txt")):
        info = {}
        for line in open(path):
            if "=" in line and not line.startswith("#"):
                key, val = line.split("=", 1)
                info[key.strip()] = val.strip()
        if info.get("kernel") != kernel or info.get("kernel_source_sha256_16") != src_hash():
            continue
        try:
            found[info["workload"]] = float(info["hbm_bytes_per_launch"])
        except (KeyError, ValueError):
            continue
    tot = 0.0
    for wl in launches:
        if wl not in found:
            return None
        tot += found[wl]
    return tot / len(launches) if launches else None


def timed(fn, reps=5, warmup=1, flush=None, warm_seconds=0.05):
    """Median seconds of fn() over `reps` runs, each bracketed by HIP events
    (the median keeps one disturbed run from moving a row); `flush`
    (untimed) runs before each rep to evict the 256 MB MALL.  The warm-up is
    at least `warmup` calls and `warm_seconds` of GPU time: the GPU takes
    some tens of milliseconds of sustained load to reach steady clocks."""
    from paper_2002_03258_amd.tune import _warm
    _warm(fn, warm_seconds, max(1, warmup))
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    torch.cuda.synchronize()
    for e0, e1 in evs:
        if flush is not None:
            flush()
        e0.record()
        fn()
        e1.record()
    torch.cuda.synchronize()
    ts = sorted(e0.elapsed_time(e1) for e0, e1 in evs)
    return ts[len(ts) // 2] / 1e3


def rows_tsm2l(dev):
    import oracle
    out = []
    seed = si.config_seed(2)
    for dtype in R_DTYPES:
        tot_b, tot_t, worst = 0.0, 0.0, 0.0
        for m in L_MS:
            for k in L_KS:
                A = si.matrix(seed + k, si.STREAM_A, m, k, dtype=dtype, device=dev)
                B = si.matrix(seed + k, si.STREAM_B, k, k, dtype=dtype, device=dev)
                C = tsm.empty_colmajor(m, k, dtype, dev)
                flush = torch.empty(1 << 29, dtype=torch.uint8, device=dev)
                t = timed(lambda: tsm.tsm2l(A, B, out=C), flush=flush.zero_)
                nb = (2 * m * k + k * k) * es(dtype)
                tot_b += nb
                tot_t += t
                rows = [0, m // 3, m - 1]
                ref = oracle.matmul(si.matrix_rows(seed + k, si.STREAM_A, m, k, rows,
                                                   dtype=dtype).double().numpy(),
                                    si.matrix(seed + k, si.STREAM_B, k, k, dtype=dtype)
                                    .double().numpy())
                worst = max(worst, oracle.normwise_error(C[rows].double().cpu().numpy(), ref))
                del A, B, C, flush
        torch.cuda.empty_cache()
        out.append({"row": "TSM2L forward (C = A*B, m in 2^20..2^24, k = n in 8..32)",
                    "dtype": str(dtype).replace("torch.", ""), "GBps": tot_b / tot_t / 1e9,
                    "frac_of_8TBps": tot_b / tot_t / 1e9 / PEAK_HBM_GBS,
                    "max_normwise_err": worst, "tol": TOL[dtype]})
    return out


def rows_kmeans(dev):
    """K-means assignment (the Introduction's tall-and-skinny GEMM user):
    m = 2^24 points, k = 16 coordinates, n = 16 centroids, points stored
    column-major and row-major.  GB/s counts X and the centroids read once and the labels
    and distances written once.  For comparison, the same result composed of
    unfused steps: the cross terms by the library's TSM2L product (an m x n
    matrix written), then the scores and the argmin by torch (that matrix
    read back)."""
    import oracle
    from paper_2002_03258_amd import kmeans
    out = []
    seed = si.config_seed(7)
    m, k, n = 1 << 24, 16, 16
    for dtype, layout in [(d, lay) for d in R_DTYPES for lay in ("column-major", "row-major")]:
        X = si.matrix(seed, si.STREAM_A, m, k, dtype=dtype, device=dev)
        if layout == "row-major":
            X = X.contiguous()
        Mu = si.matrix(seed, si.STREAM_B, k, n, dtype=dtype, device=dev)
        cent = Mu.t()
        flush = torch.empty(1 << 29, dtype=torch.uint8, device=dev)
        res = {}

        def fused():
            res["r"] = kmeans.assign(X, cent)
        t = timed(fused, flush=flush.zero_)
        lab, dist = res["r"]
        mu2 = (Mu * Mu).sum(dim=0)

        def unfused():
            G = tsm.tsm2l(X, Mu)
            return torch.min(mu2[None, :] - 2 * G, dim=1)
        t_unf = timed(unfused, flush=flush.zero_)
        nb = (m * k + k * n + m) * es(dtype) + 4 * m
        rows = [0, 1, m // 3, m // 2 + 7, m - 1]
        Xr = si.matrix_rows(seed, si.STREAM_A, m, k, rows, dtype=dtype).double().numpy()
        rlab, rdist = oracle.kmeans_assign(Xr, Mu.double().cpu().numpy())
        got = lab[rows].cpu().numpy()
        D = ((Xr[:, :, None] - Mu.double().cpu().numpy()[None]) ** 2).sum(axis=1)
        u = torch.finfo(dtype).eps / 2
        tol = 4 * (k + 2) * u * (np.sqrt((Xr ** 2).sum(1))[:, None]
                                 + np.sqrt((Mu.double().cpu().numpy() ** 2).sum(0))[None]).max(1) ** 2
        ok = bool(np.all(D[np.arange(len(rows)), got] <= rdist + tol) and
                  np.all(np.abs(dist[rows].double().cpu().numpy() - D[np.arange(len(rows)), got])
                         <= tol))
        out.append({"row": "kmeans assignment, m = 2^24 points (%s), k = 16, n = 16 centroids "
                           "(fused)" % layout,
                    "dtype": str(dtype).replace("torch.", ""), "GBps": nb / t / 1e9,
                    "frac_of_8TBps": nb / t / 1e9 / PEAK_HBM_GBS, "ms": t * 1e3,
                    "unfused_ms": t_unf * 1e3, "speedup_vs_unfused": t_unf / t,
                    "sampled_rows_ok": ok, "labels_equal_oracle_on_sample": bool(np.array_equal(got, rlab))})
        del X, Mu, cent, flush, res, lab, dist
        torch.cuda.empty_cache()
    return out


def rows_general(dev):
    """Shapes beyond one kernel launch: n > 32 in 32-column panels (A read once
    per panel, the paper's t2 < n), a TSM2L-class product with k > 32 (on the
    TSM2R kernels), and the dispatching gemm with a row-major B and beta = 1.
    GB/s counts the bytes each product moves."""
    import oracle
    out = []
    seed = si.config_seed(6)
    cases = [("TSM2R n = 64 in two panels", "tsm2r", torch.float64, 20480, 20480, 64, False, 0.0),
             ("TSM2L class with k = 64", "tsm2l", torch.float64, 1 << 22, 64, 16, False, 0.0),
             ("gemm, row-major B, beta = 1", "gemm", torch.float32, 30720, 30720, 16, True, 1.0)]
    for name, fn, dtype, m, k, n, rowB, beta in cases:
        A = si.matrix(seed, si.STREAM_A, m, k, dtype=dtype, device=dev)
        B = si.matrix(seed, si.STREAM_B, k, n, dtype=dtype, device=dev)
        if rowB:
            B = B.contiguous()
        C0 = si.matrix(seed, si.STREAM_V, m, n, dtype=dtype, device=dev)
        C = C0.clone() if beta != 0 else tsm.empty_colmajor(m, n, dtype, dev)
        f = getattr(tsm, fn)
        f(A, B, out=C, beta=beta)            # checked on this first call (from C0)
        rows = [0, m // 2, m - 1]
        Ar = si.matrix_rows(seed, si.STREAM_A, m, k, rows, dtype=dtype).double().numpy()
        Bh = si.matrix(seed, si.STREAM_B, k, n, dtype=dtype).double().numpy()
        ref = oracle.matmul(Ar, Bh)
        if beta != 0:
            ref = ref + beta * C0[rows].double().cpu().numpy()
        e = oracle.normwise_error(C[rows].double().cpu().numpy(), ref)
        t = timed(lambda: f(A, B, out=C, beta=beta))
        panels = (n + 31) // 32 if fn == "tsm2r" else 1
        nb = (panels * m * k + k * n + (2 if beta != 0 else 1) * m * n) * es(dtype)
        out.append({"row": "general shapes: %s (m=%d k=%d n=%d)" % (name, m, k, n),
                    "dtype": str(dtype).replace("torch.", ""), "GBps": nb / t / 1e9,
                    "frac_of_8TBps": nb / t / 1e9 / PEAK_HBM_GBS,
                    "kernel_A_reads": panels, "max_normwise_err": e, "tol": TOL[dtype]})
        del A, B, C, C0
        torch.cuda.empty_cache()
    return out


def rows_lowp(dev):
    """Precision form of TSM2R on A 32768 x 32768: bf16 / f16 planes, single
    and split, against plain FP32 on the same A (ratio of times vs ratio of
    bytes), plus the one-time split of A."""
    import oracle
    out = []
    seed = si.config_seed(3)
    m = k = 32768
    A = si.matrix(seed, si.STREAM_A, m, k, dtype=torch.float32, device=dev)
    rows = [0, 12345, m - 1]
    Ar = si.matrix_rows(seed, si.STREAM_A, m, k, rows, dtype=torch.float32).double().numpy()
    for n in (8, 16, 32):
        B = si.matrix(seed + n, si.STREAM_B, k, n, dtype=torch.float32, device=dev)
        C = tsm.empty_colmajor(m, n, torch.float32, dev)
        t32 = timed(lambda: tsm.tsm2r(A, B, out=C), reps=10)
        b32 = (m * k + k * n + m * n) * 4
        Bh = si.matrix(seed + n, si.STREAM_B, k, n, dtype=torch.float32).double().numpy()
        for fmt, code in (("bf16", oracle.BF16), ("f16", oracle.F16)):
            for lo in (False, True):
                S = tsm.split(A, fmt, lo=lo)
                t_split = timed(lambda: tsm.split(A, fmt, lo=lo), reps=2) if n == 8 else None
                t = timed(lambda: tsm.tsm2r(S, B, out=C), reps=10)
                nb = S.nbytes() + (k * n + m * n) * 4
                hi, lo_ = oracle.split(Ar.astype(np.float32), code)
                stored = oracle.decode_plane(hi, code) + (oracle.decode_plane(lo_, code) if lo else 0)
                Cs = C[rows].double().cpu().numpy()
                row = {"row": "precision TSM2R A 32768^2 %s %s n=%d" % (fmt, "split" if lo else "single", n),
                       "dtype": fmt + ("_split" if lo else ""), "GBps": nb / t / 1e9,
                       "frac_of_8TBps": nb / t / 1e9 / PEAK_HBM_GBS,
                       "fp32_GBps": b32 / t32 / 1e9, "speedup_vs_fp32": t32 / t,
                       "bytes_ratio_fp32_over_form": b32 / nb,
                       "err_vs_stored": oracle.normwise_error(Cs, oracle.matmul(stored, Bh)),
                       "err_vs_fp32_values": oracle.normwise_error(Cs, oracle.matmul(Ar, Bh))}
                if t_split is not None:
                    row["split_GBps"] = (m * k * 4 + S.nbytes()) / t_split / 1e9
                out.append(row)
                del S
        del B, C
    del A
    torch.cuda.empty_cache()
    return out


def rows_autograd(dev):
    """Forward + backward of C = A*B on the two autograd shapes."""
    import oracle
    out = []
    seed = si.config_seed(4)
    for shape, (m, k, n) in (("TSM2L", (8388608, 16, 16)), ("TSM2R", (16384, 16384, 8))):
        for dtype in R_DTYPES:
            A = si.matrix(seed, si.STREAM_A, m, k, dtype=dtype, device=dev)
            B = si.matrix(seed, si.STREAM_B, k, n, dtype=dtype, device=dev)
            dC = si.matrix(seed, si.STREAM_DC, m, n, dtype=dtype, device=dev, dist="normal")
            C = tsm.empty_colmajor(m, n, dtype, dev)
            dA = tsm.empty_colmajor(m, k, dtype, dev)
            dB = tsm.empty_colmajor(k, n, dtype, dev)
            fwd = (lambda: tsm.tsm2l(A, B, out=C)) if shape == "TSM2L" else \
                (lambda: tsm.tsm2r(A, B, out=C))
            s = es(dtype)
            t_f = timed(fwd)
            b_f = (m * k + k * n + m * n) * s
            if shape == "TSM2L":
                # the autograd Function's backward: one fused pass over A and dC
                res = {}

                def bwd():
                    res["g"] = tsm.tsm2l_backward(A, B, dC)
                t_bw = timed(bwd)
                dA, dB = res["g"]
                t_a, t_b = t_bw, 0.0
                b_a = (m * k + m * n + k * n + m * k + k * n) * s
                b_b = 0
            else:
                t_a = timed(lambda: tsm.grad_a(dC, B, out=dA))
                t_b = timed(lambda: tsm.grad_b(A, dC, out=dB))
                b_a = (m * n + k * n + m * k) * s
                b_b = (m * k + m * n + k * n) * s
            rows = [0, m // 2, m - 1]
            Ar = si.matrix_rows(seed, si.STREAM_A, m, k, rows, dtype=dtype).double().numpy()
            Bh = si.matrix(seed, si.STREAM_B, k, n, dtype=dtype).double().numpy()
            dCr = si.matrix_rows(seed, si.STREAM_DC, m, n, rows, dtype=dtype,
                                 dist="normal").double().numpy()
            e_f = oracle.normwise_error(C[rows].double().cpu().numpy(), oracle.matmul(Ar, Bh))
            e_a = oracle.normwise_error(dA[rows].double().cpu().numpy(), oracle.matmul(dCr, Bh.T))
            cols = [0, k // 2, k - 1]
            if m * n <= (1 << 22):
                Ac = si.matrix_cols(seed, si.STREAM_A, m, k, cols, dtype=dtype).double().numpy()
                dCh = si.matrix(seed, si.STREAM_DC, m, n, dtype=dtype,
                                dist="normal").double().numpy()
                e_b = oracle.normwise_error(dB[cols].double().cpu().numpy(),
                                            oracle.matmul(Ac.T, dCh))
            else:
                e_b = None
            out.append({"row": "autograd fwd+bwd %s shape m=%d k=%d n=%d" % (shape, m, k, n),
                        "dtype": str(dtype).replace("torch.", ""),
                        "GBps": (b_f + b_a + b_b) / (t_f + t_a + t_b) / 1e9,
                        "frac_of_8TBps": (b_f + b_a + b_b) / (t_f + t_a + t_b) / 1e9 / PEAK_HBM_GBS,
                        "fwd_GBps": b_f / t_f / 1e9,
                        ("fused_bwd_GBps" if shape == "TSM2L" else "grad_a_GBps"): b_a / t_a / 1e9,
                        "grad_b_GBps": b_b / t_b / 1e9 if t_b > 0 else None,
                        "err": {"C": e_f, "dA": e_a, "dB": e_b}, "tol": TOL[dtype]})
            del A, B, dC, C, dA, dB
            torch.cuda.empty_cache()
    # bf16-split: forward on the planes (split once, reported apart), dA in
    # float, dB on the planes
    for shape, (m, k, n) in (("TSM2L", (8388608, 16, 16)), ("TSM2R", (16384, 16384, 8))):
        A = si.matrix(seed, si.STREAM_A, m, k, dtype=torch.float32, device=dev)
        B = si.matrix(seed, si.STREAM_B, k, n, dtype=torch.float32, device=dev)
        dC = si.matrix(seed, si.STREAM_DC, m, n, dtype=torch.float32, device=dev, dist="normal")
        S = tsm.split(A, "bf16", lo=True)
        C = tsm.empty_colmajor(m, n, torch.float32, dev)
        dA = tsm.empty_colmajor(m, k, torch.float32, dev)
        dB = tsm.empty_colmajor(k, n, torch.float32, dev)
        fwd = (lambda: tsm.tsm2l(S, B, out=C)) if shape == "TSM2L" else (lambda: tsm.tsm2r(S, B, out=C))
        t_f = timed(fwd)
        b_f = S.nbytes() + (k * n + m * n) * 4
        row = {"row": "autograd fwd+bwd %s shape m=%d k=%d n=%d" % (shape, m, k, n),
               "dtype": "bf16_split", "fwd_GBps": b_f / t_f / 1e9}
        if shape == "TSM2L":
            # the autograd Function's backward: one fused pass over the planes and dC
            t_a = timed(lambda: tsm.tsm2l_backward(S, B, dC))
            t_b = 0.0
            b_a = S.nbytes() + (m * n + k * n + m * k + k * n) * 4
            b_b = 0
            row["fused_bwd_GBps"] = b_a / t_a / 1e9
        else:
            t_a = timed(lambda: tsm.grad_a(dC, B, out=dA))
            t_b = timed(lambda: tsm.grad_b(S, dC, out=dB))
            b_a = (m * n + k * n + m * k) * 4
            b_b = S.nbytes() + (m * n + k * n) * 4
            row["grad_a_GBps"] = b_a / t_a / 1e9
            row["grad_b_GBps"] = b_b / t_b / 1e9
        row["GBps"] = (b_f + b_a + b_b) / (t_f + t_a + t_b) / 1e9
        row["frac_of_8TBps"] = row["GBps"] / PEAK_HBM_GBS
        row["ms_fwd_bwd"] = (t_f + t_a + t_b) * 1e3
        out.append(row)
        del A, B, dC, S, C, dA, dB
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-rows", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--profile-kernel", default=None, metavar="DTYPE:M:N",
                    help="only launch TSM2R on one workload of the grid 5 times "
                         "(for rocprofv3 counters), e.g. f64:30720:16")
    ap.add_argument("--profile-op", default=None, metavar="OP:DTYPE:M:K[:LAYOUT]",
                    help="only launch one TSM2L (tsm2l, B k x k) or K-means assignment "
                         "(kmeans, k = n, LAYOUT col or row) product 5 times, for rocprofv3 "
                         "counters, e.g. tsm2l:f64:16777216:16 or kmeans:f32:16777216:16:row")
    ap.add_argument("--profile-copy", action="store_true",
                    help="only run a 1 GiB device copy 5 times (counter calibration)")
    ap.add_argument("--tune", action="store_true",
                    help="autotune the plan of each TSM2R workload before the warmup steps")
    ap.add_argument("--model-report", action="store_true",
                    help="only time every candidate plan of each TSM2R workload beside the "
                         "performance model's prediction, and print the table")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: --gpus %d is not supported (the kernels run on one "
              "device's share of the work; how the path shards is described with the design)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")

    if args.profile_copy:
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print("copied 5 x %d bytes" % src.numel(), flush=True)
        return
    if args.profile_op:
        f = args.profile_op.split(":")
        op, dtype, m, k = f[0], torch.float64 if f[1] == "f64" else torch.float32, int(f[2]), int(f[3])
        seed = si.config_seed(8)
        X = si.matrix(seed, si.STREAM_A, m, k, dtype=dtype, device=dev)
        B = si.matrix(seed, si.STREAM_B, k, k, dtype=dtype, device=dev)
        if op == "tsm2l":
            C = tsm.empty_colmajor(m, k, dtype, dev)
            run = lambda: tsm.tsm2l(X, B, out=C)
        elif op == "kmeans":
            from paper_2002_03258_amd import kmeans
            if len(f) > 4 and f[4] == "row":
                X = X.contiguous()
            run = lambda: kmeans.assign(X, B.t())
        else:
            raise SystemExit("--profile-op: tsm2l or kmeans")
        for _ in range(5):
            run()
        torch.cuda.synchronize()
        print("launched %s 5 times" % args.profile_op, flush=True)
        return
    if args.profile_kernel:
        dts, ms, ns = args.profile_kernel.split(":")
        dtype = torch.float64 if dts == "f64" else torch.float32
        m, n = int(ms), int(ns)
        seed = si.config_seed(1)
        A = si.matrix(seed, si.STREAM_A, m, m, dtype=dtype, device=dev)
        B = si.matrix(seed + n, si.STREAM_B, m, n, dtype=dtype, device=dev)
        C = tsm.empty_colmajor(m, n, dtype, dev)
        for _ in range(5):
            tsm.tsm2r(A, B, out=C)
        torch.cuda.synchronize()
        print("launched %s 5 times on m = k = %d, n = %d" % (nn_kernel_name(dtype, m, n), m, n),
              flush=True)
        return

    t_setup = time.perf_counter()
    calls = make_r_inputs(dev)
    torch.cuda.synchronize()
    print("inputs ready in %.1f s" % (time.perf_counter() - t_setup), file=sys.stderr, flush=True)
    if args.model_report:
        model_report(calls)
        return
    tuned = None
    if args.tune:
        tuned = {}
        for c in calls:
            r = tune.autotune_tsm2r(c["A"], c["B"], top=4)
            tuned[c["workload"]] = {"slices": r["best"]["slices"], "tall": r["best"]["tall"],
                                    "gain": r["best"]["gbs"] / r["default"]["gbs"]}
            c["kernel"] = r["best"]["kernel"]
        print("tuned %d workloads" % len(calls), file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        run_step(calls)
    torch.cuda.synchronize()
    evs = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)]
            for _ in calls] for _ in range(args.steps)]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for s in range(args.steps):
        run_step(calls, evs[s])
    e1.record()
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    step_bytes = sum(c["bytes"] for c in calls)
    step_flops = sum(2.0 * c["m"] * c["k"] * c["n"] for c in calls)
    value = step_bytes * args.steps / (total_ms / 1e3) / 1e9

    per_kernel = {}
    for s in range(args.steps):
        for i, c in enumerate(calls):
            d = per_kernel.setdefault(c["kernel"], {"t": 0.0, "b": 0.0, "n": 0, "wl": []})
            d["t"] += evs[s][i][0].elapsed_time(evs[s][i][1]) / 1e3
            d["b"] += c["bytes"]
            d["n"] += 1
            if s == 0:
                d["wl"].append(c["workload"])
    dom = max(per_kernel, key=lambda k: per_kernel[k]["t"])
    d = per_kernel[dom]
    achieved = d["b"] / d["t"] / 1e9
    per_launch = d["b"] / d["n"]
    traffic = traffic_for(dom, d["wl"])
    roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                "avg_launch_us": d["t"] / d["n"] * 1e6, "launches": d["n"],
                "algorithmic_bytes_per_launch": per_launch,
                "workloads": d["wl"], "traffic": traffic,
                "traffic_over_algorithmic": (traffic / per_launch) if traffic else None}
    line = {
        "metric": "achieved HBM GB/s (% peak), TSM2R/TSM2L fp64 vs bf16-split fwd+bwd at tol",
        "value": value, "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": total_ms / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32",
        "data": "synthetic (seeded counter-based uniform[-1,1])",
        "config": {"workload": "TSM2R plain FP64 and FP32: square A m=k in {10240,20480,30720}, "
                               "B k x n with n in {2,4,8,16}, column-major (24 products per step)",
                   "bytes_per_step": step_bytes, "frac_of_8TBps": value / PEAK_HBM_GBS,
                   "frac_of_measured_read_ceiling": value / READ_CEILING_GBS,
                   "gflop_per_s": step_flops * args.steps / (total_ms / 1e3) / 1e9},
        "roofline": roofline,
    }
    line["model"] = model_summary(calls, evs, step_bytes, value)
    line["config"]["gpu_clocks_after_timing"] = gpu_clocks()
    if tuned is not None:
        line["config"]["tuned_plans"] = tuned
    if not args.no_check:
        line["check"] = check_calls(calls)
    del calls
    torch.cuda.empty_cache()
    if not args.no_rows:
        line["rows"] = attach_ceilings(rows_tsm2l(dev) + rows_lowp(dev) + rows_autograd(dev) +
                                       rows_general(dev) + rows_kmeans(dev))
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
