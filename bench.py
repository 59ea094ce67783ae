"""Throughput benchmark of the TSM2R / TSM2L path on one MI355X.

A step is one forward and backward pass of C = A*B through the library's
autograd Function, as training runs it (C = matmul(A, B), then dA = dC*B^T
and dB = A^T*dC), on the two differentiation workloads:
  TSM2L shape  A 8388608 x 16, B 16 x 16;
  TSM2R shape  A 16384 x 16384, B 16384 x 8;
each in FP64 and in the bf16-split precision form (A kept in HBM as its
bfloat16 hi + lo planes, B, C, dA and dB float32), with the upstream gradient
dC ~ N(0, 1): four forward + backward passes per step, inputs resident in HBM,
iid uniform[-1, 1] from the seeded counter-based generator.  ``value`` is the
achieved HBM throughput: algorithmic bytes (every operand read once, every
result written once) per second over the K timed steps.

Besides the headline the JSON line carries:
  config.cases  each pass's GB/s, time and bytes, and the bf16-split speedup
                over FP64 per shape;
  err           each pass's C, dA and dB against the FP64 oracle on sampled
                rows (all of dB for the TSM2L shape): normwise and
                componentwise error, for bf16-split against both the stored
                values (hi + lo) and the float values of A;
  roofline      the dominant kernel of the step (largest total launch time),
                its algorithmic bytes per launch over its average launch time
                against 8 TB/s, and the HBM traffic rocprofv3 counted for it
                (profiles/), or null.  Launch times come from the library's
                per-launch timing (a HIP event pair on the stream each kernel
                is launched on) over a second run of the same K steps right
                after the timed one, so that the event records do not sit in
                the timed steps; its step time is reported beside;
  ceilings      the measured HBM ceilings of this device: linear 16-byte
                streams (read, copy, write) and the TSM2L tile pattern without
                its arithmetic;
  cpu_baseline  the FP64 oracle timed on this host's cores on row samples of
                the same two workloads, forward and backward;
  rows          the other hot-path workloads: the TSM2R grid (square A,
                m = k in {10240, 20480, 30720}, n in {2..16}, FP64 and FP32),
                the TSM2L grid, the precision form of TSM2R, FP32 autograd and
                bf16-split autograd with the split of A inside every pass,
                general shapes and the K-means assignment.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
       [--no-cpu-baseline] [--no-rows] [--no-check]
       [--profile-kernel DT:M:N | --profile-op SPEC | --profile-copy | --ceiling]
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
METRIC = "achieved HBM GB/s (% peak), TSM2R/TSM2L fp64 vs bf16-split fwd+bwd at tol"

R_SIZES = (10240, 20480, 30720)
R_NS = (2, 4, 8, 16)
R_DTYPES = (torch.float64, torch.float32)
L_MS = (1 << 20, 1 << 22, 1 << 24)
L_KS = (8, 16, 32)
TOL = {torch.float64: 1e-13, torch.float32: 1e-5}
# the differentiation workloads: (shape, kind, m, k, n)
AG_SHAPES = (("TSM2L", "L", 8388608, 16, 16), ("TSM2R", "R", 16384, 16384, 8))
AG_MODES = ("f64", "bf16_split")
# normwise tolerances per mode (and per view of the precision form)
AG_TOL = {"f64": 1e-13, "f32": 1e-5, "bf16_split": {"stored": 1e-5, "value": 2e-5}}
# kernels that are overhead, not a step of the product (split partial sums,
# zero fills, the transposed-B copy, the split of A)
OVERHEAD_KERNELS = ("split_reduce_kernel", "fill_scale_kernel", "transpose_kernel",
                    "split_kernel")


def attach_ceilings(rows, ceilings):
    """Each row's fraction of the measured ceiling of its traffic mix: the
    copy ceiling for products that write about as much as they read (TSM2L,
    the backward passes), the streaming-read ceiling otherwise."""
    for r in rows:
        rw = r["row"].startswith("TSM2L forward") or r["row"].startswith("autograd")
        r["measured_ceiling_GBps"] = ceilings["copy_GBps"] if rw else ceilings["read_GBps"]
        r["frac_of_measured_ceiling"] = r["GBps"] / r["measured_ceiling_GBps"]
    return rows


def es(dtype) -> int:
    return 8 if dtype == torch.float64 else 4


def nn_kernel_name(dtype, m, n) -> str:
    return tsm.kernel_name(tsm.OP_TSM2R, m, m, n, tsm.F64 if dtype == torch.float64 else tsm.F32)


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
                                    p["tiles"], p["tile_rows"], p["occupancy"], tall=p["tall"])


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
    samples, top_frac, planner_frac, planner_best = [], [], [], 0
    for c in calls:
        r = tune.autotune_tsm2r(c["A"], c["B"], top=1000, pin=False)
        d = r["default"]
        top_frac.append(r["report"][0]["gbs"] / r["best"]["gbs"])
        planner_frac.append(d["gbs"] / r["best"]["gbs"])
        planner_best += d is r["best"]
        for e in sorted(r["report"], key=lambda e: (e["tall"], e["slices"])):
            pr = perf_model.predict_tsm2r(c["m"], c["k"], c["n"], es(c["dtype"]), e["slices"],
                                          e["tiles"], e["tile_rows"], e["occupancy"],
                                          tall=e["tall"])
            mark = " planner" if (e["tall"], e["slices"]) == (d["tall"], d["slices"]) else ""
            mark += " best" if e is r["best"] else ""
            print("%-14s %4d %3d %5d %6d %9.0f %9.0f %7.2f%s" % (
                c["workload"], e["tall"], e["slices"], e["workgroups"], pr.rounds,
                e["pred_gbs"], e["gbs"], e["pred_gbs"] / e["gbs"], mark), flush=True)
            samples.append(dict(m=c["m"], k=c["k"], n=c["n"], es=es(c["dtype"]),
                                slices=e["slices"], tiles=e["tiles"], tile_rows=e["tile_rows"],
                                occupancy=e["occupancy"], tall=e["tall"], seconds=e["seconds"]))

    def rms(dev):
        return float(np.sqrt(np.mean([np.log(perf_model.predict_tsm2r(
            s["m"], s["k"], s["n"], s["es"], s["slices"], s["tiles"], s["tile_rows"],
            s["occupancy"], dev, s["tall"]).seconds / s["seconds"]) ** 2 for s in samples])))
    fitted = perf_model.fit(samples)
    print("plans %d; rms log(pred/meas) with the built-in constants %.3f, refitted %.3f: %s"
          % (len(samples), rms(perf_model.MI355X), rms(fitted), fitted), flush=True)

    def worst(dev, sel):
        return float(np.max([abs(np.log(perf_model.predict_tsm2r(
            s["m"], s["k"], s["n"], s["es"], s["slices"], s["tiles"], s["tile_rows"],
            s["occupancy"], dev, s["tall"]).seconds / s["seconds"])) for s in sel]))
    f64 = [s for s in samples if s["es"] == 8]
    f32 = [s for s in samples if s["es"] == 4]
    fit64 = perf_model.fit(f64)
    rms32 = float(np.sqrt(np.mean([np.log(perf_model.predict_tsm2r(
        s["m"], s["k"], s["n"], s["es"], s["slices"], s["tiles"], s["tile_rows"],
        s["occupancy"], fit64, s["tall"]).seconds / s["seconds"]) ** 2 for s in f32])))
    print("worst |log(pred/meas)|: built-in %.3f, refitted %.3f; fitted on FP64 only, rms on FP32 "
          "%.3f (worst %.3f)" % (worst(perf_model.MI355X, samples), worst(fitted, samples), rms32,
                                 worst(fit64, f32)), flush=True)
    print("model's top plan / best measured: mean %.4f, worst %.4f; planner's plan / best: mean "
          "%.4f, worst %.4f; planner's plan the measured best on %d of %d workloads"
          % (np.mean(top_frac), np.min(top_frac), np.mean(planner_frac), np.min(planner_frac),
             planner_best, len(calls)), flush=True)


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
        tot_b, tot_t, worst, worst_cw = 0.0, 0.0, 0.0, 0.0
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
                Ar = si.matrix_rows(seed + k, si.STREAM_A, m, k, rows, dtype=dtype).double().numpy()
                Bh = si.matrix(seed + k, si.STREAM_B, k, k, dtype=dtype).double().numpy()
                ref = oracle.matmul(Ar, Bh)
                Cs = C[rows].double().cpu().numpy()
                worst = max(worst, oracle.normwise_error(Cs, ref))
                worst_cw = max(worst_cw, oracle.componentwise_error(Cs, ref, Ar, Bh))
                del A, B, C, flush
        torch.cuda.empty_cache()
        out.append({"row": "TSM2L forward (C = A*B, m in 2^20..2^24, k = n in 8..32)",
                    "dtype": str(dtype).replace("torch.", ""), "GBps": tot_b / tot_t / 1e9,
                    "frac_of_8TBps": tot_b / tot_t / 1e9 / PEAK_HBM_GBS,
                    "max_normwise_err": worst, "max_componentwise_err": worst_cw,
                    "tol": TOL[dtype]})
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
                       "err_vs_fp32_values": oracle.normwise_error(Cs, oracle.matmul(Ar, Bh)),
                       "componentwise_err_vs_stored": oracle.componentwise_error(
                           Cs, oracle.matmul(stored, Bh), stored, Bh),
                       "componentwise_err_vs_fp32_values": oracle.componentwise_error(
                           Cs, oracle.matmul(Ar, Bh), Ar, Bh)}
                if t_split is not None:
                    row["split_GBps"] = (m * k * 4 + S.nbytes()) / t_split / 1e9
                out.append(row)
                del S
        del B, C
    del A
    torch.cuda.empty_cache()
    return out


def ag_bytes(kind: str, mode: str, m: int, k: int, n: int) -> dict:
    """Algorithmic bytes of each library call of one forward + backward of
    C = A*B: every operand read once, every result written once.  A counts as
    its stored form (8 or 4 bytes per element, or the two 2-byte planes of the
    split form); B, C, dC, dA, dB as float64 (f64) or float32."""
    s = 8 if mode == "f64" else 4
    sa = 4 if mode in ("bf16_split", "f16_split") else (2 if mode in ("bf16", "f16") else s)
    fwd = sa * m * k + s * (k * n + m * n)
    if kind == "L":
        # fused backward: reads A, dC and B, writes dA and dB
        return {"fwd": fwd, "bwd": sa * m * k + s * (m * n + k * n) + s * (m * k + k * n)}
    return {"fwd": fwd, "grad_a": s * (m * n + k * n + m * k), "grad_b": sa * m * k + s * (m * n + k * n)}


class AGCase:
    """One forward + backward of C = A*B through tsm.matmul and
    torch.autograd.grad, on resident seeded inputs.  For the precision modes
    A is split once here (its storage form, kept across steps) unless
    `split_inside`, where every forward splits it again."""

    def __init__(self, dev, shape, kind, m, k, n, mode, seed, index, split_inside=False):
        self.shape, self.kind, self.m, self.k, self.n, self.mode = shape, kind, m, k, n, mode
        self.seed, self.split_inside = seed, split_inside
        self.dtype = torch.float64 if mode == "f64" else torch.float32
        self.A = si.matrix(seed, si.STREAM_A, m, k, dtype=self.dtype, device=dev).requires_grad_()
        self.B = si.matrix(seed, si.STREAM_B, k, n, dtype=self.dtype, device=dev).requires_grad_()
        self.dC = si.matrix(seed, si.STREAM_DC, m, n, dtype=self.dtype, device=dev, dist="normal")
        lowp = mode not in ("f64", "f32")
        self.Aop = tsm.split(self.A, mode.split("_")[0], lo=mode.endswith("split")) \
            if lowp and not split_inside else self.A
        self.tag_fwd, self.tag_bwd = 2 * index + 1, 2 * index + 2
        self.bytes = ag_bytes(kind, mode, m, k, n)
        self.total_bytes = sum(self.bytes.values())
        self.name = "%s %s" % (shape, mode)

    def run(self):
        tsm.timing_tag(self.tag_fwd)
        C = tsm.matmul(self.Aop, self.B, self.mode, self.kind)
        tsm.timing_tag(self.tag_bwd)
        dA, dB = torch.autograd.grad(C, (self.A, self.B), self.dC)
        tsm.timing_tag(0)
        return C, dA, dB

    def role(self, tag: int, kernel: str):
        """Which call of the pass a kernel launched under `tag` belongs to
        (a key of self.bytes), or None for overhead kernels."""
        fam = kernel.split("<")[0]
        if fam in OVERHEAD_KERNELS:
            return None
        if tag == self.tag_fwd:
            return "fwd"
        if tag != self.tag_bwd:
            return None
        if self.kind == "L":
            return "bwd" if fam == "tsm2l_bwd_kernel" else None
        if fam == "rowtile_kernel":
            return "grad_a"
        if fam in ("tn_kernel", "tn_lp_kernel"):
            return "grad_b"
        return None


def make_ag_cases(dev, modes=AG_MODES, split_inside=False, first_index=0):
    seed = si.config_seed(4)
    cases = []
    for shape, kind, m, k, n in AG_SHAPES:
        for mode in modes:
            cases.append(AGCase(dev, shape, kind, m, k, n, mode, seed,
                                first_index + len(cases), split_inside))
    return cases


def _stored(A: np.ndarray, fmt: int, lo: bool) -> np.ndarray:
    """The values the precision form stores for float32 values A: hi (+ lo),
    split by the oracle."""
    hi, lo_ = oracle_mod().split(np.asfortranarray(A.astype(np.float32)), fmt, with_lo=lo)
    v = oracle_mod().decode_plane(hi, fmt)
    return v + oracle_mod().decode_plane(lo_, fmt) if lo else v


def oracle_mod():
    import oracle
    return oracle


def _errs(got: np.ndarray, ref: np.ndarray, X: np.ndarray, Y: np.ndarray) -> dict:
    o = oracle_mod()
    return {"normwise": o.normwise_error(got, ref), "componentwise": o.componentwise_error(got, ref, X, Y)}


def case_errors(c: AGCase, C, dA, dB) -> dict:
    """C, dA and dB of one pass against the FP64 oracle: sampled rows of C and
    dA; sampled rows of dB (every row for the TSM2L shape, where dB is 16 x 16
    and needs all of A and dC).  The precision form is compared with the
    products of the stored values (hi + lo, split by the oracle) and of the
    float values of A; dA = dC*B^T involves no stored value."""
    o = oracle_mod()
    m, k, n, dt, seed = c.m, c.k, c.n, c.dtype, c.seed
    rng = np.random.default_rng(m + k + n)
    rows = sorted(set([0, 1, m // 3, m // 2 + 7, m - 1] + rng.integers(0, m, 11).tolist()))
    Ar = si.matrix_rows(seed, si.STREAM_A, m, k, rows, dtype=dt).double().numpy()
    Bh = si.matrix(seed, si.STREAM_B, k, n, dtype=dt).double().numpy()
    dCr = si.matrix_rows(seed, si.STREAM_DC, m, n, rows, dtype=dt, dist="normal").double().numpy()
    lowp = c.mode not in ("f64", "f32")
    fmt = o.BF16 if c.mode.startswith("bf16") else o.F16
    lo = c.mode.endswith("split")

    def views(X):
        return {"stored": _stored(X, fmt, lo), "value": X} if lowp else {"value": X}

    def tol(view):
        t = AG_TOL[c.mode]
        return t[view] if isinstance(t, dict) else t

    out = {}
    Cs = C.detach()[rows].double().cpu().numpy()
    out["C"] = {v: dict(_errs(Cs, o.matmul(X, Bh), X, Bh), tol=tol(v))
                for v, X in views(Ar).items()}
    dAs = dA[rows].double().cpu().numpy()
    out["dA"] = {"value": dict(_errs(dAs, o.matmul(dCr, Bh.T), dCr, Bh.T), tol=tol("value"))}
    if c.kind == "L":
        cols = list(range(k))
        Acols = c.A.detach().double().cpu().numpy()     # every row: dB = A^T dC needs all of A
        # row-major dC: the oracle's loop over m then reads each row of dC once
        dCh = np.ascontiguousarray(c.dC.double().cpu().numpy())
        # the device inputs are the seeded generator's values (checked on the sample)
        assert np.array_equal(Acols[rows], Ar) and np.array_equal(dCh[rows], dCr)
    else:
        cols = sorted(set([0, 1, k // 2, k - 1] + rng.integers(0, k, 12).tolist()))
        Acols = si.matrix_cols(seed, si.STREAM_A, m, k, cols, dtype=dt).double().numpy()
        dCh = si.matrix(seed, si.STREAM_DC, m, n, dtype=dt, dist="normal").double().numpy()
    dBs = dB[cols].double().cpu().numpy()
    out["dB"] = {v: dict(_errs(dBs, o.matmul(np.ascontiguousarray(X.T), dCh), X.T, dCh),
                         tol=tol(v)) for v, X in views(Acols).items()}
    out["sample"] = "C, dA: %d rows; dB: %d of %d rows" % (len(rows), len(cols), k)
    ok = all(e["normwise"] <= e["tol"] for key in ("C", "dA", "dB") for e in out[key].values())
    out["ok"] = ok
    return out


def traffic_from_profiles(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    rocprofv3 counter summaries (profiles/*_counters.txt), or None when none
    matches or the summary was taken from other sources than the current ones
    (each summary names its source files and their SHA-256)."""
    import glob
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_counters.txt"))):
        info = {}
        for line in open(path):
            if "=" in line and not line.startswith("#"):
                key, val = line.split("=", 1)
                info[key.strip()] = val.strip()
        if info.get("kernel") != kernel or info.get("workload") != workload:
            continue
        sha = info.get("kernel_source_sha256_16", "")
        files = sha[sha.find("(") + 1:sha.find(")")].split(",") if "(" in sha else []
        if not files or sha.split()[0] != sources_hash(files):
            continue
        try:
            return float(info["hbm_bytes_per_launch"])
        except (KeyError, ValueError):
            continue
    return None


def sources_hash(files) -> str:
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, "paper_2002_03258_amd", "csrc", f.strip()), "rb").read())
    return h.hexdigest()[:16]


# (dtype, m) of the m x 16 TSM2L pattern probes: the TSM2L row shape and the
# headline's TSM2L shape
PATTERN_SHAPES = ((torch.float64, 1 << 24), (torch.float64, 1 << 23), (torch.float32, 1 << 23))
STREAM_CEILINGS = ("read_GBps", "copy_GBps", "write_GBps")


def pattern_key(prefix: str, dtype, m: int) -> str:
    return "%s%s_m%d_k16_GBps" % (prefix, str(dtype).replace("torch.", ""), m)


def ceiling_key(kind: str, mode: str, role: str, m: int) -> str:
    """The measured ceiling (a key of measure_ceilings) with the access mix of
    a headline call: the TSM2L patterns for the TSM2L calls (the bf16 hi and
    lo planes move 4 bytes an element, as float32 does), the streaming read
    for the TSM2R forward and dB (A read, little written), the streaming
    write for the TSM2R dA (dA written, little read)."""
    if kind == "L":
        dt = torch.float64 if mode == "f64" else torch.float32
        return pattern_key("tsm2l_pattern_" if role == "fwd" else "tsm2l_bwd_pattern_", dt, m)
    return "write_GBps" if role == "grad_a" else "read_GBps"


def attach_call_ceilings(line, ceilings):
    """Each timed call's (and the roofline kernel's) fraction of the measured
    ceiling of its access mix."""
    def put(d, key):
        v = ceilings.get(key)
        if v:
            d["measured_ceiling"] = key
            d["measured_ceiling_GBps"] = v
            d["frac_of_measured_ceiling"] = d["GBps" if "GBps" in d else "achieved"] / v
    for case in line["config"]["cases"]:
        for d in case["calls"].values():
            put(d, d["ceiling"])
    if line.get("roofline"):
        put(line["roofline"], line["roofline"]["ceiling"])


def roofline_of(cases, timing):
    """The dominant kernel of the timed steps: the (kernel, tag) row of the
    library's launch timing with the largest total time, its algorithmic
    bytes per launch (the bytes of the call it serves) over its average
    launch time."""
    by_tag = {}
    for c in cases:
        by_tag[c.tag_fwd] = c
        by_tag[c.tag_bwd] = c
    best = None
    for r in timing:
        c = by_tag.get(r["tag"])
        if c is None or c.role(r["tag"], r["kernel"]) is None:
            continue
        if best is None or r["total_ms"] > best[0]["total_ms"]:
            best = (r, c)
    if best is None:
        return None
    r, c = best
    role = c.role(r["tag"], r["kernel"])
    per_launch = c.bytes[role]
    avg_s = r["total_ms"] / 1e3 / r["launches"]
    achieved = per_launch / avg_s / 1e9
    workload = "autograd:%s:%s:%s" % (c.mode, c.kind, role)
    traffic = traffic_from_profiles(r["kernel"], workload)
    return {"bound": "hbm", "kernel": r["kernel"], "call": "%s, %s" % (c.name, role),
            "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS, "avg_launch_us": avg_s * 1e6,
            "launches": r["launches"], "algorithmic_bytes_per_launch": per_launch,
            "workload": workload, "traffic": traffic,
            "traffic_over_algorithmic": (traffic / per_launch) if traffic else None,
            "ceiling": ceiling_key(c.kind, c.mode, role, c.m)}


def headline(dev, steps, warmup, check=True):
    """The timed step: the four forward + backward passes."""
    cases = make_ag_cases(dev)
    torch.cuda.synchronize()
    for _ in range(warmup):
        for c in cases:
            c.run()
    torch.cuda.synchronize()
    evs = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            for _ in cases] for _ in range(steps)]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    last = [None] * len(cases)
    # the timed steps: nothing but the passes between the two events
    torch.cuda.synchronize()
    e0.record()
    for s in range(steps):
        for i, c in enumerate(cases):
            last[i] = c.run()
    e1.record()
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    # the same steps again with every pass and every kernel launch timed
    # (an event pair around each: per-pass times and the roofline)
    tsm.timing_start()
    for s in range(steps):
        for i, c in enumerate(cases):
            evs[s][i][0].record()
            last[i] = c.run()
            evs[s][i][1].record()
    torch.cuda.synchronize()
    tsm.timing_stop()
    timing = tsm.timing_collect()
    step_bytes = sum(c.total_bytes for c in cases)
    value = step_bytes * steps / (total_ms / 1e3) / 1e9
    per_case = []
    for i, c in enumerate(cases):
        t = float(np.median([evs[s][i][0].elapsed_time(evs[s][i][1]) for s in range(steps)])) / 1e3
        calls = {}
        for r in timing:
            role = c.role(r["tag"], r["kernel"]) if r["tag"] in (c.tag_fwd, c.tag_bwd) else None
            if role is not None:
                d = calls.setdefault(role, {"kernels": [], "ms_per_launch": 0.0})
                d["kernels"].append(r["kernel"])
                d["ms_per_launch"] += r["total_ms"] / r["launches"]
        for role, d in calls.items():
            d["GBps"] = c.bytes[role] / (d["ms_per_launch"] / 1e3) / 1e9
            d["bytes"] = c.bytes[role]
            d["ceiling"] = ceiling_key(c.kind, c.mode, role, c.m)
        per_case.append({"case": c.name, "shape": (c.m, c.k, c.n), "mode": c.mode,
                         "bytes": c.total_bytes, "ms_median": t * 1e3,
                         "GBps": c.total_bytes / t / 1e9,
                         "frac_of_8TBps": c.total_bytes / t / 1e9 / PEAK_HBM_GBS,
                         "calls": calls})
    modes = {}
    for mode in AG_MODES:
        sel = [p for p in per_case if p["mode"] == mode]
        b = sum(p["bytes"] for p in sel)
        t = sum(p["ms_median"] for p in sel) / 1e3
        modes[mode] = {"GBps": b / t / 1e9, "ms": t * 1e3, "frac_of_8TBps": b / t / 1e9 / PEAK_HBM_GBS}
    speedup = {}
    for shape, *_ in AG_SHAPES:
        t64 = [p["ms_median"] for p in per_case if p["case"] == "%s f64" % shape][0]
        tsp = [p["ms_median"] for p in per_case if p["case"] == "%s bf16_split" % shape][0]
        speedup[shape] = t64 / tsp
    timed_ms = sum(evs[s][i][0].elapsed_time(evs[s][i][1]) for s in range(steps)
                   for i in range(len(cases))) / steps
    res = {"value": value, "ms_per_step": total_ms / steps, "bytes_per_step": step_bytes,
           "ms_per_step_with_launch_timing": timed_ms,
           "cases": per_case, "modes": modes, "bf16_split_speedup_over_f64": speedup,
           "roofline": roofline_of(cases, timing),
           "kernel_timing": [dict(r, case=next((c.name for c in cases
                                                if r["tag"] in (c.tag_fwd, c.tag_bwd)), None))
                             for r in timing]}
    if check:
        res["err"] = {}
        for i, c in enumerate(cases):
            res["err"][c.name] = case_errors(c, *last[i])
            print("checked %s against the oracle" % c.name, file=sys.stderr, flush=True)
    del last, cases
    torch.cuda.empty_cache()
    return res


def measure_ceilings(dev):
    """HBM ceilings of this device with 16-byte non-temporal accesses: a
    4 GiB linear read, a 2 GiB copy, a 4 GiB write, and the TSM2L tile
    patterns without arithmetic on m x 16 FP64 (m = 2^24, 2^23) and FP32
    (m = 2^23): the forward's (A read once, a column permutation of A written
    once) and the fused backward's (two such inputs read, one output
    written).  Each the median of 5 runs after a warm-up; GB/s counts the
    bytes moved."""
    out = {}
    big = torch.empty(1 << 32, dtype=torch.uint8, device=dev).fill_(1)
    dst = torch.empty(1 << 32, dtype=torch.uint8, device=dev)
    half = 1 << 31
    t = timed(lambda: tsm.probe_stream("read", dst, big))
    out["read_GBps"] = big.numel() / t / 1e9
    t = timed(lambda: tsm.probe_stream("copy", dst, big, nbytes=half))
    out["copy_GBps"] = 2 * half / t / 1e9
    t = timed(lambda: tsm.probe_stream("write", dst))
    out["write_GBps"] = dst.numel() / t / 1e9
    del big, dst
    for dt, m in PATTERN_SHAPES:
        X = si.matrix(si.config_seed(9), si.STREAM_A, m, 16, dtype=dt, device=dev)
        Y = si.matrix(si.config_seed(9), si.STREAM_B, m, 16, dtype=dt, device=dev)
        O = tsm.empty_colmajor(m, 16, dt, dev)
        t = timed(lambda: tsm.probe_tiles(X, O))
        out[pattern_key("tsm2l_pattern_", dt, m)] = 2 * X.numel() * X.element_size() / t / 1e9
        t = timed(lambda: tsm.probe_tiles(X, O, Y=Y))
        out[pattern_key("tsm2l_bwd_pattern_", dt, m)] = 3 * X.numel() * X.element_size() / t / 1e9
        del X, Y, O
    torch.cuda.empty_cache()
    out["note"] = ("16-byte non-temporal loads/stores; read 4 GiB, copy 2 GiB -> 2 GiB (bytes "
                   "read + written), write 4 GiB; TSM2L pattern = the rowtile kernel's loads and "
                   "stores without the matrix-core work; TSM2L bwd pattern = the fused backward's "
                   "(two inputs read, one output written)")
    return out


def cpu_baseline():
    """The FP64 oracle on row samples of the headline workload, forward and
    backward (C, dA and dB's share of the sampled rows), on all of the host's
    cores and on one; each sample sized for a few seconds."""
    o = oracle_mod()
    seed = si.config_seed(4)
    cores = o.threads()

    def one(shape, kind, m, k, n, rows):
        A = si.matrix_rows(seed, si.STREAM_A, m, k, list(range(rows))).numpy()
        B = si.matrix(seed, si.STREAM_B, k, n).numpy()
        dC = si.matrix_rows(seed, si.STREAM_DC, m, n, list(range(rows)), dist="normal").numpy()
        t0 = time.perf_counter()
        o.matmul(A, B)
        o.matmul(dC, B.T)
        o.matmul(np.ascontiguousarray(A.T), dC)
        dt = time.perf_counter() - t0
        return sum(ag_bytes(kind, "f64", rows, k, n).values()), dt

    def run(target_s):
        tot_b, tot_t, desc = 0.0, 0.0, []
        for shape, kind, m, k, n in AG_SHAPES:
            probe = max(64, min(m, 4096 if kind == "R" else 1 << 16) // 64)
            b, t = one(shape, kind, m, k, n, probe)
            rows = int(min(m, max(probe, probe * target_s / max(t, 1e-4))))
            b, t = one(shape, kind, m, k, n, rows)
            tot_b += b
            tot_t += t
            desc.append("%d of %d rows of the %s shape" % (rows, m, shape))
        return tot_b / tot_t / 1e9, tot_t, desc

    v_all, t_all, d_all = run(5.0)
    o.set_threads(1)
    v_one, t_one, d_one = run(3.0)
    o.set_threads(cores)
    return {"value": v_all, "unit": "GB/s", "cores": cores, "kind": "oracle", "seconds": t_all,
            "single_thread_value": v_one, "single_thread_seconds": t_one,
            "cpu_model": _cpu_model(),
            "sample": "FP64 forward + backward (C = A*B, dA = dC*B^T, dB = A^T*dC) of the autograd "
                      "workloads on row samples, all cores: %s; one core: %s; algorithmic bytes of "
                      "the samples over the oracle's time" % ("; ".join(d_all), "; ".join(d_one))}


def rows_autograd_more(dev):
    """Forward + backward of the same workloads in FP32 (the precision form's
    baseline: same 4 bytes per element of A as the split form), and in
    bf16-split with the split of A inside every pass (a float32 A that
    changes every step).  GB/s counts the algorithmic bytes of the pass; the
    split's own traffic is not counted (its time is)."""
    out = []
    cases = make_ag_cases(dev, modes=("f32",)) + \
        make_ag_cases(dev, modes=("bf16_split",), split_inside=True, first_index=2)
    for c in cases:
        res = {}

        def run():
            res["r"] = c.run()
        t = timed(run)
        err = case_errors(c, *res["r"])
        out.append({"row": "autograd fwd+bwd %s shape m=%d k=%d n=%d%s" % (
            c.shape, c.m, c.k, c.n, ", A split inside every pass" if c.split_inside else ""),
            "dtype": c.mode, "GBps": c.total_bytes / t / 1e9,
            "frac_of_8TBps": c.total_bytes / t / 1e9 / PEAK_HBM_GBS, "ms": t * 1e3, "err": err})
        del res
    del cases
    torch.cuda.empty_cache()
    return out


def rows_tsm2r_grid(dev, steps=5, check=True, tune_plans=False):
    """The TSM2R grid: 24 products C = A*B, square A (m = k in {10240, 20480,
    30720}), n in {2, 4, 8, 16}, FP64 and FP32, as one timed sequence
    (`tune_plans`: each product's plan autotuned first)."""
    calls = make_r_inputs(dev)
    tuned = None
    if tune_plans:
        tuned = {}
        for c in calls:
            r = tune.autotune_tsm2r(c["A"], c["B"], top=4)
            tuned[c["workload"]] = {"slices": r["best"]["slices"], "tall": r["best"]["tall"],
                                    "gain": r["best"]["gbs"] / r["default"]["gbs"]}
    for _ in range(2):
        run_step(calls)
    torch.cuda.synchronize()
    evs = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)]
            for _ in calls] for _ in range(steps)]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for s in range(steps):
        run_step(calls, evs[s])
    e1.record()
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    step_bytes = sum(c["bytes"] for c in calls)
    v = step_bytes * steps / (total_ms / 1e3) / 1e9
    row = {"row": "TSM2R grid (C = A*B, m = k in 10240..30720, n in 2..16, 24 products)",
           "dtype": "f64+f32", "GBps": v, "frac_of_8TBps": v / PEAK_HBM_GBS,
           "ms_per_pass": total_ms / steps,
           "model": model_summary(calls, evs, step_bytes, v)}
    if tuned is not None:
        row["tuned_plans"] = tuned
    if check:
        row["check"] = check_calls(calls)
    del calls
    torch.cuda.empty_cache()
    return [row]


def profile_op(dev, spec):
    """Launch one workload 5 times and nothing else (for rocprofv3 counters):
    tsm2l:DT:M:K (B k x k), kmeans:DT:M:K[:row], or autograd:MODE:KIND (one
    forward + backward of the autograd workload of that shape, KIND L or R)."""
    f = spec.split(":")
    if f[0] == "autograd":
        mode, kind = f[1], f[2]
        shape = [s for s in AG_SHAPES if s[1] == kind][0]
        c = AGCase(dev, shape[0], kind, shape[2], shape[3], shape[4], mode, si.config_seed(4), 0)
        run = c.run
    elif f[0] == "lowp":
        # lowp:FORM:M:N, FORM bf16 / bf16_split / f16 / f16_split: the split of
        # a square float A, then the precision-form TSM2R product 5 times
        form, m, n = f[1], int(f[2]), int(f[3])
        A = si.matrix(si.config_seed(3), si.STREAM_A, m, m, dtype=torch.float32, device=dev)
        B = si.matrix(si.config_seed(3) + n, si.STREAM_B, m, n, dtype=torch.float32, device=dev)
        S = tsm.split(A, form.split("_")[0], lo=form.endswith("split"))
        del A
        C = tsm.empty_colmajor(m, n, torch.float32, dev)
        run = lambda: tsm.tsm2r(S, B, out=C)
    elif f[0] == "grid":
        # grid:DT:M:N, one TSM2R product of the square grid
        dtype, m, n = torch.float64 if f[1] == "f64" else torch.float32, int(f[2]), int(f[3])
        seed = si.config_seed(1)
        A = si.matrix(seed, si.STREAM_A, m, m, dtype=dtype, device=dev)
        B = si.matrix(seed + n, si.STREAM_B, m, n, dtype=dtype, device=dev)
        C = tsm.empty_colmajor(m, n, dtype, dev)
        run = lambda: tsm.tsm2r(A, B, out=C)
    else:
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
            raise SystemExit("--profile-op: tsm2l, kmeans, autograd, lowp or grid")
    for _ in range(5):
        run()
    torch.cuda.synchronize()
    print("launched %s 5 times" % spec, flush=True)


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
    ap.add_argument("--profile-op", default=None, metavar="SPEC",
                    help="only launch one workload 5 times, for rocprofv3 counters: "
                         "tsm2l:DT:M:K, kmeans:DT:M:K[:row], autograd:MODE:KIND, "
                         "lowp:FORM:M:N or grid:DT:M:N, e.g. tsm2l:f64:16777216:16, "
                         "autograd:f64:L or lowp:bf16_split:32768:8")
    ap.add_argument("--profile-copy", action="store_true",
                    help="only run a 1 GiB device copy 5 times (counter calibration)")
    ap.add_argument("--ceiling", action="store_true",
                    help="only measure the HBM ceilings (stream and TSM2L-pattern probes) and "
                         "print them")
    ap.add_argument("--tune", action="store_true",
                    help="autotune the plan of each TSM2R grid workload before it is timed")
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
    if args.ceiling:
        print(json.dumps({"ceilings": measure_ceilings(dev)}), flush=True)
        return
    if args.profile_op:
        profile_op(dev, args.profile_op)
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
    if args.model_report:
        model_report(make_r_inputs(dev))
        return

    t_setup = time.perf_counter()
    h = headline(dev, args.steps, args.warmup, check=not args.no_check)
    print("headline timed (setup + timing %.1f s)" % (time.perf_counter() - t_setup),
          file=sys.stderr, flush=True)
    clocks = gpu_clocks()
    shapes = "; ".join("%s A %dx%d, B %dx%d" % (s, m, k, k, n) for s, _, m, k, n in AG_SHAPES)
    line = {
        "metric": METRIC, "value": h["value"], "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": h["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64 vs bf16_split",
        "data": "synthetic (seeded counter-based uniform[-1,1] A, B; N(0,1)-like dC)",
        "config": {"workload": "autograd forward + backward of C = A*B (dA = dC*B^T, "
                               "dB = A^T*dC), FP64 and bf16-split (A stored as bf16 hi + lo "
                               "planes; B, C, dA, dB float32), " + shapes,
                   "bytes_per_step": h["bytes_per_step"],
                   "frac_of_8TBps": h["value"] / PEAK_HBM_GBS,
                   "modes": h["modes"],
                   "bf16_split_speedup_over_f64": h["bf16_split_speedup_over_f64"],
                   "cases": h["cases"], "gpu_clocks_after_timing": clocks,
                   "ms_per_step_with_launch_timing": h["ms_per_step_with_launch_timing"]},
        "roofline": h["roofline"],
        "kernel_timing": h["kernel_timing"],
    }
    if "err" in h:
        line["err"] = h["err"]
    ceil = measure_ceilings(dev)
    line["ceilings"] = ceil
    line["config"]["frac_of_measured_copy_ceiling"] = h["value"] / ceil["copy_GBps"]
    attach_call_ceilings(line, ceil)
    print("ceilings measured", file=sys.stderr, flush=True)
    if not args.no_rows:
        rows = []
        for fn in (rows_tsm2r_grid, rows_tsm2l, rows_lowp, rows_autograd_more, rows_general,
                   rows_kmeans):
            rows += fn(dev, tune_plans=True) if (fn is rows_tsm2r_grid and args.tune) else fn(dev)
            print("rows: %s done" % fn.__name__, file=sys.stderr, flush=True)
        line["rows"] = attach_ceilings(rows, ceil)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
