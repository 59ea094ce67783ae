"""Empirical autotuner for the TSM2R launch plan.

The paper fixes t2 and t3 from its performance model and picks t1 (and, for
TSM2L, tcf) by offline profiling on each GPU (Algorithm 5 and the text after
it).  Here the plan of a TSM2R product has two free choices, the k split S
and the tile height; the library's planner takes them from the occupancy
query and a measured target, and this tuner replaces that guess for one shape
by measurement on the caller's own operands:

1. enumerate the distinct plans (every S the planner's rounding can produce,
   both tile heights), asking the library what each would launch;
2. rank them with the performance model (`model.predict_tsm2r`);
3. time the best few, and the planner's own choice, with HIP events on the
   current stream.  Every candidate runs once first (so the library's
   grow-only workspace reaches its final size), then the GPU is warmed up
   (it takes some tens of milliseconds of load to reach its steady clocks,
   and whatever is timed first otherwise looks slow); the candidates are
   then timed in rounds, each in its own (seeded) random order so that no
   plan always follows the same one, each sample a block of back-to-back
   calls, and each plan's median is kept;
4. pin the fastest for that shape (`pin_tsm2r`), so later calls use it.

Every candidate computes the same product (up to the order of the k sums), so
tuning never changes results beyond rounding.
"""
from __future__ import annotations

import random

import torch

from . import F32, F64, empty_colmajor, pin_tsm2r, tsm2r, tsm2r_plan, unpin_tsm2r
from . import model


def candidates(m: int, k: int, n: int, dtype: int, max_rounds: int = 3,
               max_partial_frac: float = 0.1) -> list:
    """Distinct plans the library can launch for this shape: dicts of the
    plan query for each tile height and k split S whose grid needs at most
    `max_rounds` rounds of resident workgroups and whose split partials stay
    below `max_partial_frac` of A's bytes.  Leaves the shape unpinned."""
    es = 8 if dtype == F64 else 4
    seen, out = set(), []
    try:
        for tall in (0, 1):
            pin_tsm2r(m, k, n, dtype, 1, tall)
            base = tsm2r_plan(m, k, n, dtype)
            slots = base["cus"] * base["occupancy"]
            s_hi = max(1, (max_rounds * slots) // base["tiles"])
            for S in range(1, min(s_hi, k) + 1):
                pin_tsm2r(m, k, n, dtype, S, tall)
                p = tsm2r_plan(m, k, n, dtype)
                key = (p["tall"], p["slices"])
                if key in seen:
                    continue
                np_ = 16 if n <= 16 else 32
                part = p["workgroups"] * np_ * p["tile_rows"] * 8 if p["slices"] > 1 else 0
                if part > max_partial_frac * es * m * k:
                    continue
                seen.add(key)
                out.append(p)
    finally:
        unpin_tsm2r(m, k, n, dtype)
    return out


def _warm(fn, seconds: float = 0.1, min_calls: int = 3) -> None:
    """Run fn() until `seconds` of GPU time have passed (and min_calls)."""
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    calls = 0
    while True:
        fn()
        calls += 1
        e1 = torch.cuda.Event(enable_timing=True)
        e1.record(st)
        e1.synchronize()
        if calls >= min_calls and e0.elapsed_time(e1) >= seconds * 1e3:
            return


def _time_block(fn, reps: int) -> float:
    """Seconds per call of `reps` back-to-back runs of fn() on the current
    stream, timed as one block."""
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        fn()
    e1.record(st)
    e1.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / reps


def autotune_tsm2r(A: torch.Tensor, B: torch.Tensor, top: int = 6, reps: int = 4,
                   rounds: int = 5, warm_seconds: float = 0.2, pin: bool = True) -> dict:
    """Tune the TSM2R plan of C = A*B (A column-major F64/F32 m x k on the
    GPU, B k x n, n <= 32) on these operands.

    Returns {"best": plan, "default": plan, "report": [...]}: each report
    entry is a plan with its model prediction (`pred_gbs`) and, for the timed
    ones, the measured rate (`gbs`, algorithmic bytes per second / 1e9).
    With `pin`, the fastest plan is pinned for this shape; otherwise the
    shape is left unpinned (a previous pin is removed either way)."""
    if A.dtype not in (torch.float64, torch.float32):
        raise TypeError("autotune_tsm2r: F64 or F32 operands")
    m, k = A.shape
    n = B.shape[1]
    if n > 32:
        raise ValueError("autotune_tsm2r: n <= 32 (wider products run in 32-column panels)")
    dt = F64 if A.dtype == torch.float64 else F32
    es = A.element_size()
    cands = candidates(m, k, n, dt)
    default = tsm2r_plan(m, k, n, dt)
    if not any(p["tall"] == default["tall"] and p["slices"] == default["slices"] for p in cands):
        cands.append(default)
    ranked = model.rank(m, k, n, es, cands)
    chosen = ranked[:top]
    if not any(p["tall"] == default["tall"] and p["slices"] == default["slices"] for p in chosen):
        chosen.append(next(p for p in ranked
                           if p["tall"] == default["tall"] and p["slices"] == default["slices"]))
    C = empty_colmajor(m, n, A.dtype, A.device)
    alg = model.algorithmic_bytes(m, k, n, es)
    for p in chosen:                             # workspace at its final size
        pin_tsm2r(m, k, n, dt, p["slices"], p["tall"])
        tsm2r(A, B, out=C)
    unpin_tsm2r(m, k, n, dt)
    _warm(lambda: tsm2r(A, B, out=C), warm_seconds)
    times = [[] for _ in chosen]
    order = list(range(len(chosen)))
    rng = random.Random(1234)
    for _ in range(rounds):
        rng.shuffle(order)
        for i in order:
            p = chosen[i]
            pin_tsm2r(m, k, n, dt, p["slices"], p["tall"])
            tsm2r(A, B, out=C)                   # first call of this plan untimed
            times[i].append(_time_block(lambda: tsm2r(A, B, out=C), reps))
    report = []
    for p in ranked:
        entry = {key: p[key] for key in ("tall", "slices", "tiles", "tile_rows", "occupancy",
                                          "workgroups", "kernel")}
        entry["pred_gbs"] = p["pred"].gbs
        for i, c in enumerate(chosen):
            if p is c:
                ts = sorted(times[i])
                entry["seconds"] = ts[len(ts) // 2]
                entry["gbs"] = alg / entry["seconds"] / 1e9
        report.append(entry)
    timed = [e for e in report if "gbs" in e]
    best = max(timed, key=lambda e: e["gbs"])
    if pin:
        pin_tsm2r(m, k, n, dt, best["slices"], best["tall"])
    else:
        unpin_tsm2r(m, k, n, dt)
    d = next(e for e in timed
             if e["tall"] == default["tall"] and e["slices"] == default["slices"])
    return {"best": best, "default": d, "report": report}
