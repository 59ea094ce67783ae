"""Performance model of the TSM2R kernel, re-parameterised for gfx950.

The paper sizes TSM2R from a parameter-based model (Design of TSM2R,
performance model and parameter choice, Algorithm 5):

- the kernel is memory-bound while n stays below the ridge
  t2_threshold = PeakPerf / PeakBand * bytes_per_element;
- its bandwidth utilisation follows Little's law: the loads of A in flight
  per SM (occupancy times t3 per thread) against the concurrency the memory
  system needs, latency_mem * PeakBand / #SM;
- occupancy is estimated from registers and shared memory per thread, and
  latency_mem comes from offline profiling.

The same terms, counted the gfx950 way:

- occupancy is the runtime's occupancy query of the compiled kernel (the
  plan query reports it), not a register estimate;
- concurrency is counted in bytes: a wavefront keeps one 8 KB chunk of A in
  flight (RG * ST 16-byte loads per lane), or two where the kernel holds the
  next chunk in flight across its waits (the library turns that on per plan;
  `chunks_in_flight` restates its rule), a workgroup 4 wavefronts;
- the grid is finite: W = tiles * S workgroups run in rounds of at most
  CUs * occupancy, and a last partial round runs at the concurrency it has;
- a k split S > 1 adds its double partials (written by the kernel, read back
  by the reduction) and a second launch.

latency_mem, the attainable streaming rate and the launch cost are measured
constants, as in the paper.  `predict_tsm2r` gives the time and rate of one
plan; the autotuner (`tune.py`) ranks candidate plans with it and times the
best few.
"""
from __future__ import annotations

import math
from dataclasses import dataclass


@dataclass(frozen=True)
class Device:
    """Figures of the GPU the model is evaluated for (MI355X defaults)."""
    cus: int = 256
    clock_ghz: float = 2.4
    peak_band_gbs: float = 8000.0      # HBM3E datasheet
    peak_fp64_gflops: float = 78600.0  # vector FP64
    peak_fp32_gflops: float = 157300.0
    stream_gbs: float = 7090.0         # measured: 16-byte streaming read of one large buffer
    # fitted by `fit` to the measured rates of every candidate plan of the 24
    # square TSM2R products (m = k in {10240, 20480, 30720}, n in {2, 4, 8, 16},
    # FP64 and FP32; 816 plans, timed after a warm-up in shuffled rounds):
    latency_us: float = 1.51           # loaded memory latency
    eta: float = 0.946                 # fraction of the streaming rate reached at full concurrency
    balance_exp: float = 0.53          # weight of the per-CU balance term
    t0_us: float = 7.4                 # fixed cost per product (launches, ramp-up, drain)
    round_us: float = 3.4              # cost of each round of resident workgroups


MI355X = Device()

WAVES_PER_WG = 4
INFLIGHT_PER_WAVE = 8192               # bytes of A a wavefront keeps in flight


def t2_threshold(peak_perf_gflops: float, peak_band_gbs: float, bytes_per_elem: int) -> float:
    """Columns of C per pass below which streaming A is memory-bound: the
    ridge where compute time equals memory time."""
    return peak_perf_gflops / peak_band_gbs * bytes_per_elem


def regime(n: int, bytes_per_elem: int, dev: Device = MI355X) -> str:
    """'memory' or 'compute' for a TSM2R product of n columns."""
    perf = dev.peak_fp64_gflops if bytes_per_elem == 8 else dev.peak_fp32_gflops
    return "memory" if n <= t2_threshold(perf, dev.peak_band_gbs, bytes_per_elem) else "compute"


def concurrent_max_mem(dev: Device = MI355X) -> float:
    """Bytes a CU must keep in flight to sustain its share of the streaming
    rate (Little's law: latency times throughput)."""
    return dev.latency_us * 1e-6 * dev.stream_gbs * 1e9 / dev.cus


def util_mem(bytes_in_flight_per_cu: float, dev: Device = MI355X) -> float:
    """Fraction of the streaming rate reached with this concurrency per CU."""
    if bytes_in_flight_per_cu <= 0:
        return 0.0
    return min(1.0, bytes_in_flight_per_cu / concurrent_max_mem(dev))


def chunks_in_flight(n: int, es: int, tall: int, workgroups: int, cus: int) -> int:
    """Chunks of A a wavefront of the library's TSM2R kernel keeps in flight:
    two where the library holds the next chunk in flight (the shorter tiles
    only; n > 16, FP32 with n <= 4, or a grid of 7/8 to all of the CUs), one
    otherwise."""
    if tall:
        return 1
    if n > 16 or (es == 4 and n <= 4):
        return 2
    return 2 if workgroups <= cus and 8 * workgroups >= 7 * cus else 1


def algorithmic_bytes(m: int, k: int, n: int, es: int) -> int:
    """A and B read once, C written once."""
    return es * (m * k + k * n + m * n)


@dataclass(frozen=True)
class Prediction:
    seconds: float
    gbs: float                 # algorithmic bytes per second / 1e9
    rounds: int                # rounds of resident workgroups
    tail_util: float           # utilisation of the last (partial) round
    partial_bytes: int


def balance(a: int, cus: int) -> float:
    """Mean over maximum workgroups per CU when `a` workgroups are spread over
    `cus` CUs (1 when every CU holds the same number or some hold none)."""
    if a < cus:
        return 1.0
    return (a / cus) / math.ceil(a / cus)


def predict_tsm2r(m: int, k: int, n: int, es: int, slices: int, tiles: int, tile_rows: int,
                  occupancy: int, dev: Device = MI355X, tall: int = 0) -> Prediction:
    """Time of one TSM2R product with a given plan (k split `slices`, `tiles`
    row tiles of `tile_rows`, `occupancy` workgroups per CU, `tall` tiles).

    Each round of resident workgroups streams its share of A at
    eta * stream * util_mem * balance ** balance_exp; a split adds its
    partials' round trip and the fixed cost t0 covers the launches."""
    W = tiles * slices
    slots = dev.cus * max(1, occupancy)
    np_ = 16 if n <= 16 else 32
    partial = W * np_ * tile_rows * 8 if slices > 1 else 0
    bw = dev.stream_gbs * 1e9
    # each workgroup streams its share of A (and writes its partial or C rows)
    per_wg = (es * m * k + partial + (0 if slices > 1 else es * m * n)) / W
    full, rem = divmod(W, slots)
    rounds = [slots] * full + ([rem] if rem else [])
    t = dev.t0_us * 1e-6
    u = 0.0
    chunks = chunks_in_flight(n, es, tall, W, dev.cus)
    for a in rounds:
        u = util_mem(a * WAVES_PER_WG * INFLIGHT_PER_WAVE * chunks / dev.cus, dev)
        t += a * per_wg / (dev.eta * bw * u * balance(a, dev.cus) ** dev.balance_exp)
        t += dev.round_us * 1e-6
    if slices > 1:
        t += (partial + es * m * n) / bw
    return Prediction(t, algorithmic_bytes(m, k, n, es) / t / 1e9, len(rounds), u, partial)


def fit(samples, dev: Device = MI355X) -> Device:
    """Fit latency_us, eta, balance_exp, t0_us and round_us to measured plans.

    samples: dicts with m, k, n, es, slices, tiles, tile_rows, occupancy,
    optionally tall, and the measured `seconds`.  Minimises the squared log ratio of predicted to
    measured time (scipy's bounded least squares)."""
    from dataclasses import replace

    from scipy.optimize import least_squares

    def resid(x):
        d = replace(dev, latency_us=x[0], eta=x[1], balance_exp=x[2], t0_us=x[3], round_us=x[4])
        return [math.log(predict_tsm2r(s["m"], s["k"], s["n"], s["es"], s["slices"], s["tiles"],
                                       s["tile_rows"], s["occupancy"], d,
                                       s.get("tall", 0)).seconds / s["seconds"])
                for s in samples]

    r = least_squares(resid, [dev.latency_us, dev.eta, dev.balance_exp, dev.t0_us, dev.round_us],
                      bounds=([0.2, 0.3, 0.0, 0.0, 0.0], [10.0, 1.2, 4.0, 500.0, 500.0]))
    return replace(dev, latency_us=float(r.x[0]), eta=float(r.x[1]), balance_exp=float(r.x[2]),
                   t0_us=float(r.x[3]), round_us=float(r.x[4]))


def rank(m: int, k: int, n: int, es: int, plans, dev: Device = MI355X):
    """Plans (dicts with slices, tiles, tile_rows, occupancy, optionally tall)
    sorted by predicted time, each with its prediction attached as 'pred'."""
    out = []
    for p in plans:
        pr = predict_tsm2r(m, k, n, es, p["slices"], p["tiles"], p["tile_rows"], p["occupancy"],
                           dev, p.get("tall", 0))
        out.append(dict(p, pred=pr))
    return sorted(out, key=lambda p: (p["pred"].seconds, p["slices"]))


def knee_workgroups(dev: Device = MI355X) -> int:
    """Resident workgroups at which Little's law is first satisfied (4
    wavefronts of 8 KB each)."""
    return math.ceil(concurrent_max_mem(dev) * dev.cus / (WAVES_PER_WG * INFLIGHT_PER_WAVE))
