"""Benchmark of the checkerboard Metropolis sweep on one MI355X.

Default workload (single large lattice): q = 6, L = 32768 (2^30 uint8 spins),
beta = beta_c(6) = ln(1 + sqrt 6), one lattice from the ordered start and one
from the random start (seed 1), per-sweep int64 energy and q-bin population
records.  One step = one full sweep (colour 0 then colour 1, records included)
of both lattices.  The timed region holds exactly --steps sweeps of each
lattice, right after its first --warmup sweeps (untimed; the first call packs
the lattice into its colour-split copy).

Prints one JSON line: ns per spin flip (whole-job wall time / site updates),
the roofline of the dominant kernel (the half-sweep kernel, timed with events
on its own stream), the serial CPU oracle timed on a bounded sample, and the
metric's other two parts at their workloads' own sizes: batched replicas in
jobs/s beside the plain one-lattice-at-a-time loop, and the serving burst in
jobs/s with p50/p99 latency; and the plain method and the metastability
ramps in ns per spin flip (--no-extras skips these four).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 64 lanes of full-rate 32-bit VALU issue x 2.4 GHz
VALU_PEAK_OPS = 256 * 64 * 2.4e9
HBM_PEAK_GBS = 8000.0
# one Philox4x32-10 block = 10 rounds x (2 v_mad_u64_u32 + 2 v_bitop3_b32) = 40
# full-rate VALU instructions, and serves two site updates
ALGO_OPS_PER_SITE = 20.0
# a sweep reads and writes every uint8 spin once: 2 bytes per site update
ALGO_BYTES_PER_SITE = 2.0
KERNEL_SOURCES = ["paper_1101_0876_amd/csrc/packed.hip", "paper_1101_0876_amd/csrc/sweep_row.hpp",
                  "paper_1101_0876_amd/csrc/device.hpp", "paper_1101_0876_amd/csrc/kernels.hpp"]
# the simple-cubic workload's dominant kernel
CUBE_SOURCES = ["paper_1101_0876_amd/csrc/cubic_packed.hip", "paper_1101_0876_amd/csrc/cubic.hpp",
                "paper_1101_0876_amd/csrc/sweep_row.hpp", "paper_1101_0876_amd/csrc/device.hpp",
                "paper_1101_0876_amd/csrc/kernels.hpp"]
# the first-plus-second-neighbour workload's kernels (one sweep)
NNN_SOURCES = ["paper_1101_0876_amd/csrc/nnn.hip", "paper_1101_0876_amd/csrc/sweep_row.hpp",
               "paper_1101_0876_amd/csrc/device.hpp", "paper_1101_0876_amd/csrc/kernels.hpp"]
# the mid-size workload's kernel (64 sweeps per launch)
MID_SOURCES = ["paper_1101_0876_amd/csrc/band.hip", "paper_1101_0876_amd/csrc/band.hpp", "paper_1101_0876_amd/csrc/sweep_row.hpp",
               "paper_1101_0876_amd/csrc/device.hpp", "paper_1101_0876_amd/csrc/kernels.hpp"]
SOURCES_OF = {"large": KERNEL_SOURCES, "cubic": CUBE_SOURCES, "nnn": NNN_SOURCES, "mid": MID_SOURCES}


def kernel_hash(sources=None) -> str:
    """Hash of the dominant kernel's sources without comments and blank space, so
    edits of comments keep counter data taken on the same code valid."""
    h = hashlib.sha256()
    for rel in sources or KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel)) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def counter_traffic(workload: str):
    """HBM bytes per launch of the dominant kernel (per sweep for the nnn
    workload, per 64-sweep launch for the mid-size one) from the committed
    rocprofv3 --pmc summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_hash") != kernel_hash(SOURCES_OF.get(workload)):
        return None
    return rec.get("bytes_per_launch")


def host_cpu() -> str:
    """The host's CPU model and hardware thread count (the oracle runs on one)."""
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{model}, {os.cpu_count()} hardware threads visible"


def cpu_baseline(seconds_target: float = 15.0):
    """The oracle (serial C, one thread) on a bounded sample of the workload:
    an L = 4096 lattice, q = 6, beta_c, random start, sweeps with records."""
    import oracle

    L, q, seed = 4096, 6, 1
    beta = math.log1p(math.sqrt(q))
    thr = oracle.threshold_table(beta)
    spins = oracle.init(L, q, seed, oracle.RANDOM)
    n = 0
    t0 = time.perf_counter()
    while True:
        oracle.sweeps(spins, q, seed, n, 1, thr, record=True)
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds_target or n >= 64:
            break
    return {"value": el * 1e9 / (n * L * L), "unit": "ns per spin flip", "cores": 1, "kind": "oracle", "host": host_cpu(),
            "sample": f"L={L} q={q} beta_c random start, {n} sweeps with per-sweep records, 1 thread"}


def run_large(args):
    import torch

    import paper_1101_0876_amd as potts

    L, q, seed = 32768, 6, 1
    beta = math.log1p(math.sqrt(q))
    N = L * L
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    stream = torch.cuda.Stream(device=dev)

    def make():
        # library-owned buffers (the colour-split copy is kept between calls) on
        # this stream, so that the events below time the kernels' own stream
        lats = [potts.Lattice.on_stream(L, q, seed, start, stream=stream)
                for start in (potts.ORDERED, potts.RANDOM)]
        for lat in lats:
            lat.tune(kernel=args.kernel)
            lat.tune_occupancy(args.occupancy)
        return lats

    # warm-up: the first --warmup sweeps of the same two chains, right before
    # the timed ones (the first call packs the colour-split copy; no idle gap
    # for allocation lets the clocks drop in between)
    lats = make()
    for lat in lats:
        lat.sweep(beta, max(0, args.warmup))
    stream.synchronize()

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for lat in lats:
        lat.sweep(beta, args.steps)
    ev1.record(stream)
    stream.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = ev0.elapsed_time(ev1)

    # sanity on the last records (cheap): populations sum to N
    for lat in lats:
        rec = lat.records(max(0, args.warmup) + args.steps - 1, 1)
        assert int(rec[0, 1:].sum()) == N, "population sum != N"
    for lat in lats:
        lat.close()

    site_updates = 2 * args.steps * N
    launches = 2 * 2 * args.steps  # two half-sweep launches per sweep per lattice
    per_launch_s = ev_ms * 1e-3 / launches
    per_launch_sites = N / 2
    achieved_ops = ALGO_OPS_PER_SITE * per_launch_sites / per_launch_s
    achieved_gbs = ALGO_BYTES_PER_SITE * per_launch_sites / per_launch_s / 1e9
    traffic = counter_traffic("large") if args.kernel in (0, 4) else None
    out = {
        "metric": "ns per spin flip",
        "value": wall * 1e9 / site_updates,
        "unit": "ns",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "single large lattice", "q": q, "L": L, "lattices": 2,
                   "starts": ["ordered", "random"], "beta": beta, "seed": seed,
                   "sweeps_per_lattice": args.steps, "warmup_sweeps_before": max(0, args.warmup),
                   "records": "every sweep"},
        # the metric's "% HBM roofline": algorithmic bytes (2 per site update)
        # per launch over the launch's duration, against the 8 TB/s peak
        "roofline": {
            "bound": "hbm",
            "achieved": achieved_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved_gbs / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": {0: "packed_kernel (colour-split half sweep)", 4: "packed_kernel (colour-split half sweep)",
                       1: "strip_kernel (row-major half sweep)", 2: "sweep4_kernel (chunk half sweep)"}[args.kernel],
            "avg_launch_us": per_launch_s * 1e6,
            "algorithmic_bytes_per_site_update": ALGO_BYTES_PER_SITE,
            "limiter": "valu issue (the Philox4x32-10 words are 17 of ~28 VALU ops per site update)",
        },
        # what binds: 32-bit VALU issue, against 256 CUs x 64 lanes x 2.4 GHz
        "alu_roofline": {
            "bound": "alu",
            "achieved": achieved_ops / 1e12,
            "peak": VALU_PEAK_OPS / 1e12,
            "unit": "Tops/s",
            "frac": achieved_ops / VALU_PEAK_OPS,
            "algorithmic_ops_per_site_update": ALGO_OPS_PER_SITE,
        },
        "event_ms": ev_ms,
        "site_updates_per_s": site_updates / wall,
        "paper_context": {"ns_per_spin_flip": 0.147, "hardware": "GTX 480 (its fastest card)"},
    }
    return out


def run_copy(args):
    """A plain device copy of 1 GiB (torch), the calibration for HBM counters
    and the practical bandwidth ceiling."""
    import torch

    n = 1 << 30
    a = torch.ones(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    torch.cuda.synchronize()
    reps = max(1, args.steps)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        b.copy_(a)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    return {"metric": "copy bandwidth", "value": 2 * n / (ms * 1e-3) / 1e9, "unit": "GB/s (read+write)",
            "bytes_read_per_launch": n, "bytes_written_per_launch": n, "ms_per_launch": ms, "reps": reps}


def run_batch(args):
    """Batched replicas: 1024 lattices of mixed L (128..4096), q (3..12) and beta
    near beta_c, 500 sweeps each, random starts; one batch (tile table, resident
    launches, hipGraph, in-run tuning) against the plain loop of one lattice at a
    time through the single-lattice path on the same GPU."""
    import torch

    import paper_1101_0876_amd as potts
    from paper_1101_0876_amd.workloads import batch_jobs

    import tempfile

    sweeps = args.steps if args.steps != 2000 else 500
    jobs = batch_jobs(n=args.batch_jobs, sweeps=sweeps)
    torch.cuda.set_device(0)
    site_updates = sum(j["L"] ** 2 * j["nsweeps"] for j in jobs)
    # warm-up: a small batch touches every kernel variant used below
    with potts.Batch(jobs[:16], graph=True, tune=False) as w:
        w.run()
    torch.cuda.synchronize()
    cache = args.tune_cache or os.path.join(tempfile.mkdtemp(), "tune.json")

    def one(tune, tune_cache):
        t0 = time.perf_counter()
        with potts.Batch(jobs, graph=True, tune=tune, tune_cache=tune_cache) as b:
            t_create = time.perf_counter()
            dev_ms = b.run()
            t_run = time.perf_counter()
            tuning = b.tuning()
            res = b.results()
        assert all(r["t"] == j["nsweeps"] for r, j in zip(res, jobs))
        return t_run - t_create, dev_ms, t_create - t0, tuning

    # untuned shapes, then the in-run tuner (writing the cache), then the cached shapes
    wall_plain_shape, _, _, _ = one(False, None)
    wall_tuning, _, _, _ = one(True, cache)
    wall, dev_ms, setup_s, tuning = one(False, cache)
    t0, t_create = 0.0, setup_s
    out = {
        "metric": "jobs/s", "value": len(jobs) / wall, "unit": "jobs/s", "n_gpus": 1,
        "steps": sweeps, "warmup": 0, "ms_per_step": wall * 1e3 / sweeps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "batched replicas", "jobs": len(jobs), "L": "2^U{7..12}", "q": "U{3..12}",
                   "beta": "beta_c(q) U[0.98,1.02]", "sweeps": sweeps, "list_seed": 1101,
                   "launch_shapes": "tuned (from the cache a tuning run wrote)"},
        "ns_per_spin_flip": wall * 1e9 / site_updates,
        "device_ms": dev_ms, "setup_s": t_create - t0, "tuning": tuning,
        "untuned_jobs_per_s": len(jobs) / wall_plain_shape,
        "tuning_run_jobs_per_s": len(jobs) / wall_tuning,
    }
    if not args.no_plain:
        # the plain loop: one lattice at a time, single-lattice path, same stream order
        tp = time.perf_counter()
        for j in jobs:
            with potts.Lattice(j["L"], j["q"], j["seed"], j["start"]) as lat:
                lat.sweep(j["beta"], j["nsweeps"])
                lat.observables()
        plain = time.perf_counter() - tp
        out["plain_loop"] = {"jobs_per_s": len(jobs) / plain, "wall_s": plain,
                             "speedup_of_batch": plain / wall}
    return out


def run_serve(args):
    """Serving: a burst of Poisson arrivals (200 jobs/s) of ramp jobs (L up to
    8192, q 3..15, 8..32 beta points), submitted at their arrival times while
    the server runs; reports completed jobs/s and p50/p99 latency (completion
    minus submission).  Sweep counts are scaled by --serve-scale (the full
    10^3..10^5 sweeps per job offer ~100x one GPU's throughput)."""
    import numpy as np
    import torch

    import paper_1101_0876_amd as potts
    from paper_1101_0876_amd.workloads import serve_jobs

    torch.cuda.set_device(0)
    jobs = serve_jobs(n=args.serve_jobs, rate=args.serve_rate, sweep_scale=args.serve_scale)
    site_updates = sum(j["L"] ** 2 * sum(j["sweeps"]) for j in jobs)
    import tempfile

    cache = args.tune_cache or os.path.join(tempfile.mkdtemp(), "serve_tune.json")
    # warm-up, outside the timed burst: loads every kernel variant once, and a
    # tuning server times the launch shapes of every lattice size of the
    # workload (one tiny job each) into the cache the timed server reads
    with potts.Server(quantum=args.serve_quantum, tune=True, tune_cache=cache) as warm:
        ts = [warm.submit(L, 6, 1, 1, [1.0, 1.2], [2, 2]) for L in (256, 512, 1024, 2048, 4096, 8192)]
        ts.append(warm.submit(256, 15, 1, 0, [1.0], [4]))
        warm.drain()
        for t in ts:
            warm.collect(t)
    with potts.Server(quantum=args.serve_quantum, max_slots=args.serve_slots, tune_cache=cache) as srv:
        start = time.perf_counter()
        tickets = []
        for j in jobs:
            delay = j["arrival"] - (time.perf_counter() - start)
            if delay > 0:
                time.sleep(delay)
            tickets.append(srv.submit(j["L"], j["q"], j["seed"], j["start"], j["betas"], j["sweeps"]))
        # drain in slices, with a progress line on stderr (long bursts at full sweep counts)
        while True:
            try:
                srv.drain(30000)
                break
            except potts.PottsError as exc:
                if exc.code != -4:  # anything but the slice's time-out
                    raise
                print(f"serve: {time.perf_counter() - start:.0f} s, {srv.iterations()} iterations",
                      file=sys.stderr, flush=True)
        got = [srv.collect(t) for t in tickets]
        iterations = srv.iterations()
        tuning = srv.tuning()
    lat = np.array([g["t_done"] - g["t_submit"] for g in got])
    span = max(g["t_done"] for g in got) - min(g["t_submit"] for g in got)
    assert all(g["status"] == 0 for g in got)
    return {
        "metric": "served jobs/s", "value": len(got) / span, "unit": "jobs/s", "n_gpus": 1,
        "steps": iterations, "warmup": 0, "ms_per_step": span * 1e3 / max(iterations, 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": "serving loop", "jobs": len(got), "arrival_rate_per_s": args.serve_rate,
                   "L": "2^U{8..13}", "q": "U{3..15}", "points": "U{8..32}",
                   "sweeps": f"round(10^U[3,5] x {args.serve_scale})", "quantum": args.serve_quantum,
                   "slots": args.serve_slots, "hbm_budget_GiB": 200, "list_seed": 1101},
        "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                      "max": float(lat.max())},
        "ns_per_spin_flip": span * 1e9 / site_updates,
        "span_s": span,
        "tuning": tuning,
    }


def run_extras(args):
    """The metric's batched and served parts, at their own workloads' default
    sizes whatever --steps says: the batched replicas (1024 jobs, 500 sweeps,
    tuned launch shapes) beside the plain one-lattice-at-a-time loop, and the
    serving burst (1000 Poisson arrivals at 200/s) with its sweep counts scaled
    by 0.01 (the stated 10^3..10^5 sweeps per job offer ~60x one GPU's
    throughput and take minutes: `--workload serve --serve-scale 1.0`).  Also
    the other two configurations in ns per spin flip: the plain method in full
    (L = 64, q = 9, 1000 sweeps, 20 runs) and the metastability ramps with 100
    sweeps per point (10^4 in the configuration: `--workload ramp
    --ramp-sweeps 10000`)."""
    import copy

    p_args = copy.copy(args)
    p_args.steps, p_args.no_cpu = 20, True
    pl = run_plain(p_args)
    r_args = copy.copy(args)
    r_args.ramp_sweeps = 100
    rp = run_ramp(r_args)
    b_args = copy.copy(args)
    b_args.steps, b_args.no_plain, b_args.tune_cache = 500, False, None
    b = run_batch(b_args)
    s_args = copy.copy(args)
    s_args.serve_jobs, s_args.serve_rate, s_args.serve_scale, s_args.tune_cache = 1000, 200.0, 0.01, None
    sv = run_serve(s_args)
    return {
        "batched": {"jobs_per_s": b["value"], "ns_per_spin_flip": b["ns_per_spin_flip"],
                    "plain_loop_jobs_per_s": b["plain_loop"]["jobs_per_s"],
                    "speedup_over_plain_loop": b["plain_loop"]["speedup_of_batch"],
                    "untuned_jobs_per_s": b["untuned_jobs_per_s"], "config": b["config"]},
        "served": {"jobs_per_s": sv["value"], "latency_s": sv["latency_s"],
                   "ns_per_spin_flip": sv["ns_per_spin_flip"], "span_s": sv["span_s"], "config": sv["config"],
                   "note": "sweep counts x0.01 of the stated 10^3..10^5 per job"},
        "plain": {"ns_per_spin_flip": pl["value"], "ms_per_run": pl["ms_per_step"], "runs": pl["steps"],
                  "config": pl["config"]},
        "ramp": {"ns_per_spin_flip": rp["value"], "wall_s": rp["wall_s"], "config": rp["config"],
                 "note": "100 sweeps per point of the stated 10^4"},
    }


def run_plain(args):
    """Plain method: q=9, L=64, random start, seed 1, beta = 1.02 ln 4, 1000
    sweeps with a record every sweep, repeated --steps times on fresh states
    (one LDS-resident launch per run)."""
    import torch

    import paper_1101_0876_amd as potts

    torch.cuda.set_device(0)
    L, q, seed, n = 64, 9, 1, 1000
    beta = 1.02 * math.log(4.0)
    reps = max(1, args.steps if args.steps != 2000 else 20)
    with potts.Lattice(L, q, seed, potts.RANDOM) as w:
        w.sweep(beta, n)
        w.observables()
    times = []
    for _ in range(reps):
        with potts.Lattice(L, q, seed, potts.RANDOM) as lat:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lat.sweep(beta, n)
            obs = lat.observables()  # synchronizes
            times.append(time.perf_counter() - t0)
    best = min(times)
    med = sorted(times)[len(times) // 2]
    cpu = None
    if not args.no_cpu:
        # the whole workload fits the oracle's budget: one full run, 1 thread
        import oracle

        spins = oracle.init(L, q, seed, oracle.RANDOM)
        t0 = time.perf_counter()
        oracle.sweeps(spins, q, seed, 0, n, oracle.threshold_table(beta), record=True)
        el = time.perf_counter() - t0
        cpu = {"value": el * 1e9 / (n * L * L), "unit": "ns per spin flip", "cores": 1, "kind": "oracle", "host": host_cpu(),
               "sample": f"the whole workload (L={L} q={q}, {n} sweeps with records), 1 thread"}
    return {"metric": "ns per spin flip", "value": med * 1e9 / (n * L * L), "unit": "ns", "n_gpus": 1,
            "steps": reps, "warmup": 1, "ms_per_step": med * 1e3, "higher_is_better": False,
            "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
            "config": {"workload": "plain method", "q": q, "L": L, "beta": beta, "seed": seed,
                       "sweeps": n, "records": "every sweep"},
            "best_ms": best * 1e3, "e_sat_last": obs["e_sat"], "cpu_baseline": cpu}


def run_ramp(args):
    """Metastability ramp: q in {6,9,12,15}, L=8192, 64 beta points within
    +-2% of beta_c(q), heating (ordered start, beta descending) and cooling
    (random start, beta ascending), --ramp-sweeps sweeps per point (the full
    workload has 10^4; stats over the second half of each point)."""
    import numpy as np
    import torch

    import paper_1101_0876_amd as potts
    from paper_1101_0876_amd.workloads import beta_c

    from concurrent.futures import ThreadPoolExecutor

    torch.cuda.set_device(0)
    L, per = 8192, args.ramp_sweeps
    half = per // 2
    k = np.arange(64)
    runs = []
    for q in (6, 9, 12, 15):
        grid = beta_c(q) * (0.98 + 0.04 * k / 63)
        for name, start, betas in (("heating", potts.ORDERED, grid[::-1]), ("cooling", potts.RANDOM, grid)):
            runs.append((q, name, start, betas))
    # the eight ramps are independent: each on its own state (own stream), one
    # host thread each, so that one ramp's kernel boundaries are filled by the
    # others' kernels
    lats = [potts.Lattice(L, q, 1, start) for q, _, start, _ in runs]
    for lat, (_, _, _, betas) in zip(lats, runs):
        # eight lattices share the GPU, so no launch needs to fill it alone:
        # 16-row items (fewer passive-row reloads and item set-ups than the
        # 4 a single L = 8192 lattice takes) measured 0.785 against 0.820 ps
        # per spin flip for the eight ramps; results do not depend on it
        if getattr(args, "kernel", 0) == 0:
            lat.tune(kernel=0, strip_rows=16)
        lat.sweep(float(betas[0]), 1)  # first launch outside the timing
        lat.observables()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    # eight segments of eight points per ramp (state carried over, the same
    # chain as one call), with a progress line after each: at the stated
    # 10^4 sweeps per point the whole run takes minutes
    results = [[] for _ in runs]
    with ThreadPoolExecutor(max_workers=len(runs)) as pool:
        for seg in range(8):
            parts = list(pool.map(lambda i: lats[i].ramp(runs[i][3][8 * seg: 8 * seg + 8], per - half, half),
                                  range(len(runs))))
            for i, pts in enumerate(parts):
                results[i].extend(pts)
            print(f"ramp: {8 * seg + 8} of 64 points, {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    t_all = time.perf_counter() - t0
    for lat in lats:
        lat.close()
    total = len(runs) * 64 * per
    curves = {}
    for (q, name, _, betas), pts in zip(runs, results):
        curves[f"q{q}_{name}"] = {"beta": [float(b) for b in betas[:: 21]],
                                  "e": [p["e"] for p in pts[:: 21]], "C": [p["C"] for p in pts[:: 21]]}
    return {"metric": "ns per spin flip", "value": t_all * 1e9 / (total * L * L), "unit": "ns", "n_gpus": 1,
            "steps": total, "warmup": 1, "ms_per_step": t_all * 1e3 / total, "higher_is_better": False,
            "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
            "config": {"workload": "metastability ramp", "q": [6, 9, 12, 15], "L": L, "points": 64,
                       "sweeps_per_point": per, "window": half, "directions": ["heating", "cooling"],
                       "concurrent_ramps": 8},
            "wall_s": t_all, "sample_points": curves}


def run_slabs(args):
    """The single large lattice (L=32768, q=6, beta_c, random start) split into
    8 row slabs of 4096 rows, the share of each of 8 devices, all swept on this
    one: halos refreshed by device copies before every half sweep, then one
    potts_slab_half_sweep per slab.  --steps sweeps (default 200)."""
    import torch

    import paper_1101_0876_amd as potts

    L, q, seed, G = 32768, 6, 1, 8
    beta = math.log1p(math.sqrt(q))
    torch.cuda.set_device(0)
    steps = args.steps if args.steps != 2000 else 200
    sl = potts.Slabs(L, q, seed, potts.RANDOM, nslabs=G, ring_slots=4)
    sl.sweep(beta, max(1, args.warmup))
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    sl.sweep(beta, steps)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = ev0.elapsed_time(ev1)
    rec = sl.records(sl.t - 1, 1)
    assert int(rec[0, 1:].sum()) == L * L, "population sum != N"
    site_updates = steps * L * L
    return {"metric": "ns per spin flip", "value": wall * 1e9 / site_updates, "unit": "ns", "n_gpus": 1,
            "steps": steps, "warmup": max(1, args.warmup), "ms_per_step": wall * 1e3 / steps,
            "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
            "config": {"workload": "row slabs of the single large lattice", "q": q, "L": L, "slabs": G,
                       "slab_rows": L // G, "beta": beta, "seed": seed, "start": "random"},
            "event_ms": ev_ms,
            "per_device_share_ms_per_sweep": ev_ms / steps / G,
            "launches_per_sweep": 2 * G, "halo_copies_per_sweep": 4 * G}


def run_metastability(args):
    """Binder's criterion (Sec. 6): both energy branches of q=9 at L=2048 (the
    paper's size), 20 samples each, 8 temperatures with |T - T_c|/T_c from
    10^-1.5 down to 10^-3.5, --meta-sweeps sweeps per point (the paper uses
    5*10^4..2*10^5 of equilibration and 5*10^4 of measurement); samples run
    concurrently through the serving loop.  Reports the rate and the fitted
    exponents."""
    import numpy as np
    import torch

    from paper_1101_0876_amd.metastability import analyse, branch, spinodal_std

    torch.cuda.set_device(0)
    q, L, samples = 9, 2048, 20
    taus = np.logspace(-1.5, -3.5, 8)
    per = args.meta_sweeps
    branch(q, 256, 2, taus[:2], 10, "high")  # warm-up outside the timing
    fits, total, wall = {}, 0, 0.0
    for side in ("high", "low"):
        t0 = time.perf_counter()
        b = branch(q, L, samples, taus, per, side)
        wall += time.perf_counter() - t0
        total += samples * len(taus) * per * L * L
        r = analyse(b)
        fits[side] = {"tau": [float(t) for t in b["tau"]], "e": [float(x) for x in b["e_mean"]],
                      "e_err": [float(x) for x in b["e_err"]],
                      "fit_all": r["fit_all"], "fit_near": r.get("fit_near"), "fit_far": r.get("fit_far")}
    return {"metric": "ns per spin flip", "value": wall * 1e9 / total, "unit": "ns", "n_gpus": 1,
            "steps": per, "warmup": 1, "ms_per_step": wall * 1e3 / (2 * len(taus) * per),
            "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
            "data": "synthetic",
            "config": {"workload": "metastability branches", "q": q, "L": L, "samples": samples,
                       "points": len(taus), "sweeps_per_point": per, "spinodal_tau_std": spinodal_std(q)},
            "wall_s": wall, "site_updates": total, "branches": fits}


def run_heatbath(args):
    """Heat-bath sweeps (Sec. 7): q=9, L=8192, random start, seed 1, beta =
    1.02 ln 4 (the plain-method temperature), --steps sweeps (default 200),
    with records every sweep; the oracle's heat-bath chain on an L=1024
    sample as the CPU baseline."""
    import torch

    import paper_1101_0876_amd as potts

    torch.cuda.set_device(0)
    L, q, seed = 8192, 9, 1
    beta = 1.02 * math.log(4.0)
    steps = args.steps if args.steps != 2000 else 200
    st = torch.cuda.Stream()
    with potts.Lattice.on_stream(L, q, seed, potts.RANDOM, stream=st) as lat:
        lat.tune(kernel=args.kernel)
        lat.sweep_heatbath(beta, max(1, args.warmup))
        st.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record(st)
        lat.sweep_heatbath(beta, steps)
        ev1.record(st)
        st.synchronize()
        wall = time.perf_counter() - t0
        rec = lat.records(lat.t - 1, 1)
        assert int(rec[0, 1:].sum()) == L * L, "population sum != N"
    cpu = None
    if not args.no_cpu:
        import oracle

        Ls = 1024
        spins = oracle.init(Ls, q, seed, oracle.RANDOM)
        thr = oracle.threshold_table(beta)
        n, t1 = 0, time.perf_counter()
        while True:
            oracle.heatbath_sweeps(spins, q, seed, n, 1, thr, record=True)
            n += 1
            el = time.perf_counter() - t1
            if el >= args.cpu_seconds or n >= 64:
                break
        cpu = {"value": el * 1e9 / (n * Ls * Ls), "unit": "ns per spin flip", "cores": 1, "kind": "oracle", "host": host_cpu(),
               "sample": f"L={Ls} q={q} heat-bath, random start, {n} sweeps with records, 1 thread"}
    ev_ms = ev0.elapsed_time(ev1)
    per_launch_s = ev_ms * 1e-3 / (2 * steps)
    achieved_ops = ALGO_OPS_PER_SITE * (L * L / 2) / per_launch_s
    return {"metric": "ns per spin flip", "value": wall * 1e9 / (steps * L * L), "unit": "ns", "n_gpus": 1,
            "steps": steps, "warmup": max(1, args.warmup), "ms_per_step": wall * 1e3 / steps,
            "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
            "config": {"workload": "heat-bath sweeps", "q": q, "L": L, "beta": beta, "seed": seed,
                       "start": "random", "records": "every sweep"},
            "roofline": {
                "bound": "alu",
                "achieved": achieved_ops / 1e12,
                "peak": VALU_PEAK_OPS / 1e12,
                "unit": "Tops/s",
                "frac": achieved_ops / VALU_PEAK_OPS,
                "traffic": None,
                "kernel": "heatbath4_kernel (chunk half sweep)" if args.kernel == 2
                          else "hb_packed_kernel (colour-split heat-bath half sweep)",
                "avg_launch_us": per_launch_s * 1e6,
                "algorithmic_ops_per_site_update": ALGO_OPS_PER_SITE,
            },
            "event_ms": ev_ms, "cpu_baseline": cpu}


def run_mid(args):
    """Mid-size single lattices, where a half sweep is too short to hide a
    kernel boundary: q=6, beta_c(6), random start, seed 1, records every
    sweep.  The value is L=4096 with the automatic kernel (the band kernel:
    64 sweeps per cooperative launch, --steps sweeps, default 640); beside it
    L = 1024 / 2048 / 4096 with the automatic kernel and with the streaming
    colour-split kernel (two launches per sweep; --no-extras skips these)."""
    import torch

    import paper_1101_0876_amd as potts

    torch.cuda.set_device(0)
    q, seed = 6, 1
    beta = math.log1p(math.sqrt(q))
    steps = args.steps if args.steps != 2000 else 640
    st = torch.cuda.Stream()

    def timed(L, kernel, n):
        with potts.Lattice.on_stream(L, q, seed, potts.RANDOM, stream=st) as lat:
            lat.tune(kernel=kernel)
            lat.sweep(beta, max(1, args.warmup))
            st.synchronize()
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            t0 = time.perf_counter()
            ev0.record(st)
            lat.sweep(beta, n)
            ev1.record(st)
            st.synchronize()
            wall = time.perf_counter() - t0
            rec = lat.records(lat.t - 1, 1)
            assert int(rec[0, 1:].sum()) == L * L, "population sum != N"
            return wall, ev0.elapsed_time(ev1)

    sizes = {}
    for L in (() if args.no_extras else (1024, 2048, 4096)):
        n = max(64, steps * (4096 // L) ** 2)
        _, ev_auto = timed(L, args.kernel, n)
        _, ev_split = timed(L, 4, n)
        sizes[str(L)] = {"auto_ps": ev_auto * 1e9 / (n * L * L), "colour_split_ps": ev_split * 1e9 / (n * L * L),
                         "sweeps": n}
        print(f"mid: L={L} automatic {sizes[str(L)]['auto_ps']:.3f} ps, colour-split "
              f"{sizes[str(L)]['colour_split_ps']:.3f} ps per spin flip", file=sys.stderr, flush=True)
    L = 4096
    wall, ev_ms = timed(L, args.kernel, steps)
    cpu = None if args.no_cpu else cpu_baseline(args.cpu_seconds)
    launches = -(-steps // 64)
    per_launch_s = ev_ms * 1e-3 / launches
    achieved_ops = ALGO_OPS_PER_SITE * L * L * (steps / launches) / per_launch_s
    return {"metric": "ns per spin flip", "value": wall * 1e9 / (steps * L * L), "unit": "ns", "n_gpus": 1,
            "steps": steps, "warmup": max(1, args.warmup), "ms_per_step": wall * 1e3 / steps,
            "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
            "config": {"workload": "mid-size single lattice", "q": q, "L": L, "beta": beta, "seed": seed,
                       "start": "random", "records": "every sweep", "kernel": args.kernel},
            "roofline": {
                "bound": "alu",
                "achieved": achieved_ops / 1e12,
                "peak": VALU_PEAK_OPS / 1e12,
                "unit": "Tops/s",
                "frac": achieved_ops / VALU_PEAK_OPS,
                "traffic": counter_traffic("mid") if args.kernel in (0, 7) and steps % 64 == 0 else None,
                "kernel": "band_kernel (64 sweeps per launch)" if args.kernel in (0, 7) else f"kernel {args.kernel}",
                "avg_launch_us": per_launch_s * 1e6,
                "algorithmic_ops_per_site_update": ALGO_OPS_PER_SITE,
            },
            "sizes": sizes, "event_ms": ev_ms, "cpu_baseline": cpu}


def run_cubic(args):
    """Simple-cubic lattice (Sec. 7's three-dimensional variant): q = 3,
    L = 1024 (2^30 uint8 spins, the default workload's site count), beta =
    0.5505, random start, seed 1, --steps sweeps (default 200) with records
    every sweep; the oracle's cubic chain on an L = 128 sample as the CPU
    baseline.  Roofline of the half-sweep kernel from HIP events on the
    state's own stream."""
    import torch

    import paper_1101_0876_amd as potts

    torch.cuda.set_device(0)
    L, q, seed, beta = 1024, 3, 1, 0.5505
    N = L ** 3
    steps = args.steps if args.steps != 2000 else 200
    warm = max(1, args.warmup)
    kernel = args.kernel if args.kernel in (0, 1, 2) else 0
    with potts.Cube(L, q, seed, potts.RANDOM) as c:
        c.tune(kernel)
        st = torch.cuda.ExternalStream(c.stream_handle())
        c.sweep(beta, warm)
        c.records(c.t - 1, 1)  # synchronizes
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record(st)
        c.sweep(beta, steps)
        ev1.record(st)
        rec = c.records(c.t - 1, 1)
        wall = time.perf_counter() - t0
        ev1.synchronize()
        ev_ms = ev0.elapsed_time(ev1)
        assert int(rec[0, 1:].sum()) == N, "population sum != N"
    cpu = None
    if not args.no_cpu:
        import oracle

        Ls = 128
        spins = oracle.init3d(Ls, q, seed, oracle.RANDOM)
        thr = oracle.threshold_table6(beta)
        n, t1 = 0, time.perf_counter()
        while True:
            oracle.sweeps3d(spins, q, seed, n, 1, thr, record=True)
            n += 1
            el = time.perf_counter() - t1
            if el >= args.cpu_seconds or n >= 64:
                break
        cpu = {"value": el * 1e9 / (n * Ls ** 3), "unit": "ns per spin flip", "cores": 1, "kind": "oracle", "host": host_cpu(),
               "sample": f"L={Ls}^3 q={q} cubic, random start, {n} sweeps with records, 1 thread"}
    ns = wall * 1e9 / (steps * N)
    packed = kernel in (0, 1)
    per_launch_s = ev_ms * 1e-3 / (2 * steps)
    achieved_ops = ALGO_OPS_PER_SITE * (N / 2) / per_launch_s
    return {"metric": "ns per spin flip", "value": ns, "unit": "ns", "n_gpus": 1, "steps": steps, "warmup": warm,
            "ms_per_step": wall * 1e3 / steps, "higher_is_better": False, "scaling": "weak",
            "vs_baseline": None, "dtype": "u8", "data": "synthetic",
            "config": {"workload": "simple-cubic sweeps", "q": q, "L": L, "beta": beta, "seed": seed,
                       "start": "random", "records": "every sweep",
                       "kernel": "colour-split" if packed else "chunk"},
            "roofline": {
                "bound": "alu",
                "achieved": achieved_ops / 1e12,
                "peak": VALU_PEAK_OPS / 1e12,
                "unit": "Tops/s",
                "frac": achieved_ops / VALU_PEAK_OPS,
                "traffic": counter_traffic("cubic") if packed else None,
                "kernel": "cube_packed_kernel (colour-split half sweep)" if packed
                          else "cube_sweep_kernel (chunk half sweep)",
                "avg_launch_us": per_launch_s * 1e6,
                "algorithmic_ops_per_site_update": ALGO_OPS_PER_SITE,
            },
            "hbm": {
                "achieved_gbs": ALGO_BYTES_PER_SITE * N / (2 * per_launch_s) / 1e9,
                "peak_gbs": HBM_PEAK_GBS,
                "frac": ALGO_BYTES_PER_SITE * N / (2 * per_launch_s) / 1e9 / HBM_PEAK_GBS,
                "algorithmic_bytes_per_site_update": ALGO_BYTES_PER_SITE,
            },
            "event_ms": ev_ms, "cpu_baseline": cpu}


def run_nnn(args):
    """First plus second neighbours (Sec. 7: nine colour passes per sweep):
    q = 9, L = 8184 (the temperature-ramp size 8192 rounded down to a
    multiple of 12), j2 = 0.5, beta = 0.8,
    random start, seed 1, --steps sweeps (default 100) with records every
    sweep; the oracle's chain on an L = 1200 sample as the CPU baseline.
    Roofline of the sweep (three row-class launches, which also count the
    record, and the fold of its partial sums) from HIP events on the state's
    stream."""
    import torch

    import paper_1101_0876_amd as potts

    torch.cuda.set_device(0)
    L, q, seed, beta, j2 = 8184, 9, 1, 0.8, 0.5  # the ramp size rounded to L % 12 == 0
    N = L * L
    steps = args.steps if args.steps != 2000 else 100
    warm = max(1, args.warmup)
    with potts.NnnLattice(L, q, seed, potts.RANDOM) as lat:
        st = torch.cuda.ExternalStream(lat.stream_handle())
        lat.sweep(beta, j2, warm)
        lat.records(lat.t - 1, 1)  # synchronizes
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record(st)
        lat.sweep(beta, j2, steps)
        ev1.record(st)
        rec = lat.records(lat.t - 1, 1)
        wall = time.perf_counter() - t0
        ev1.synchronize()
        ev_ms = ev0.elapsed_time(ev1)
        assert int(rec[0, 2:].sum()) == N, "population sum != N"
    cpu = None
    if not args.no_cpu:
        import oracle

        Ls = 1200
        spins = oracle.init(Ls, q, seed, oracle.RANDOM)
        thr = oracle.nnn_table(beta, j2)
        n, t1 = 0, time.perf_counter()
        while True:
            oracle.nnn_sweeps(spins, q, seed, n, 1, thr, record=True)
            n += 1
            el = time.perf_counter() - t1
            if el >= args.cpu_seconds or n >= 64:
                break
        cpu = {"value": el * 1e9 / (n * Ls * Ls), "unit": "ns per spin flip", "cores": 1, "kind": "oracle", "host": host_cpu(),
               "sample": f"L={Ls} q={q} j2={j2} nine-colour chain, random start, {n} sweeps with records, 1 thread"}
    ns = wall * 1e9 / (steps * N)
    sweep_s = ev_ms * 1e-3 / steps
    # Philox work the contract fixes: one 40-op block per 6-byte segment and
    # colour pass, 9 passes over L/3 rows x L/6 segments = N/2 blocks a sweep
    ops_per_site = 0.5 * 40.0
    achieved_ops = ops_per_site * N / sweep_s
    # bytes a sweep must move: each of the three row-class launches reads the
    # lattice once (its active rows and the rows above and below them, N) and
    # writes its active rows (N/3); the record is counted on the way
    sweep_bytes = 3 * (N + N / 3)
    return {"metric": "ns per spin flip", "value": ns, "unit": "ns", "n_gpus": 1, "steps": steps, "warmup": warm,
            "ms_per_step": wall * 1e3 / steps, "higher_is_better": False, "scaling": "weak",
            "vs_baseline": None, "dtype": "u8", "data": "synthetic",
            "config": {"workload": "first and second neighbours (nine colours)", "q": q, "L": L, "beta": beta,
                       "j2": j2, "seed": seed, "start": "random", "records": "every sweep"},
            "roofline": {
                "bound": "alu",
                "achieved": achieved_ops / 1e12,
                "peak": VALU_PEAK_OPS / 1e12,
                "unit": "Tops/s",
                "frac": achieved_ops / VALU_PEAK_OPS,
                "traffic": counter_traffic("nnn"),
                "kernel": "one sweep: three nnn_rows_kernel launches (record counted in them) + nnn_fold_kernel",
                "avg_sweep_us": sweep_s * 1e6,
                "algorithmic_ops_per_site_update": ops_per_site,
            },
            "hbm": {
                "achieved_gbs": sweep_bytes / sweep_s / 1e9,
                "peak_gbs": HBM_PEAK_GBS,
                "frac": sweep_bytes / sweep_s / 1e9 / HBM_PEAK_GBS,
                "algorithmic_bytes_per_sweep": sweep_bytes,
            },
            "event_ms": ev_ms, "cpu_baseline": cpu}


def run_e2e(args):
    """The paper's end-to-end run (Sec. 5): q = 9, L = 1024, 3 samples, T from
    0.71 to 0.73 in steps of 0.002 (11 points), at each point 2000
    equilibration and 8000 measurement sweeps, heating from the ordered start
    (Sec. 3), the state carried from point to point; the three samples run
    concurrently (one host thread and stream each).  Every measurement sweep
    is recorded (the paper samples every 50th).  Value: wall seconds of the
    whole run (all samples, all points, per-point statistics included); the
    paper's own run took 193 s on its GPU and 8115 s on its CPU.  The oracle
    times a bounded sample of the same protocol on one host core."""
    import paper_1101_0876_amd as potts

    L, q, samples = 1024, 9, 3
    temps = [0.71 + 0.002 * k for k in range(11)]
    betas = [1.0 / T for T in temps]
    t_tran, t_max = 2000, 8000
    # warm-up: one short ramp on a throwaway lattice (module load, first launches)
    with potts.Lattice(L, q, 99, potts.ORDERED) as lat:
        lat.ramp(betas[:2], 2, 2)
    # the samples are independent: one host thread and one state (own stream)
    # each, so their launches and kernels overlap
    from concurrent.futures import ThreadPoolExecutor

    lats = [potts.Lattice(L, q, s + 1, potts.ORDERED) for s in range(samples)]
    for lat in lats:
        lat.reserve_records(t_max + 2)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=samples) as pool:
        curves = list(pool.map(lambda lat: lat.ramp(betas, t_tran, t_max), lats))
    wall = time.perf_counter() - t0
    for lat in lats:
        lat.close()
    sweeps = samples * len(temps) * (t_tran + t_max)
    e_mean = [sum(c[k]["e"] for c in curves) / samples for k in range(len(temps))]
    m_mean = [sum(c[k]["m"] for c in curves) / samples for k in range(len(temps))]
    cpu = None
    if not args.no_cpu:
        import oracle

        # the same protocol on the oracle: first point, first sample, as many
        # sweeps as fit the time budget
        spins = oracle.init(L, q, 1, oracle.ORDERED)
        thr = oracle.threshold_table(betas[0])
        n, t1 = 0, time.perf_counter()
        while True:
            oracle.sweeps(spins, q, 1, n, 1, thr, record=True)
            n += 1
            el = time.perf_counter() - t1
            if el >= args.cpu_seconds or n >= 200:
                break
        per_sweep = el / n
        cpu = {"value": per_sweep * sweeps, "unit": "s (extrapolated whole run)", "cores": 1, "kind": "oracle", "host": host_cpu(),
               "sample": f"L={L} q={q} T={temps[0]} ordered start, {n} sweeps with records timed, "
                         f"x {sweeps} sweeps of the run, 1 thread"}
    return {"metric": "end-to-end run time", "value": wall, "unit": "s", "n_gpus": 1, "steps": sweeps, "warmup": 1,
            "ms_per_step": wall * 1e3 / sweeps, "higher_is_better": False, "scaling": "strong",
            "vs_baseline": None, "dtype": "u8", "data": "synthetic",
            "config": {"workload": "end-to-end heating ramp", "q": q, "L": L, "samples": samples,
                       "T": [round(T, 3) for T in temps], "t_tran": t_tran, "t_max": t_max,
                       "start": "ordered", "records": "every sweep"},
            "ns_per_spin_flip": wall * 1e9 / (sweeps * L * L),
            "curve": {"T": [round(T, 3) for T in temps], "e": e_mean, "m": m_mean},
            "paper_context": {"gpu_s": 193, "cpu_s": 8115, "hardware": "GTX 280 / Core 2 Duo E8400"},
            "cpu_baseline": cpu}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="large", choices=["large", "copy", "batch", "serve", "plain", "ramp", "slabs", "mid",
                                                     "metastability", "heatbath", "cubic", "nnn", "e2e"])
    ap.add_argument("--kernel", type=int, default=0,
                    help="large: 0 automatic (colour-split), 1 strip, 2 chunk, 4 colour-split; "
                         "cubic: 0 automatic (colour-split), 1 colour-split, 2 chunk")
    ap.add_argument("--ramp-sweeps", type=int, default=100)
    ap.add_argument("--meta-sweeps", type=int, default=1000)
    ap.add_argument("--batch-jobs", type=int, default=1024)
    ap.add_argument("--no-plain", action="store_true", help="batch: skip the one-lattice-at-a-time loop")
    ap.add_argument("--serve-jobs", type=int, default=1000)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-scale", type=float, default=0.01)
    ap.add_argument("--serve-quantum", type=int, default=32)
    ap.add_argument("--serve-slots", type=int, default=256)
    ap.add_argument("--occupancy", type=int, default=0, choices=[0, 8],
                    help="large: colour-split kernel waves per SIMD (0: the compiler's choice)")
    ap.add_argument("--tune-cache", default=None, help="batch/serve: launch-shape cache file (default: a fresh one)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-extras", action="store_true",
                    help="default workload: skip the batched, served, plain-method and ramp summaries")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "this build has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.workload == "copy":
        print(json.dumps(run_copy(args)), flush=True)
        return
    if args.workload == "plain":
        print(json.dumps(run_plain(args)), flush=True)
        return
    if args.workload == "ramp":
        print(json.dumps(run_ramp(args)), flush=True)
        return
    if args.workload == "mid":
        print(json.dumps(run_mid(args)), flush=True)
        return
    if args.workload == "heatbath":
        print(json.dumps(run_heatbath(args)), flush=True)
        return
    if args.workload == "cubic":
        print(json.dumps(run_cubic(args)), flush=True)
        return
    if args.workload == "nnn":
        print(json.dumps(run_nnn(args)), flush=True)
        return
    if args.workload == "e2e":
        print(json.dumps(run_e2e(args)), flush=True)
        return
    if args.workload == "metastability":
        print(json.dumps(run_metastability(args)), flush=True)
        return
    if args.workload == "slabs":
        print(json.dumps(run_slabs(args)), flush=True)
        return
    if args.workload == "serve":
        print(json.dumps(run_serve(args)), flush=True)
        return
    if args.workload == "batch":
        if args.steps == 2000:  # the batch workload's own default
            args.steps = 500
        print(json.dumps(run_batch(args)), flush=True)
        return
    out = run_large(args)
    out["cpu_baseline"] = None if args.no_cpu else cpu_baseline(args.cpu_seconds)
    if not args.no_extras:
        out.update(run_extras(args))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
