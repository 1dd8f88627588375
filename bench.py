"""Benchmark: useful simplex elements/s of one step of the hot path, H vs BB.

Default workload (the largest configuration that fits one GPU): m = 3,
n = 1024, one step of the 3-D automaton B6/S567 on uint8 cells,
Bernoulli(0.2), (n+1)^3 box (1.08 GB per buffer), ping-pong between two
device-resident buffers.  A step is one launch of the whole path (plan
lookup, H decode, tile walk, op).  The other workloads (c1 m = 2 n = 1024
ACCUM, c2 m = 2 n = 16384 Life, c4 m = 4 n = 128 HASH, c5 serving) are
selected with --workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c3]
                    [--no-cpu] [--no-bb]

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E, published

# algorithmic HBM bytes per useful element (read + write)
BYTES_PER_ELEMENT = {"accum": 8, "ca2": 2, "ca3": 2, "hash": 4, "hits": 8, "map": 0, "edm": 4}

# kernel sources whose change invalidates stored counter readings, per op
KERNEL_SOURCES = {
    "ca2": ["smap_decode.hpp", "smap_ca2.hpp"],
    "ca3": ["smap_decode.hpp", "smap_ca2.hpp", "smap_ca3.hpp"],
    "point": ["smap_decode.hpp", "smap_point.hpp"],
    "copy": ["smap_copy.hpp"],
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sha(op: str) -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(op, KERNEL_SOURCES["point"]):
        with open(os.path.join(ROOT, "paper_2208_11617_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(workload: str, op: str, info: dict):
    """HBM bytes per launch of the H kernel from the committed rocprofv3
    counter summary, or None when there is none, the kernel's sources
    changed since the counters were taken, or the launch differs from the
    one measured (tile side, and launched workgroups where recorded)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_sha") != kernel_sha(op):
        return None
    if info is not None:
        if rec.get("rho") != info["rho"]:
            return None
        if "launched_wgs" in rec and rec["launched_wgs"] != info["launched_wgs"]:
            return None
    return rec.get("hbm_bytes_per_launch")


def _batch_stats(per):
    """Median, mean and standard error of the mean of per-batch means."""
    nb = len(per)
    per = sorted(per)
    mean = sum(per) / nb
    sem = (sum((x - mean) ** 2 for x in per) / (nb - 1) / nb) ** 0.5 if nb > 1 else None
    mid = per[nb // 2] if nb % 2 else 0.5 * (per[nb // 2 - 1] + per[nb // 2])
    return {"batches": nb, "median_ms": mid, "mean_ms": mean, "sem_ms": sem,
            "sem_rel": None if sem is None else sem / mean}


def time_launches(fn, steps, warmup, stream, stats=None, batches=10, sem_target=0.01, extra_s=10.0):
    """Mean ms per launch over exactly `steps` back-to-back launches (HIP
    events on `stream`); that figure is the one returned.

    With a dict `stats`, the timed region is cut into `batches` equal
    batches, and the median, mean and standard error of the per-batch
    means (ms per launch) go into `stats`.  If the standard error is then
    not below `sem_target` of the mean (the measurement protocol: repeat
    until it is), further batches of the same size are timed after the
    region, for at most `extra_s` seconds, and the statistics cover all of
    them (`converged` says whether the target was reached)."""
    import torch
    for i in range(warmup):
        fn(i)
    torch.cuda.synchronize()
    nb = max(1, min(batches, steps)) if stats is not None else 1
    cuts = [round(k * steps / nb) for k in range(nb + 1)]
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(nb + 1)]
    evs[0].record(stream)
    for b in range(nb):
        for i in range(cuts[b], cuts[b + 1]):
            fn(warmup + i)
        evs[b + 1].record(stream)
    torch.cuda.synchronize()
    ms = evs[0].elapsed_time(evs[-1]) / steps      # ms per launch over the K timed steps
    if stats is not None:
        per = [evs[b].elapsed_time(evs[b + 1]) / (cuts[b + 1] - cuts[b]) for b in range(nb)]
        st = _batch_stats(per)
        size = max(1, steps // nb)
        t0 = time.perf_counter()
        i = warmup + steps
        while (st["sem_rel"] is None or st["sem_rel"] >= sem_target) and time.perf_counter() - t0 < extra_s:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(size):
                fn(i)
                i += 1
            e1.record(stream)
            torch.cuda.synchronize()
            per.append(e0.elapsed_time(e1) / size)
            st = _batch_stats(per)
        st["timed_steps_ms"] = ms
        st["converged"] = st["sem_rel"] is not None and st["sem_rel"] < sem_target
        stats.update(st)
    return ms


def tile_sweep(m, op, fn_for, steps, warmup, stream):
    """H and BB at every compiled (rho, workgroup size, tiles per workgroup)
    of the op class, each pair with the same shape (same-shape); returns the
    list of timings."""
    from paper_2208_11617_amd import binding as smap
    rows = []
    smap.autotune_reset()   # H launches follow set_shape only without a tuned choice
    try:
        for rho in (4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096):
            for wg in (64, 128, 256, 512):
                for grp in (1, 2, 4, 8, 16):
                    try:
                        smap.set_shape(m, op, rho, wg, grp)
                    except smap.SimplexMapError:
                        continue   # not compiled for this class
                    row = {"rho": rho, "wg_threads": wg, "tiles_per_wg": grp}
                    for name, launch in (("h", smap.map_launch), ("bb", smap.bb_launch)):
                        try:
                            row[f"{name}_ms"] = time_launches(fn_for(launch), steps, warmup, stream)
                        except smap.SimplexMapError:
                            row[f"{name}_ms"] = None   # beyond the grid limits
                    rows.append(row)
    finally:
        smap.set_tile(m, op, 0)
    return rows


def best_vs_best(rows):
    """The fastest H and the fastest BB of a tile sweep, each tuned on its own."""
    h = min((r for r in rows if r["h_ms"] is not None), key=lambda r: r["h_ms"])
    b = min((r for r in rows if r["bb_ms"] is not None), key=lambda r: r["bb_ms"])
    return {"h": {"rho": h["rho"], "wg_threads": h["wg_threads"], "tiles_per_wg": h["tiles_per_wg"],
                  "ms_per_step": h["h_ms"]},
            "bb": {"rho": b["rho"], "wg_threads": b["wg_threads"], "tiles_per_wg": b["tiles_per_wg"],
                   "ms_per_step": b["bb_ms"]},
            "h_vs_bb_speedup": b["bb_ms"] / h["h_ms"], "same_shape": rows}


def read_power_w():
    """Socket power of GPU 0 in watts, from amd-smi (a child process), or None."""
    import subprocess
    try:
        r = subprocess.run(["amd-smi", "metric", "--power", "--json"], capture_output=True,
                           text=True, timeout=10)
        d = json.loads(r.stdout)
        return float(d["gpu_data"][0]["power"]["socket_power"]["value"])
    except Exception:
        return None


def power_leg(fn, seconds, stream):
    """Run fn(i) back to back for about `seconds` while sampling socket power
    every ~0.25 s in a thread; returns (launches per second, mean watts,
    samples)."""
    import threading

    import torch
    samples, stop = [], threading.Event()

    def sampler():
        while not stop.is_set():
            w = read_power_w()
            if w is not None:
                samples.append(w)
            stop.wait(0.25)
    for i in range(5):
        fn(i)
    torch.cuda.synchronize()
    th = threading.Thread(target=sampler, daemon=True)
    t0 = time.perf_counter()
    th.start()
    count = 0
    while time.perf_counter() - t0 < seconds:
        for _ in range(50):
            fn(count)
            count += 1
        torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stop.set()
    th.join()
    steady = samples[1:] if len(samples) > 2 else samples     # drop the ramp-up sample
    return count / dt, (sum(steady) / len(steady)) if steady else None, len(samples)


def copy_probe(nbytes, steps, stream):
    """A plain streaming kernel over ``nbytes`` (torch's elementwise
    bitwise_not on uint8: one read and one write per byte, like a copy, but
    always a kernel rather than a DMA transfer): the achievable read+write
    rate on this GPU, and the known-size kernel that calibrates the HBM byte
    counters."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    ms = time_launches(lambda i: torch.bitwise_not(src, out=dst), steps, 3, stream)
    del src, dst
    return {"bytes_read": nbytes, "bytes_written": nbytes, "ms": ms,
            "gbs": 2 * nbytes / (ms * 1e-3) / 1e9}


def simplex_copy_probe(smap, m, n, src, dst, steps, stream):
    """The copy of just the simplex cells (simplex_copy_launch): one read and
    one write per simplex cell, row by row, no tiles and no halo -- the
    floor the (n+1)^m layout puts on one pass over the simplex.  Its HBM
    counters, when stored for this workload, come with it."""
    useful = smap.count(m, n)
    stats = {}
    ms = time_launches(lambda i: smap.copy_launch(m, n, src, dst, stream=stream), steps, 3, stream, stats)
    return {"ms": ms, "bytes_algorithmic": 2 * useful, "gbs": 2 * useful / (ms * 1e-3) / 1e9,
            "frac_of_peak": 2 * useful / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, "timing": stats}


def set_layout3(smap, name):
    smap.set_layout(3, {"auto": smap.LAYOUT_AUTO, "packed": smap.LAYOUT_PACKED,
                        "levels": smap.LAYOUT_LEVELS}[name])


def bench_serve(args):
    """The serving workload: a stream of one-step automaton jobs (60 % m = 2
    with n log-uniform in [64, 4096], 40 % m = 3 with n log-uniform in
    [32, 512]), inputs resident in HBM, outputs in an arena of --budget-gib.
    Saturated throughput (every job at t = 0) of sequential plain-H launches
    and of continuous batching (batched launches, and persistent work-queue
    launches), then all three at a Poisson load of --load times
    the sequential saturated rate, with p50/p99 latency (arrival to the end
    of the job's launch, device events)."""
    import math

    import numpy as np
    import torch

    import simplex_inputs as si
    from paper_2208_11617_amd import binding as smap

    set_layout3(smap, args.layout3)
    torch.cuda.set_device(0)
    jobs0 = si.serve_trace(args.jobs, None)
    shapes = sorted(set((m, n) for m, n, _ in jobs0))
    log(f"serving: {args.jobs} jobs, {len(shapes)} distinct sizes; generating inputs")
    inputs = {(m, n): si.box_torch(m, n, "bern", si.serve_seed(m, n), p=si.SERVE["p"], device="cuda")
              for m, n in shapes}
    arena = torch.empty(int(args.budget_gib * (1 << 30)), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    cells = {mn: math.comb(mn[1] + mn[0], mn[0]) for mn in shapes}
    op = {2: "ca2", 3: "ca3"}

    def replay(trace, mode):
        recs = smap.serve_run([(m, op[m], n, inputs[(m, n)], t) for m, n, t in trace], arena, mode,
                              max_inflight=args.max_inflight)
        lat = np.array([r["done_s"] - t for r, (_, _, t) in zip(recs, trace)])
        span = max(r["done_s"] for r in recs) - min(t for _, _, t in trace)
        useful = sum(cells[(m, n)] for m, n, _ in trace)
        return {"jobs_per_s": len(trace) / span, "elements_per_s": useful / span,
                "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
                "mean_ms": float(lat.mean() * 1e3), "launches": int(max(r["batch"] for r in recs)) + 1,
                "makespan_s": span}

    modes = (("sequential", smap.SERVE_SEQUENTIAL), ("batched", smap.SERVE_BATCHED),
             ("persistent", smap.SERVE_PERSISTENT))
    res = {}
    for name, mode in modes:
        for _ in range(args.warmup_replays):
            replay(jobs0, mode)
        log(f"saturated replay: {name}")
        res[f"saturated_{name}"] = replay(jobs0, mode)
    rate = args.load * res["saturated_sequential"]["jobs_per_s"]
    trace = si.serve_trace(args.jobs, rate)
    for name, mode in modes:
        log(f"Poisson replay at {rate:.0f} jobs/s: {name}")
        res[f"load_{name}"] = replay(trace, mode)
    sat_b = res["saturated_batched"]
    out = {
        "metric": "useful simplex elements/s (serving, continuous batching, saturated)",
        "value": sat_b["elements_per_s"],
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": args.warmup_replays,
        "ms_per_step": sat_b["makespan_s"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic (seeded splitmix64 cells, seeded Poisson arrivals)",
        "config": {"workload": f"c5: serving, {args.jobs} one-step automaton jobs, "
                               f"{len(shapes)} sizes, budget {args.budget_gib} GiB",
                   "jobs": args.jobs, "budget_gib": args.budget_gib, "load": args.load,
                   "offered_rate_jobs_per_s": rate, "max_inflight": args.max_inflight,
                   "layout3": args.layout3},
        "serving": res,
        "batched_vs_sequential_saturated": sat_b["jobs_per_s"] / res["saturated_sequential"]["jobs_per_s"],
        "persistent_vs_sequential_saturated":
            res["saturated_persistent"]["jobs_per_s"] / res["saturated_sequential"]["jobs_per_s"],
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def cpu_baseline(w, budget_s=12.0):
    """The oracle, single-threaded, on a bounded sample of the same workload:
    whole slabs of the outermost coordinate x_m, starting at x_m = 0, until
    about ``budget_s`` seconds of work (or the whole workload) are done."""
    import numpy as np

    import simplex_inputs as si
    from oracle import oracle

    m, n, op = w["m"], w["n"], w["op"]
    dt = np.uint8 if op.startswith("ca") else np.uint32
    inp = None
    if w["dist"] is not None:
        inp = np.zeros((n + 1,) * m, dtype=dt)   # lazily mapped; slabs filled below
    out = np.zeros((n + 1,) * m, dtype=dt)
    slab_cells = (n + 1) ** (m - 1)
    done_cells, elapsed, lo = 0, 0.0, 0
    step = max(1, (n + 1) // 64)
    # the oracle runs on one core: pin the process to one allowed CPU meanwhile
    allowed = os.sched_getaffinity(0)
    pinned = min(allowed)
    os.sched_setaffinity(0, {pinned})
    try:
        while lo <= n and elapsed < budget_s:
            hi = min(lo + step, n + 1)
            if inp is not None:  # this slab and the next one (read by the automaton)
                for z in range(lo, min(hi + 1, n + 1)):
                    flat = si.values_at(w["seed"], w["dist"], w["p"],
                                        np.arange(z * slab_cells, (z + 1) * slab_cells))
                    inp[z] = flat.reshape((n + 1,) * (m - 1))
            t0 = time.perf_counter()
            done_cells += oracle.apply_slab(m, n, op, inp, out, lo, hi)
            elapsed += time.perf_counter() - t0
            lo = hi
    finally:
        os.sched_setaffinity(0, allowed)
    return {
        "value": done_cells / elapsed if elapsed > 0 else None,
        "unit": "useful elements/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{done_cells} of {oracle.count(m, n)} elements (slabs x_{m} < {lo}), "
                  f"{elapsed:.1f} s single-threaded",
        "host_cpu": host_cpu(),
        "pinned_cpu": pinned,
    }


def host_cpu():
    """The host's CPU model and the logical CPUs this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus_available": len(os.sched_getaffinity(0))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c3", choices=["c1", "c2", "c3", "c4", "c5"])
    ap.add_argument("--jobs", type=int, default=10000, help="c5: jobs in the stream")
    ap.add_argument("--budget-gib", type=float, default=8.0, help="c5: output arena")
    ap.add_argument("--load", type=float, default=0.8, help="c5: offered load / sequential rate")
    ap.add_argument("--max-inflight", type=int, default=4, help="c5: batches in flight")
    ap.add_argument("--warmup-replays", type=int, default=1, help="c5: untimed replays")
    ap.add_argument("--no-cpu", action="store_true", help="skip the cpu_baseline leg")
    ap.add_argument("--no-bb", action="store_true", help="skip timing the BB baseline")
    ap.add_argument("--no-copy", action="store_true", help="skip the plain-copy and simplex-copy probes")
    ap.add_argument("--beta", type=int, default=0)
    ap.add_argument("--power", type=float, default=0.0,
                    help="also run H and BB for this many seconds each while sampling socket power (amd-smi)")
    ap.add_argument("--autotune", action="store_true",
                    help="pick rho / workgroup size / beta for the H launch by timing first")
    ap.add_argument("--tune-cache", default=None, help="autotune result file (read and appended)")
    ap.add_argument("--graph", type=int, default=0,
                    help="time H as replays of a captured graph of this many launches")
    ap.add_argument("--general", default="fused", choices=["fused", "streams"],
                    help="H launches: all pieces in one launch, or one launch per piece on streams of their own")
    ap.add_argument("--layout3", default="auto", choices=["auto", "packed", "levels"],
                    help="native layout of the 3-D H map")
    ap.add_argument("--shape", default=None,
                    help="rho,threads,tiles_per_wg for H and BB (simplex_set_shape); default: the library's")
    ap.add_argument("--gens", type=int, default=0,
                    help="automata: time simplex_map_launch_steps advancing this many generations per call")
    ap.add_argument("--best-vs-best", action="store_true",
                    help="also time H and BB at every compiled tile: same-shape pairs and best vs best")
    ap.add_argument("--op", default=None, choices=["map", "accum", "hash", "hits", "edm"],
                    help="run this per-element op on the workload's m and n instead of its own")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    if args.workload == "c5":
        bench_serve(args)
        return

    import torch

    import simplex_inputs as si
    from paper_2208_11617_amd import binding as smap

    w = dict(si.WORKLOADS[args.workload])
    if args.op is not None and args.op != w["op"]:
        # the same domain with another per-element op (MAP shows the map alone)
        w.update(op=args.op, dist="u31" if args.op == "accum" else None, p=None)
    if w["op"] == "edm":
        w["dist"] = None          # the input is a point set, generated below
    m, n, op = w["m"], w["n"], w["op"]
    u8 = op.startswith("ca")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    useful = smap.count(m, n)
    if m == 3:
        set_layout3(smap, args.layout3)
    if args.shape:
        rho, wg, grp = (int(v) for v in args.shape.split(","))
        smap.set_shape(m, op, rho, wg, grp)
    smap.set_general(smap.GENERAL_STREAMS if args.general == "streams" else smap.GENERAL_FUSED)

    log(f"generating {args.workload}: m={m} n={n} op={op}")
    bufs = []
    if op == "edm":
        if m != 2:
            raise SystemExit("--op edm needs a 2-D workload (c1 or c2)")
        bufs.append(torch.from_numpy(si.points(n, w["seed"])).to(dev))   # n+1 points in R^3
    elif w["dist"] is not None:
        bufs.append(si.box_torch(m, n, w["dist"], w["seed"], p=w["p"], device=dev))
    out_a = si.sentinel_box_torch(m, n, u8, device=dev)
    torch.cuda.synchronize()

    def step_fn(launch):
        def fn(i):
            if u8:   # ping-pong: in -> a, a -> in, ...
                src, dst = (bufs[0], out_a) if i % 2 == 0 else (out_a, bufs[0])
                launch(m, n, op, src, dst, stream=stream)
            elif op in ("accum", "edm"):
                launch(m, n, op, bufs[0], out_a, stream=stream)
            elif op == "map":
                launch(m, n, op, None, None, stream=stream)
            else:
                launch(m, n, op, None, out_a, stream=stream)
        return fn

    tuned = None
    if args.autotune:
        log("autotuning the H launch")
        src = bufs[0] if bufs else None
        tuned = smap.autotune(m, n, op, src, out_a if op != "map" else None, reps=20,
                              cache_path=args.tune_cache, stream=stream)
        log(f"tuned: {tuned}")
    h_launch = lambda *a, **k: smap.map_launch(*a, beta=args.beta, **k)  # noqa: E731
    gens = 1
    if args.gens > 0:
        if op not in ("ca2", "ca3"):
            raise SystemExit("--gens applies to the automata (workloads c2 and c3)")
        gens = args.gens
        h_launch = lambda m_, n_, op_, s_, d_, stream=None: smap.map_launch_steps(  # noqa: E731
            m_, n_, op_, gens, s_, d_, beta=args.beta, stream=stream)
    h_stats, bb_stats = {}, {}
    if args.graph > 0:
        # one replay = args.graph launches (automata: ping-pong, pointwise: repeated)
        K = args.graph if not u8 else args.graph + (args.graph % 2)
        src = bufs[0] if bufs else None
        dst = None if op == "map" else out_a
        reps = max(1, args.steps // K)

        def graph_ms(use_bb):
            g = smap.Graph(m, n, op, src, dst, steps=K, beta=args.beta, use_bb=use_bb)
            ms = time_launches(lambda i: g.launch(stream), reps, max(1, args.warmup // K), stream) / K
            g.close()
            return ms
        log(f"timing H as graph replays: {reps} x {K} launches")
        h_ms = graph_ms(False)
    else:
        log(f"timing H: {args.warmup} warmup + {args.steps} steps")
        h_ms = time_launches(step_fn(h_launch), args.steps, args.warmup, stream, stats=h_stats)
    bb_ms = None
    if not args.no_bb:
        log("timing BB" + (" as graph replays" if args.graph > 0 else ""))
        if args.graph > 0:
            bb_ms = graph_ms(True)
        elif args.gens > 0:
            bb_steps = lambda m_, n_, op_, s_, d_, stream=None: smap.bb_launch_steps(  # noqa: E731
                m_, n_, op_, gens, s_, d_, stream=stream)
            bb_ms = time_launches(step_fn(bb_steps), args.steps, args.warmup, stream)
        else:
            bb_ms = time_launches(step_fn(smap.bb_launch), args.steps, args.warmup, stream, stats=bb_stats)
    sweep = None
    if args.best_vs_best and args.gens == 0 and args.graph == 0:
        log("H and BB at every compiled tile")
        sweep = tile_sweep(m, op, step_fn, max(10, args.steps // 4), max(2, args.warmup // 4), stream)

    power = None
    if args.power > 0:
        log(f"power legs: {args.power} s each")
        idle = read_power_w()
        h_rate, h_w, h_n = power_leg(step_fn(h_launch), args.power, stream)
        power = {"idle_w": idle, "h": {"launches_per_s": h_rate, "watts": h_w, "samples": h_n,
                                       "elements_per_joule": None if not h_w else useful * gens * h_rate / h_w}}
        if not args.no_bb and args.graph == 0:
            bb_fn = smap.bb_launch
            if args.gens > 0:
                bb_fn = lambda m_, n_, op_, s_, d_, stream=None: smap.bb_launch_steps(  # noqa: E731
                    m_, n_, op_, gens, s_, d_, stream=stream)
            b_rate, b_w, b_n = power_leg(step_fn(bb_fn), args.power, stream)
            power["bb"] = {"launches_per_s": b_rate, "watts": b_w, "samples": b_n,
                           "elements_per_joule": None if not b_w else useful * gens * b_rate / b_w}

    copy = None
    scopy = None
    if not args.no_copy:
        log("timing a plain copy of the same byte count")
        copy = copy_probe(max(useful * BYTES_PER_ELEMENT[op] // 2, 1 << 20), 20, stream)
        if u8 and m in (2, 3):
            log("timing the copy of just the simplex cells")
            scopy = simplex_copy_probe(smap, m, n, bufs[0], out_a, max(20, args.steps // 4), stream)
            scopy["traffic"] = stored_traffic(f"copy_{args.workload}", "copy", None)

    info_h = smap.plan_info(m, n, op, beta=tuned["beta"] if tuned else args.beta)
    info_bb = smap.plan_info(m, n, op, use_bb=True)
    alg_bytes = useful * BYTES_PER_ELEMENT[op]        # per pass over HBM
    achieved = alg_bytes / (h_ms * 1e-3) / 1e9
    traffic = stored_traffic(args.workload, op, info_h) if args.gens == 0 else None
    value = useful * gens / (h_ms * 1e-3)             # useful cell updates per second

    res = {
        "metric": "useful simplex elements/s (H map)",
        "value": value,
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8" if u8 else "u32",
        "data": "synthetic (seeded splitmix64)",
        "config": {"workload": f"{args.workload}: m={m} n={n} op={op}", "m": m, "n": n,
                   "op": op, "useful_elements": useful,
                   "rho": info_h["rho"] if args.gens == 0 else (256 if m == 2 else 64),
                   "beta": info_h["beta"], "autotuned": tuned, "graph_launches": args.graph or None,
                   "generations_per_call": gens, "layout3": args.layout3 if m == 3 else None,
                   "general": args.general,
                   "wg_threads": None if args.gens else info_h["wg_threads"],
                   "tiles_per_wg": None if args.gens else info_h["tiles_per_wg"]},
        "hbm_gbs_algorithmic": achieved,
        "bb": None if bb_ms is None else {
            "ms_per_step": bb_ms, "value": useful * gens / (bb_ms * 1e-3),
            "hbm_gbs_algorithmic": alg_bytes / (bb_ms * 1e-3) / 1e9},
        "h_vs_bb_speedup": None if bb_ms is None else bb_ms / h_ms,
        "timing": {"h": h_stats or None, "bb": bb_stats or None},
        "best_vs_best": None if not sweep else best_vs_best(sweep),
        # (plan info describes the one-step launch; the multi-generation
        # kernels have tiles of their own)
        "tiles": None if args.gens else {
            "useful": info_h["useful_tiles"], "h_launched": info_h["launched_tiles"],
            "bb_launched": info_bb["launched_tiles"], "wgs_per_tile": info_h["wgs_per_tile"],
            "h_workgroups": info_h["launched_wgs"], "bb_workgroups": info_bb["launched_wgs"]},
        "roofline": {
            "bound": "hbm" if op != "map" else "alu",
            "achieved": achieved,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS,
            "traffic": traffic,
            "kernel": f"{op} H launch" + (f" ({gens} generations per call, "
                                          + ("rho 256, halo 32)" if m == 2 else "rho 64, halo 16)")
                                          if args.gens else ""),
            "kernel_sha": kernel_sha(op),
            "bytes_per_launch": alg_bytes,
            "copy_gbs": None if copy is None else copy["gbs"],
            "frac_of_copy": None if copy is None else achieved / copy["gbs"],
            "simplex_copy_gbs": None if scopy is None else scopy["gbs"],
            "frac_of_simplex_copy": None if scopy is None else achieved / scopy["gbs"],
        },
        "copy": copy,
        "simplex_copy": scopy,
        "power": power,
        "cpu_baseline": None,
    }
    if op == "map":
        res["roofline"] = None   # the map alone moves no bytes: see tiles and timings
    if not args.no_cpu and op != "edm":
        log("cpu_baseline: oracle on a bounded sample")
        res["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
