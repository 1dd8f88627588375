"""Benchmark: useful simplex elements/s of one step of the hot path, H vs BB.

Default workload (the 2-D automaton step the metric is quoted on):
m = 2, n = 16384, one Life step B3/S23 on uint8 cells, Bernoulli(0.3),
(n+1)^2 box, ping-pong between two device-resident buffers.  A step is one
launch of the whole path (plan lookup, H decode, tile walk, op).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2]
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
BYTES_PER_ELEMENT = {"accum": 8, "ca2": 2, "ca3": 2, "hash": 4, "hits": 8, "map": 0}

# kernel sources whose change invalidates stored counter readings, per op
KERNEL_SOURCES = {
    "ca2": ["smap_decode.hpp", "smap_ca2.hpp"],
    "ca3": ["smap_decode.hpp", "smap_ca2.hpp", "smap_ca3.hpp"],
    "point": ["smap_decode.hpp", "smap_point.hpp"],
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sha(op: str) -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(op, KERNEL_SOURCES["point"]):
        with open(os.path.join(ROOT, "paper_2208_11617_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(workload: str, op: str):
    """HBM bytes per launch of the H kernel from the committed rocprofv3
    counter summary, or None when there is none or the kernel's sources
    changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_sha") != kernel_sha(op):
        return None
    return rec.get("hbm_bytes_per_launch")


def time_launches(fn, steps, warmup, stream):
    import torch
    for i in range(warmup):
        fn(i)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for i in range(steps):
        fn(warmup + i)
    end.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(end) / steps  # ms per launch


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
    return {
        "value": done_cells / elapsed if elapsed > 0 else None,
        "unit": "useful elements/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{done_cells} of {oracle.count(m, n)} elements (slabs x_{m} < {lo}), "
                  f"{elapsed:.1f} s single-threaded",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the cpu_baseline leg")
    ap.add_argument("--no-bb", action="store_true", help="skip timing the BB baseline")
    ap.add_argument("--no-copy", action="store_true", help="skip the plain-copy probe")
    ap.add_argument("--beta", type=int, default=0)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch

    import simplex_inputs as si
    from paper_2208_11617_amd import binding as smap

    w = si.WORKLOADS[args.workload]
    m, n, op = w["m"], w["n"], w["op"]
    u8 = op.startswith("ca")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    useful = smap.count(m, n)

    log(f"generating {args.workload}: m={m} n={n} op={op}")
    bufs = []
    if w["dist"] is not None:
        bufs.append(si.box_torch(m, n, w["dist"], w["seed"], p=w["p"], device=dev))
    out_a = si.sentinel_box_torch(m, n, u8, device=dev)
    torch.cuda.synchronize()

    def step_fn(launch):
        def fn(i):
            if u8:   # ping-pong: in -> a, a -> in, ...
                src, dst = (bufs[0], out_a) if i % 2 == 0 else (out_a, bufs[0])
                launch(m, n, op, src, dst, stream=stream)
            elif op == "accum":
                launch(m, n, op, bufs[0], out_a, stream=stream)
            else:
                launch(m, n, op, None, out_a, stream=stream)
        return fn

    h_launch = lambda *a, **k: smap.map_launch(*a, beta=args.beta, **k)  # noqa: E731
    log(f"timing H: {args.warmup} warmup + {args.steps} steps")
    h_ms = time_launches(step_fn(h_launch), args.steps, args.warmup, stream)
    bb_ms = None
    if not args.no_bb:
        log("timing BB")
        bb_ms = time_launches(step_fn(smap.bb_launch), args.steps, args.warmup, stream)

    copy = None
    if not args.no_copy:
        log("timing a plain copy of the same byte count")
        copy = copy_probe(max(useful * BYTES_PER_ELEMENT[op] // 2, 1 << 20), 20, stream)

    info_h = smap.plan_info(m, n, op, beta=args.beta)
    info_bb = smap.plan_info(m, n, op, use_bb=True)
    alg_bytes = useful * BYTES_PER_ELEMENT[op]
    achieved = alg_bytes / (h_ms * 1e-3) / 1e9
    traffic = stored_traffic(args.workload, op)
    value = useful / (h_ms * 1e-3)

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
                   "op": op, "useful_elements": useful, "rho": info_h["rho"],
                   "beta": info_h["beta"]},
        "hbm_gbs_algorithmic": achieved,
        "bb": None if bb_ms is None else {
            "ms_per_step": bb_ms, "value": useful / (bb_ms * 1e-3),
            "hbm_gbs_algorithmic": alg_bytes / (bb_ms * 1e-3) / 1e9},
        "h_vs_bb_speedup": None if bb_ms is None else bb_ms / h_ms,
        "tiles": {"useful": info_h["useful_tiles"], "h_launched": info_h["launched_tiles"],
                  "bb_launched": info_bb["launched_tiles"], "wgs_per_tile": info_h["wgs_per_tile"],
                  "h_workgroups": info_h["launched_wgs"], "bb_workgroups": info_bb["launched_wgs"]},
        "roofline": {
            "bound": "hbm" if op != "map" else "alu",
            "achieved": achieved,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS,
            "traffic": traffic,
            "kernel": f"{op} H launch",
            "kernel_sha": kernel_sha(op),
            "bytes_per_launch": alg_bytes,
            "copy_gbs": None if copy is None else copy["gbs"],
            "frac_of_copy": None if copy is None else achieved / copy["gbs"],
        },
        "copy": copy,
        "cpu_baseline": None,
    }
    if not args.no_cpu:
        log("cpu_baseline: oracle on a bounded sample")
        res["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
