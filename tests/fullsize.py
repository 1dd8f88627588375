"""Whole-box expected results at the workload sizes, computed by the oracle.

Test infrastructure: the inputs come from the shared seeded generator
(``simplex_inputs``, numpy side), generated chunk by chunk on several host
threads; the expected outputs come from the oracle's own slab entry point,
run over disjoint ranges of the outermost coordinate x_m on several host
threads (each slab is the plain definition; the threads only split the
loop, and ctypes releases the GIL during each call).  Nothing here touches
the GPU or the HIP library.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import simplex_inputs as si
from oracle import oracle

THREADS = max(1, min(16, len(os.sched_getaffinity(0))))


def box(m, n, dist, seed, p=None, chunk=1 << 22):
    """si.box(m, n, dist, seed, p) (same values), generated on THREADS threads."""
    total = (n + 1) ** m
    flat = np.empty(total, dtype=np.uint8 if dist == "bern" else np.uint32)

    def fill(s):
        c = min(chunk, total - s)
        flat[s:s + c] = si._draw(si.splitmix64(seed, s, c), dist, p)
    with ThreadPoolExecutor(THREADS) as ex:
        list(ex.map(fill, range(0, total, chunk)))
    arr = flat.reshape((n + 1,) * m)
    si.poison_outside(arr, m, n)
    return arr


def slab_ranges(m, n, parts):
    """Split x_m = 0..n into at most `parts` ranges of about equal cell counts
    (slab t holds C(n - t + m - 1, m - 1) cells)."""
    sizes = [math.comb(n - t + m - 1, m - 1) for t in range(n + 1)]
    total, target = sum(sizes), sum(sizes) / parts
    out, lo, acc = [], 0, 0
    for t, s in enumerate(sizes):
        acc += s
        if acc >= target * (len(out) + 1) or t == n:
            out.append((lo, t + 1))
            lo = t + 1
    assert out[-1][1] == n + 1 and sum(sizes[a] for a, b in out for a in range(a, b)) == total
    return out


def apply(m, n, op, inp, out):
    """oracle.apply(m, n, op, inp, out) over disjoint x_m ranges in parallel."""
    ranges = slab_ranges(m, n, THREADS * 2)
    with ThreadPoolExecutor(THREADS) as ex:
        visited = sum(ex.map(lambda r: oracle.apply_slab(m, n, op, inp, out, r[0], r[1]), ranges))
    assert visited == math.comb(n + m, m)
    return visited


def expected(m, n, op, inp):
    out = si.sentinel_box(m, n, oracle.dtype_of(op))
    apply(m, n, op, inp, out)
    return out
