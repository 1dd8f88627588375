"""Seeded synthetic inputs shared by the CPU oracle side and the HIP side.

This module holds no part of the method: it only draws numbers, fills boxes
and marks the cells outside the simplex with poison.  Both sides of every
parity test get their inputs from here, so the two never exchange data.

Generator: splitmix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014), in its usual counter form: the i-th output
(i = 0, 1, ...) of stream ``seed`` is ``mix(seed + (i+1) * 0x9E3779B97F4A7C15)``.
Being counter-based, any single cell of a box can be regenerated from its
linear index alone, which lets sampled checks of huge boxes rebuild exactly
the neighbourhoods they read.

Box layout: the (n+1)^m bounding box, row-major, x_1 fastest.  As a numpy or
torch array it has shape ``(n+1,)*m`` with the LAST axis being x_1; the cell
x is at linear index ``sum_k x_k (n+1)^(k-1)`` and the box is filled in that
linear order.

Distributions:
  * ``u31``   uint32 uniform on [0, 2^31): the top 31 bits of each output.
  * ``bern``  uint8 Bernoulli(p): 1 iff (top 32 bits) < floor(p * 2^32).
Poison (cells outside the simplex, which no operation may read as data):
0xFFFFFFFF for uint32 inputs and 1 ("alive") for uint8 cells.  Output
buffers start as the sentinel 0xDEADBEEF (uint32) or 0xA5 (uint8) everywhere.

The synthetic workloads follow the shapes of the paper's test kernels
(Section 5.1, Table tab:tests); the paper draws from no public dataset.
"""
from __future__ import annotations

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
MIX1 = 0xBF58476D1CE4E5B9
MIX2 = 0x94D049BB133111EB
U64 = (1 << 64) - 1

POISON_U32 = 0xFFFFFFFF
POISON_U8 = 1
SENTINEL_U32 = 0xDEADBEEF
SENTINEL_U8 = 0xA5

# Seeded synthetic workloads (sizes of the paper's 2-D and 3-D tests, plus a
# 4-D hash).  ``dist`` describes buf_in; None means the op reads no input.
WORKLOADS = {
    "c1": dict(m=2, n=1024, op="accum", seed=22081161701, dist="u31", p=None),
    "c2": dict(m=2, n=16384, op="ca2", seed=22081161702, dist="bern", p=0.3),
    "c3": dict(m=3, n=1024, op="ca3", seed=22081161703, dist="bern", p=0.2),
    "c4": dict(m=4, n=128, op="hash", seed=22081161704, dist=None, p=None),
}

# Serving stream: one automaton step per job, mixed sizes, Poisson arrivals.
SERVE = dict(seed=22081161705, frac_m2=0.6, n2=(64, 4096), n3=(32, 512), p=0.25, levels=64)


def serve_trace(count: int, rate_per_s=None, seed: int = SERVE["seed"], levels: int = SERVE["levels"]):
    """Job stream [(m, n, arrival_s)]: a fraction frac_m2 of jobs with m = 2
    and n log-uniform in n2, the rest m = 3 with n log-uniform in n3; each n
    is rounded to one of ``levels`` log-spaced sizes of its class, so jobs of
    one size can share an input box.  Arrivals are a Poisson process of rate
    ``rate_per_s`` (None or 0: every job arrives at t = 0)."""
    rng = np.random.default_rng(seed)
    grids = {2: np.unique(np.round(np.geomspace(*SERVE["n2"], levels)).astype(np.int64)),
             3: np.unique(np.round(np.geomspace(*SERVE["n3"], levels)).astype(np.int64))}
    jobs, t = [], 0.0
    for _ in range(count):
        m = 2 if rng.random() < SERVE["frac_m2"] else 3
        lo, hi = SERVE["n2"] if m == 2 else SERVE["n3"]
        want = np.exp(rng.uniform(np.log(lo), np.log(hi)))
        g = grids[m]
        n = int(g[np.argmin(np.abs(np.log(g) - np.log(want)))])
        if rate_per_s:
            t += rng.exponential(1.0 / rate_per_s)
        jobs.append((m, n, t))
    return jobs


def serve_seed(m: int, n: int) -> int:
    """Seed of the shared input box of the jobs of size (m, n)."""
    return SERVE["seed"] * 1000003 + m * 100000 + n


def bern_threshold(p: float) -> int:
    """floor(p * 2^32), the comparison threshold on the top 32 bits."""
    return int(np.floor(p * 4294967296.0))


# ---------------------------------------------------------------- numpy side

def splitmix64(seed: int, start: int, count: int) -> np.ndarray:
    """Outputs start .. start+count-1 of the splitmix64 stream ``seed`` (uint64)."""
    with np.errstate(over="ignore"):
        i = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        z = np.uint64(seed & U64) + i * np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(MIX1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(MIX2)
        return z ^ (z >> np.uint64(31))


def splitmix64_at(seed: int, idx: np.ndarray) -> np.ndarray:
    """Outputs at arbitrary stream positions ``idx`` (any integer array)."""
    with np.errstate(over="ignore"):
        i = np.asarray(idx, dtype=np.uint64) + np.uint64(1)
        z = np.uint64(seed & U64) + i * np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(MIX1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(MIX2)
        return z ^ (z >> np.uint64(31))


def _draw(z: np.ndarray, dist: str, p) -> np.ndarray:
    if dist == "u31":
        return (z >> np.uint64(33)).astype(np.uint32)
    if dist == "bern":
        return ((z >> np.uint64(32)) < np.uint64(bern_threshold(p))).astype(np.uint8)
    raise ValueError(dist)


def values_at(seed: int, dist: str, p, idx) -> np.ndarray:
    """Generator values (before poisoning) at linear box indices ``idx``."""
    return _draw(splitmix64_at(seed, idx), dist, p)


def outside_mask_rows(m: int, n: int, lead_sum: int) -> np.ndarray:
    """Boolean mask over the trailing (m-1)-dim box block of shape (n+1,)*(m-1)
    whose coordinates sum with ``lead_sum`` to more than n."""
    r = np.arange(n + 1, dtype=np.int64)
    s = np.full((), lead_sum, dtype=np.int64)
    for _ in range(m - 1):
        s = np.add.outer(s, r)
    return s > n


def box(m: int, n: int, dist: str, seed: int, p=None, poison: bool = True,
        chunk: int = 1 << 18) -> np.ndarray:
    """The full (n+1)^m input box, generated in linear order, then poisoned."""
    total = (n + 1) ** m
    dt = np.uint8 if dist == "bern" else np.uint32
    flat = np.empty(total, dtype=dt)
    for s in range(0, total, chunk):
        c = min(chunk, total - s)
        flat[s:s + c] = _draw(splitmix64(seed, s, c), dist, p)
    arr = flat.reshape((n + 1,) * m)
    if poison:
        poison_outside(arr, m, n)
    return arr


def poison_outside(arr: np.ndarray, m: int, n: int, value=None) -> None:
    """Overwrite every cell outside Delta_n^m with the poison (or ``value``)."""
    if value is None:
        value = POISON_U8 if arr.dtype == np.uint8 else POISON_U32
    for lead in range(n + 1):  # slab x_m = lead
        arr[lead][outside_mask_rows(m, n, lead)] = value


def sentinel_box(m: int, n: int, dtype) -> np.ndarray:
    dtype = np.dtype(dtype)
    val = SENTINEL_U8 if dtype == np.uint8 else SENTINEL_U32
    return np.full((n + 1,) * m, val, dtype=dtype)


def inside_mask(m: int, n: int) -> np.ndarray:
    """Boolean box mask of Delta_n^m (for small boxes only)."""
    r = np.arange(n + 1, dtype=np.int64)
    s = np.zeros((), dtype=np.int64)
    for _ in range(m):
        s = np.add.outer(s, r)
    return s <= n


def linear_index(m: int, n: int, x) -> int:
    """i(x) = sum_k x_k (n+1)^(k-1), with x given as (x_1, ..., x_m)."""
    i, stride = 0, 1
    for k in range(m):
        i += int(x[k]) * stride
        stride *= n + 1
    return i


# ---------------------------------------------------------------- torch side
# The same stream computed with torch int64 arithmetic (two's-complement
# wrap-around), so boxes can be generated directly in device memory.

def _s64(c: int) -> int:
    c &= U64
    return c - (1 << 64) if c >= (1 << 63) else c


def _lsr(z, s: int):
    """Logical right shift of an int64 tensor."""
    return (z >> s) & ((1 << (64 - s)) - 1)


def splitmix64_torch(seed: int, start: int, count: int, device="cpu"):
    import torch
    i = torch.arange(start + 1, start + count + 1, dtype=torch.int64, device=device)
    z = i * _s64(GAMMA) + _s64(seed)
    z = (z ^ _lsr(z, 30)) * _s64(MIX1)
    z = (z ^ _lsr(z, 27)) * _s64(MIX2)
    return z ^ _lsr(z, 31)


def box_torch(m: int, n: int, dist: str, seed: int, p=None, device="cuda",
              poison: bool = True, chunk: int = 1 << 26):
    """Device-resident version of :func:`box` (bit-identical values)."""
    import torch
    total = (n + 1) ** m
    dt = torch.uint8 if dist == "bern" else torch.int32
    flat = torch.empty(total, dtype=dt, device=device)
    thr = bern_threshold(p) if dist == "bern" else 0
    for s in range(0, total, chunk):
        c = min(chunk, total - s)
        z = splitmix64_torch(seed, s, c, device)
        if dist == "u31":
            flat[s:s + c] = _lsr(z, 33).to(torch.int32)
        else:
            flat[s:s + c] = (_lsr(z, 32) < thr).to(torch.uint8)
        del z
    arr = flat.view((n + 1,) * m)
    if poison:
        poison_outside_torch(arr, m, n)
    return arr


def poison_outside_torch(arr, m: int, n: int) -> None:
    import torch
    val = POISON_U8 if arr.dtype == torch.uint8 else -1  # -1 == 0xFFFFFFFF as int32
    r = torch.arange(n + 1, dtype=torch.int64, device=arr.device)
    # trailing (m-1)-dim coordinate sums, built once
    if m == 2:
        arr.masked_fill_((r.unsqueeze(-1) + r) > n, val)
        return
    s = torch.zeros((), dtype=torch.int64, device=arr.device)
    for _ in range(m - 1):
        s = s.unsqueeze(-1) + r
    for lead in range(n + 1):
        arr[lead].masked_fill_(s > (n - lead), val)


def sentinel_box_torch(m: int, n: int, u8: bool, device="cuda"):
    import torch
    shape = (n + 1,) * m
    if u8:
        return torch.full(shape, SENTINEL_U8, dtype=torch.uint8, device=device)
    return torch.full(shape, SENTINEL_U32 - (1 << 32), dtype=torch.int32, device=device)


def points(n: int, seed: int, dim: int = 3) -> np.ndarray:
    """n+1 points in [0, 1)^dim, float32: coordinate c of point k is the top
    24 bits of splitmix64 output k*dim + c, divided by 2^24 (exact in
    float32)."""
    z = splitmix64(seed, 0, (n + 1) * dim)
    return ((z >> np.uint64(40)).astype(np.float64) / 16777216.0).astype(np.float32).reshape(n + 1, dim)
