"""Tiny-input brute force, written independently of the oracle.

Test infrastructure: enumerates the whole (n+1)^m box with itertools.product
and keeps the cells whose coordinates sum to at most n (Section 1, Eq. 1),
then applies each operation by direct neighbour enumeration.  It shares no
code with ``oracle/`` and is only meant for n up to ~20.
"""
from __future__ import annotations

import itertools


def cells(m, n):
    """All x in Delta_n^m, as tuples (x_1, ..., x_m)."""
    return [x for x in itertools.product(range(n + 1), repeat=m) if sum(x) <= n]


def flat_index(n, x):
    return sum(v * (n + 1) ** k for k, v in enumerate(x))


def life_step(m, n, grid, birth, survive):
    """One outer-totalistic step on Delta_n^m.  ``grid`` maps x -> 0/1 for
    cells inside the simplex only; anything not in it is dead."""
    offs = [d for d in itertools.product((-1, 0, 1), repeat=m) if any(d)]
    nxt = {}
    for x in grid:
        c = sum(grid.get(tuple(a + b for a, b in zip(x, d)), 0) for d in offs)
        nxt[x] = 1 if (c in survive if grid[x] == 1 else c in birth) else 0
    return nxt
