"""Boxes larger than 4 GiB: the 64-bit address path.

Each case steps a box of more than 2^32 bytes with H and with BB, checks
that the two agree on every byte, that every cell outside the simplex kept
its sentinel, and compares sampled rows with the oracle (the corner rows
included: the row x_2 = n, or the plane x_3 = n, sits past the first 4 GiB
of the buffer).  Poisoning and the outside checks run in row or plane
blocks so that no mask the size of the box is built.
"""
import numpy as np
import pytest

import simplex_inputs as si
from oracle import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def smap():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2208_11617_amd import binding
    binding.lib()
    return binding


def _outside_blocks(m, n, block=2048):
    """(index, mask) pairs covering the box: mask marks cells outside the
    simplex within arr[index] (rows of a 2-D box, planes of a 3-D or 4-D one)."""
    r = torch.arange(n + 1, device="cuda", dtype=torch.int64)
    if m == 2:
        for y0 in range(0, n + 1, block):
            y = r[y0:y0 + block]
            yield slice(y0, y0 + len(y)), r.view(1, -1) > (n - y).view(-1, 1)
    elif m == 3:
        s2 = r.view(-1, 1) + r
        for z in range(n + 1):
            yield z, s2 > n - z
    else:
        s2 = r.view(-1, 1) + r
        for w in range(n + 1):
            for z in range(n + 1):
                yield (w, z), s2 > n - w - z


def _poison(arr, m, n):
    val = si.POISON_U8 if arr.dtype == torch.uint8 else -1
    for idx, mask in _outside_blocks(m, n):
        arr[idx].masked_fill_(mask, val)


def _outside_untouched(arr, m, n, sentinel):
    for idx, mask in _outside_blocks(m, n):
        assert bool((arr[idx][mask] == sentinel).all()), idx


def _row_inputs(m, n, dist, seed, p, rows):
    """Lazily allocated host box with only the input rows the oracle reads
    for the sampled output rows, regenerated from the seed."""
    box = np.zeros((n + 1,) * m, dtype=np.uint8 if dist == "bern" else np.uint32)
    need = set()
    for hi in rows:
        for d in np.ndindex(*(3,) * (m - 1)):
            nb = tuple(int(h) + int(k) - 1 for h, k in zip(hi, d))
            if min(nb) >= 0 and sum(nb) <= n:
                need.add(nb)
    for nb in need:
        base = si.linear_index(m, n, (0,) + nb)
        length = n - sum(nb) + 1
        box[tuple(reversed(nb))][:length] = si.values_at(seed, dist, p, np.arange(base, base + length))
    return box


CASES = [
    # (m, n, op, dist, p): every box is above 4 GiB
    (2, 70000, "ca2", "bern", 0.3),     # 4.90e9 bytes
    (3, 1700, "ca3", "bern", 0.2),      # 4.92e9 bytes
    (2, 35000, "accum", "u31", None),   # 4.90e9 bytes (uint32)
    (4, 200, "hash", None, None),       # 6.53e9 bytes (uint32)
]


@pytest.mark.parametrize("m,n,op,dist,p", CASES)
def test_box_beyond_4gib(smap, m, n, op, dist, p):
    u8 = op.startswith("ca")
    esize = 1 if u8 else 4
    assert (n + 1) ** m * esize > (1 << 32)
    seed = 9100 + m
    say(f"large box m={m} n={n} op={op}: {(n + 1) ** m * esize / 1e9:.2f} GB per buffer")
    d_in = None
    if dist is not None:
        d_in = si.box_torch(m, n, dist, seed, p=p, device="cuda", poison=False)
        _poison(d_in, m, n)
    sentinel = si.SENTINEL_U8 if u8 else si.SENTINEL_U32 - (1 << 32)
    out_h = si.sentinel_box_torch(m, n, u8)
    smap.map_launch(m, n, op, d_in, out_h)
    torch.cuda.synchronize()
    say("  H done")
    out_b = si.sentinel_box_torch(m, n, u8)
    smap.bb_launch(m, n, op, d_in, out_b)
    torch.cuda.synchronize()
    say("  BB done")
    assert torch.equal(out_h, out_b)
    del out_b
    say("  outside untouched")
    _outside_untouched(out_h, m, n, sentinel)
    rng = np.random.default_rng(17)
    rows = {(0,) * (m - 1), (n,) + (0,) * (m - 2), (0,) * (m - 2) + (n,), (0,) * (m - 2) + (n - 1,)}
    while len(rows) < 24:
        v = rng.integers(0, n + 1, size=m - 1)
        if v.sum() <= n:
            rows.add(tuple(int(a) for a in v))
    rows = sorted(rows)
    inp = _row_inputs(m, n, dist, seed, p, rows) if dist is not None else None
    say(f"  {len(rows)} sampled rows against the oracle")
    for hi in rows:
        want = oracle.row(m, n, op, inp, hi)
        got = out_h[tuple(reversed(hi))][: len(want)].cpu().numpy().view(want.dtype)
        assert np.array_equal(got, want), (m, n, op, hi)
