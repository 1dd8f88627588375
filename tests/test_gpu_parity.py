"""GPU parity: the HIP kernels, called through the C ABI, against the oracle.

Integer work, so the bar is bit-exact equality everywhere, including the
sentinel left untouched outside the simplex.  Small and medium sizes compare
whole boxes; the workload sizes compare sampled rows (recomputed by the
oracle from inputs it regenerates itself from the shared seeded generator)
plus properties that hold at any size: H and BB give identical buffers, and
nothing outside the simplex is written.
"""
import math

import numpy as np
import pytest

import simplex_inputs as si
from oracle import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

POINT_TILES = {2: [16, 32, 64, 128], 3: [8, 16, 32], 4: [4, 8, 16]}
# (rho, threads, tiles per workgroup): one tile per workgroup at each compiled
# rho, plus every compiled grouping of x_1-adjacent tiles
POINT_SHAPES = {m: [(rho, 0, 1) for rho in POINT_TILES[m]] for m in POINT_TILES}
POINT_SHAPES[2] += [(32, 64, 1), (32, 64, 2)]
POINT_SHAPES[3] += [(16, 256, 2), (8, 256, 4), (16, 64, 1), (16, 64, 2)]
POINT_SHAPES[4] += [(8, 256, 4), (8, 128, 4), (8, 256, 2), (8, 256, 8), (4, 256, 8), (4, 256, 16),
                    (8, 64, 1), (8, 64, 2), (8, 64, 4), (8, 128, 2)]
CA2_TILES = [(1024, 64), (1024, 128), (1024, 256), (512, 512), (256, 256), (128, 128),
             (2048, 128), (2048, 256), (4096, 256)]


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def smap():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2208_11617_amd import binding  # raises if the library is missing
    binding.lib()
    return binding


def to_dev(a):
    t = torch.from_numpy(np.ascontiguousarray(a).view(np.int32 if a.dtype == np.uint32 else np.uint8))
    return t.cuda()


def to_host(t, dtype):
    return t.cpu().numpy().view(dtype)


def launch(smap, kind, m, n, op, d_in, d_out, beta=0):
    if kind == "h":
        smap.map_launch(m, n, op, d_in, d_out, beta=beta)
    else:
        smap.bb_launch(m, n, op, d_in, d_out)
    torch.cuda.synchronize()


def expected(m, n, op, inp):
    out = si.sentinel_box(m, n, oracle.dtype_of(op))
    oracle.apply(m, n, op, inp, out)
    return out


def fresh_out(m, n, op):
    return si.sentinel_box_torch(m, n, oracle.dtype_of(op) == np.uint8)


def same(d, want_dev):
    return torch.equal(d.reshape(-1), want_dev.reshape(-1))


def kinds(m):
    ks = [("h", 0), ("bb", 0)]
    if m == 4:
        ks.append(("h", 4))
    return ks


# --------------------------------------------------------------- pointwise

def _sweep(m):
    if m == 2:
        return list(range(0, 66)) + [100, 255, 256, 257, 1000]
    if m == 3:
        return list(range(0, 41)) + [63, 64, 65, 100]
    return list(range(0, 25)) + [31, 32, 33]


@pytest.mark.parametrize("m", [2, 3, 4])
def test_hits_cover_simplex_exactly_once(smap, m):
    try:
        for n in _sweep(m):
            want = to_dev(expected(m, n, "hits", None))
            for rho, wg, grp in POINT_SHAPES[m]:
                smap.set_shape(m, "hits", rho, wg, grp)
                for kind, beta in kinds(m):
                    say(f"hits m={m} n={n} shape={rho},{wg},{grp} {kind} beta={beta}")
                    d = fresh_out(m, n, "hits")
                    launch(smap, kind, m, n, "hits", None, d, beta)
                    assert same(d, want), (m, n, rho, wg, grp, kind, beta)
    finally:
        smap.set_tile(m, "hits", 0)


@pytest.mark.parametrize("m", [2, 3, 4])
@pytest.mark.parametrize("op", ["accum", "hash"])
def test_pointwise_parity(smap, m, op):
    try:
        for n in _sweep(m)[::3] + _sweep(m)[-4:]:
            inp = si.box(m, n, "u31", 1000 + n) if op == "accum" else None
            want = to_dev(expected(m, n, op, inp))
            d_in = to_dev(inp) if inp is not None else None
            for rho, wg, grp in POINT_SHAPES[m]:
                smap.set_shape(m, op, rho, wg, grp)
                for kind, beta in kinds(m):
                    say(f"{op} m={m} n={n} shape={rho},{wg},{grp} {kind} beta={beta}")
                    d_out = fresh_out(m, n, op)
                    launch(smap, kind, m, n, op, d_in, d_out, beta)
                    assert same(d_out, want), (m, n, rho, wg, grp, kind, beta)
    finally:
        smap.set_tile(m, op, 0)


def test_accum_in_place_and_wrap(smap):
    m, n = 2, 333
    inp = si.box(m, n, "u31", 5)
    inp[0, 0] = 0xFFFFFFFF
    want = expected(m, n, "accum", inp)
    want[~si.inside_mask(m, n)] = inp[~si.inside_mask(m, n)]  # in place: outside keeps input
    for kind in ("h", "bb"):
        d = to_dev(inp)
        launch(smap, kind, m, n, "accum", d, d)
        assert np.array_equal(to_host(d, np.uint32).reshape(want.shape), want)


def test_map_writes_nothing(smap):
    for m, n in ((2, 300), (3, 50), (4, 20)):
        d = to_dev(si.sentinel_box(m, n, np.uint32))
        for kind, beta in kinds(m):
            launch(smap, kind, m, n, "map", None, None, beta)
        assert np.all(to_host(d, np.uint32) == si.SENTINEL_U32)


# --------------------------------------------------------------- automata

CA2_SIZES = list(range(0, 70)) + [127, 128, 129, 255, 256, 257, 300, 511, 512, 513,
                                  767, 1000, 1023, 1024, 1025, 2047, 2049, 4095, 4097, 8200]


def test_ca2_parity(smap):
    try:
        for n in CA2_SIZES:
            inp = si.box(2, n, "bern", 2000 + n, p=0.3)
            want = to_dev(expected(2, n, "ca2", inp))
            d_in = to_dev(inp)
            for rho, wg in CA2_TILES:
                smap.set_tile(2, "ca2", rho, wg)
                for kind in ("h", "bb"):
                    say(f"ca2 n={n} rho={rho} wg={wg} {kind}")
                    d_out = fresh_out(2, n, "ca2")
                    launch(smap, kind, 2, n, "ca2", d_in, d_out)
                    assert same(d_out, want), (n, rho, wg, kind)
    finally:
        smap.set_tile(2, "ca2", 0)


CA3_SIZES = list(range(0, 41)) + [62, 63, 64, 65, 66, 95, 96, 97, 127, 128, 150]


CA3_TILES = [(128, 256), (128, 128), (128, 512), (256, 256), (256, 128), (256, 512), (64, 128), (64, 256),
             (32, 64)]


def test_ca3_parity(smap):
    try:
        for n in CA3_SIZES:
            inp = si.box(3, n, "bern", 3000 + n, p=0.2 if n % 2 else 0.5)
            want = to_dev(expected(3, n, "ca3", inp))
            d_in = to_dev(inp)
            for rho, wg in CA3_TILES:
                smap.set_tile(3, "ca3", rho, wg)
                for kind in ("h", "bb"):
                    say(f"ca3 n={n} rho={rho} wg={wg} {kind}")
                    d_out = fresh_out(3, n, "ca3")
                    launch(smap, kind, 3, n, "ca3", d_in, d_out)
                    assert same(d_out, want), (n, rho, wg, kind)
    finally:
        smap.set_tile(3, "ca3", 0)


def test_ca3_unaligned_buffers(smap):
    """Boxes that start k bytes past a 16-byte boundary, for input and
    output: the CA3 staging loads and the stores then meet every alignment
    of a row against 16 bytes, including the first row of the buffer; the
    bytes around the output view stay untouched."""
    cases = [(15, (1, 5, 8, 15)), (16, (3, 12)), (17, (0, 7, 14)), (40, (1, 9)), (130, (4, 11)),
             (300, (2, 13))]
    try:
        for n, shifts in cases:
            inp = si.box(3, n, "bern", 3300 + n, p=0.3)
            want = to_dev(expected(3, n, "ca3", inp)).reshape(-1)
            src = to_dev(inp).reshape(-1)
            total = (n + 1) ** 3
            for k in shifts:
                raw_in = torch.zeros(total + 32, dtype=torch.uint8, device="cuda")
                d_in = raw_in[k:k + total]
                d_in.copy_(src)
                ko = (7 * k + 3) % 16
                for rho, wg in ((256, 256), (256, 128), (128, 256), (64, 128), (32, 64)):
                    smap.set_tile(3, "ca3", rho, wg)
                    for kind in ("h", "bb"):
                        say(f"ca3 unaligned n={n} in+{k} out+{ko} rho={rho} wg={wg} {kind}")
                        raw_out = torch.full((total + 32,), si.SENTINEL_U8, dtype=torch.uint8, device="cuda")
                        d_out = raw_out[ko:ko + total]
                        launch(smap, kind, 3, n, "ca3", d_in, d_out)
                        assert same(d_out, want), (n, k, ko, rho, wg, kind)
                        assert bool((raw_out[:ko] == si.SENTINEL_U8).all()), (n, k, ko, rho, kind)
                        assert bool((raw_out[ko + total:] == si.SENTINEL_U8).all()), (n, k, ko, rho, kind)
    finally:
        smap.set_tile(3, "ca3", 0)


def test_ca2_unaligned_buffers(smap):
    """The 2-D step on boxes that start k bytes past a 16-byte boundary (input
    and output), at several tiles; the bytes around the output view stay
    untouched."""
    try:
        for n in (15, 16, 17, 100, 1000, 2100):
            inp = si.box(2, n, "bern", 2300 + n, p=0.3)
            want = to_dev(expected(2, n, "ca2", inp)).reshape(-1)
            src = to_dev(inp).reshape(-1)
            total = (n + 1) ** 2
            for k in (1, 7, 13):
                raw_in = torch.zeros(total + 32, dtype=torch.uint8, device="cuda")
                d_in = raw_in[k:k + total]
                d_in.copy_(src)
                ko = (5 * k + 2) % 16
                for rho, wg in ((1024, 64), (256, 256), (128, 128)):
                    smap.set_tile(2, "ca2", rho, wg)
                    for kind in ("h", "bb"):
                        say(f"ca2 unaligned n={n} in+{k} out+{ko} rho={rho} wg={wg} {kind}")
                        raw_out = torch.full((total + 32,), si.SENTINEL_U8, dtype=torch.uint8, device="cuda")
                        d_out = raw_out[ko:ko + total]
                        launch(smap, kind, 2, n, "ca2", d_in, d_out)
                        assert same(d_out, want), (n, k, ko, rho, wg, kind)
                        assert bool((raw_out[:ko] == si.SENTINEL_U8).all()), (n, k, ko, rho, kind)
                        assert bool((raw_out[ko + total:] == si.SENTINEL_U8).all()), (n, k, ko, rho, kind)
    finally:
        smap.set_tile(2, "ca2", 0)


@pytest.mark.parametrize("op", ["accum", "hash", "hits"])
def test_pointwise_unaligned_buffers(smap, op):
    """The 32-bit element ops on boxes that start 4, 8 or 12 bytes past a
    16-byte boundary (input and output), one tile per workgroup and grouped;
    the words around the output view stay untouched."""
    sent = si.SENTINEL_U32 - (1 << 32)
    cases = {2: (40, 257), 3: (33, 70), 4: (17, 40)}
    for m, ns in cases.items():
        shapes = [(0, 0, 1)] + [s for s in POINT_SHAPES[m] if s[2] > 1][:1]
        try:
            for n in ns:
                inp = si.box(m, n, "u31", 1700 + n) if op == "accum" else None
                want = to_dev(expected(m, n, op, inp)).reshape(-1)
                total = (n + 1) ** m
                for k in (1, 2, 3):
                    d_in = None
                    if inp is not None:
                        raw_in = torch.zeros(total + 8, dtype=torch.int32, device="cuda")
                        d_in = raw_in[k:k + total]
                        d_in.copy_(to_dev(inp).reshape(-1))
                    ko = 4 - k
                    for rho, wg, grp in shapes:
                        smap.set_shape(m, op, rho, wg, grp)
                        for kind, beta in kinds(m):
                            say(f"{op} unaligned m={m} n={n} in+{4 * k} out+{4 * ko} shape={rho},{wg},{grp} {kind}")
                            raw_out = torch.full((total + 8,), sent, dtype=torch.int32, device="cuda")
                            d_out = raw_out[ko:ko + total]
                            launch(smap, kind, m, n, op, d_in, d_out, beta)
                            assert same(d_out, want), (m, n, k, rho, wg, grp, kind, beta)
                            assert bool((raw_out[:ko] == sent).all()) and bool((raw_out[ko + total:] == sent).all())
        finally:
            smap.set_tile(m, op, 0)


def test_ca2_two_steps_ping_pong(smap):
    n = 700
    a = si.box(2, n, "bern", 77, p=0.35)
    step1 = expected(2, n, "ca2", a)
    step2 = expected(2, n, "ca2", step1)  # outside cells of step1 hold the sentinel: never read
    for kind in ("h", "bb"):
        d_a, d_b = to_dev(a), to_dev(si.sentinel_box(2, n, np.uint8))
        launch(smap, kind, 2, n, "ca2", d_a, d_b)
        launch(smap, kind, 2, n, "ca2", d_b, d_a)
        got = to_host(d_a, np.uint8).reshape(a.shape)
        inside = si.inside_mask(2, n)
        assert np.array_equal(got[inside], step2[inside])
        assert np.array_equal(got[~inside], a[~inside])


def test_side_stream(smap):
    n = 1500
    inp = si.box(2, n, "bern", 91, p=0.3)
    want = expected(2, n, "ca2", inp)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        d_in = to_dev(inp)
        d_out = to_dev(si.sentinel_box(2, n, np.uint8))
        smap.map_launch(2, n, "ca2", d_in, d_out, stream=s)
    s.synchronize()
    assert np.array_equal(to_host(d_out, np.uint8).reshape(want.shape), want)


# --------------------------------------------------- workload sizes (sampled)

def _row_inputs(m, n, dist, seed, p, rows):
    """Full-size (lazily allocated) host box holding only the input rows the
    oracle reads for the sampled output rows, regenerated from the seed."""
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
        vals = si.values_at(seed, dist, p, np.arange(base, base + length))
        box[tuple(reversed(nb))][:length] = vals
    return box


def _sample_rows(m, n, rng, k):
    rows = set()
    corner = [(0,) * (m - 1), (n,) + (0,) * (m - 2), (0,) * (m - 2) + (n,)]
    for c in corner:
        rows.add(c)
    if m == 3:  # rows on both sides of the 256-cell tile faces in y and z
        faces = [v for v in (0, 255, 256, 511, 512, 767, 768) if v <= n]
        rows.update((y, z) for y in faces for z in faces if y + z <= n)
    while len(rows) < k:
        v = rng.integers(0, n + 1, size=m - 1)
        if v.sum() <= n:
            rows.add(tuple(int(a) for a in v))
    return sorted(rows)


def _check_outside_untouched(d, m, n, sentinel):
    r = torch.arange(n + 1, device=d.device)
    if m == 2:
        mask = (r.unsqueeze(1) + r) > n
        assert bool((d[mask] == sentinel).all())
        return
    s2 = r.view(-1, 1) + r
    if m == 3:
        for z in range(n + 1):
            assert bool((d[z][s2 > n - z] == sentinel).all()), z
        return
    for w in range(n + 1):
        for z in range(n + 1 - w if w <= n else 0):
            assert bool((d[w, z][s2 > n - w - z] == sentinel).all()), (w, z)
        for z in range(max(n + 1 - w, 0), n + 1):
            assert bool((d[w, z] == sentinel).all()), (w, z)


@pytest.mark.parametrize("name", ["c1", "c2", "c3", "c4"])
def test_workload_parity(smap, name):
    w = si.WORKLOADS[name]
    m, n, op = w["m"], w["n"], w["op"]
    u8 = op.startswith("ca")
    sentinel = si.SENTINEL_U8 if u8 else si.SENTINEL_U32 - (1 << 32)
    say(f"workload {name}: m={m} n={n} op={op}")
    d_in = None
    if w["dist"] is not None:
        d_in = si.box_torch(m, n, w["dist"], w["seed"], p=w["p"], device="cuda")
    outs = {}
    for kind, beta in kinds(m):
        say(f"  launch {kind} beta={beta}")
        d_out = si.sentinel_box_torch(m, n, u8)
        launch(smap, kind, m, n, op, d_in, d_out, beta)
        outs[(kind, beta)] = d_out
    ref = outs[("h", 0)]
    for key, d in outs.items():
        assert torch.equal(d, ref), f"{key} differs from H"
    say("  outside untouched")
    _check_outside_untouched(ref, m, n, sentinel)
    if name == "c1":  # small enough for the whole box
        inp = si.box(m, n, w["dist"], w["seed"], p=w["p"])
        want = expected(m, n, op, inp)
        assert np.array_equal(to_host(ref, np.uint32).reshape(want.shape), want)
        return
    rng = np.random.default_rng(5)
    rows = _sample_rows(m, n, rng, 48)
    say(f"  {len(rows)} sampled rows")
    inp = _row_inputs(m, n, w["dist"], w["seed"], w["p"], rows) if w["dist"] else None
    for hi in rows:
        want = oracle.row(m, n, op, inp, hi)
        idx = tuple(reversed(hi))
        got = ref[idx][: len(want)].cpu().numpy().view(want.dtype)
        assert np.array_equal(got, want), (name, hi)
    assert smap.count(m, n) == math.comb(n + m, m)


# ---- EDM (Section 5.1, test 3): float32 against the float64 oracle ----------
#
# Tolerance: the kernel computes three float32 differences, their squares,
# a sum and sqrtf; with each operation rounded to nearest (relative error
# at most u = 2^-24) the sum of squares is within 5u relative and its
# square root within 2.5u + the square root's own rounding, at most 3.5u
# relative, i.e. at most 3.5 ulp of the float32 result (an ulp is at least
# u times the value); 4 ulp also covers a square root good to 1 ulp.  The
# diagonal (i = j) is exactly 0.
EDM_SIZES = [0, 1, 2, 3, 4, 5, 7, 30, 31, 32, 33, 63, 64, 65, 127, 129, 300, 1000]
EDM_TILES = [32, 16, 64, 128]


def _edm_check(got_bits, want, n):
    got = got_bits.view(np.float32).astype(np.float64)
    inside = ~np.isnan(want)
    ulp = np.spacing(want[inside].astype(np.float32)).astype(np.float64)
    err = np.abs(got[inside] - want[inside])
    assert (err <= 4 * ulp).all(), (n, float((err / ulp).max()))
    x1 = np.arange(n + 1)[None, :]
    x2 = np.arange(n + 1)[:, None]
    assert (got[(x1 + x2) == n] == 0).all()
    assert (got_bits.view(np.uint32)[~inside] == si.SENTINEL_U32).all()   # outside never written


def test_edm_parity(smap):
    try:
        for n in EDM_SIZES:
            pts = si.points(n, 9000 + n)
            want = oracle.edm(n, pts)
            d_pts = torch.from_numpy(pts).cuda()
            for rho in EDM_TILES:
                smap.set_tile(2, "edm", rho)
                for kind in ("h", "bb"):
                    say(f"edm n={n} rho={rho} {kind}")
                    d_out = torch.from_numpy(si.sentinel_box(2, n, np.uint32).view(np.int32)).cuda()
                    launch(smap, kind, 2, n, "edm", d_pts, d_out)
                    _edm_check(d_out.cpu().numpy().view(np.uint32), want, n)
    finally:
        smap.set_tile(2, "edm", 0)


def test_levels_layout_3d(smap):
    """The level-ordered 3-D layout: exactly-once hits and bit-exact CA3."""
    smap.set_layout(3, smap.LAYOUT_LEVELS)
    try:
        for n in _sweep(3):
            want = to_dev(expected(3, n, "hits", None))
            for rho in POINT_TILES[3]:
                smap.set_tile(3, "hits", rho)
                say(f"levels hits n={n} rho={rho}")
                d = fresh_out(3, n, "hits")
                launch(smap, "h", 3, n, "hits", None, d)
                assert same(d, want), (n, rho)
        smap.set_tile(3, "hits", 0)
        for n in [0, 1, 14, 15, 16, 40, 63, 64, 65, 97, 128, 150]:
            inp = si.box(3, n, "bern", 3500 + n, p=0.25)
            want = to_dev(expected(3, n, "ca3", inp))
            d_in = to_dev(inp)
            for rho, wg in CA3_TILES:
                smap.set_tile(3, "ca3", rho, wg)
                say(f"levels ca3 n={n} rho={rho} wg={wg}")
                d_out = fresh_out(3, n, "ca3")
                launch(smap, "h", 3, n, "ca3", d_in, d_out)
                assert same(d_out, want), (n, rho, wg)
    finally:
        smap.set_tile(3, "hits", 0)
        smap.set_tile(3, "ca3", 0)
        smap.set_layout(3, smap.LAYOUT_AUTO)


# ---- the pieces as concurrent launches (Section 4.2's concurrent trapezoids)

def test_pieces_on_streams(smap):
    """SMAP_GENERAL_STREAMS: the native part and each shell piece run as
    launches of their own on separate streams.  Exactly-once coverage (HITS)
    over the n sweep for every m, every op bit-exact against the oracle, and
    the full-size workloads equal to the fused launch."""
    smap.set_general(smap.GENERAL_STREAMS)
    try:
        for m in (2, 3, 4):
            for n in _sweep(m):
                want = to_dev(expected(m, n, "hits", None))
                for beta in ((3, 4) if m == 4 else (0,)):
                    say(f"streams hits m={m} n={n} beta={beta}")
                    d = fresh_out(m, n, "hits")
                    launch(smap, "h", m, n, "hits", None, d, beta)
                    assert same(d, want), (m, n, beta)
        for m, op, sizes in ((2, "ca2", [0, 1, 14, 15, 16, 100, 1000, 1025, 2049]),
                             (3, "ca3", [0, 14, 15, 16, 40, 65, 130]),
                             (2, "accum", [0, 1, 40, 300]), (4, "hash", [0, 5, 33]),
                             (2, "edm", [0, 1, 31, 33, 300])):
            for n in sizes:
                say(f"streams {op} m={m} n={n}")
                if op == "edm":
                    pts = si.points(n, 3600 + n)
                    d_out = fresh_out(m, n, "accum")
                    smap.map_launch(m, n, "edm", torch.from_numpy(pts).cuda(), d_out)
                    torch.cuda.synchronize()
                    _edm_check(to_host(d_out, np.uint32).reshape(n + 1, n + 1), oracle.edm(n, pts), n)
                    continue
                dist = {"ca2": "bern", "ca3": "bern", "accum": "u31"}.get(op)
                inp = si.box(m, n, dist, 3600 + n, p=0.3) if dist else None
                want = to_dev(expected(m, n, op, inp))
                d_out = fresh_out(m, n, op)
                launch(smap, "h", m, n, op, None if inp is None else to_dev(inp), d_out)
                assert same(d_out, want), (op, n)
        for name in ("c2", "c3", "c4"):
            w = si.WORKLOADS[name]
            m, n, op = w["m"], w["n"], w["op"]
            u8 = op.startswith("ca")
            d_in = si.box_torch(m, n, w["dist"], w["seed"], p=w["p"], device="cuda") if w["dist"] else None
            outs = []
            for strategy in (smap.GENERAL_STREAMS, smap.GENERAL_FUSED):
                smap.set_general(strategy)
                say(f"streams workload {name} strategy={strategy}")
                d_out = si.sentinel_box_torch(m, n, u8)
                launch(smap, "h", m, n, op, d_in, d_out)
                outs.append(d_out)
            assert torch.equal(outs[0], outs[1]), name
            del outs, d_in
            smap.set_general(smap.GENERAL_STREAMS)
    finally:
        smap.set_general(smap.GENERAL_FUSED)
