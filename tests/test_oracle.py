"""Pins of the CPU oracle against facts fixed outside the oracle itself.

Every check here compares the oracle with something it does not contain:
the closed-form element count (Section 1, Eq. 1; Section 2, eq_volume with
the side-length shift), the stacking recurrence behind eq_volume_enum,
published hash vectors, the invertibility of fmix32, brute force on tiny
boxes, a library convolution (scipy) for the neighbour counts, and textbook
automaton patterns (still lifes, an oscillator, a glider).
"""
import math
import os
import random

import numpy as np
import pytest
from scipy import ndimage

import simplex_inputs as si
from oracle import oracle
from tests import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


# ------------------------------------------------------------------ counts

@pytest.mark.parametrize("m", [2, 3, 4])
def test_count_closed_form(m):
    # Eq. 1 has C(n+m, m) elements; eq_volume counts C(s+m-1, m) for an edge
    # of s cells, and an edge of Delta_n^m holds s = n+1 cells.
    for n in range(0, 41 if m < 4 else 25):
        s = n + 1
        assert oracle.count(m, n) == math.comb(n + m, m) == math.comb(s + m - 1, m)


@pytest.mark.parametrize("m", [2, 3])
def test_count_stacking_recurrence(m):
    # eq_volume_enum: an (m+1)-simplex is a stack of m-simplices of every size.
    for n in range(0, 20):
        assert oracle.count(m + 1, n) == sum(oracle.count(m, k) for k in range(n + 1))


def test_paper_volume_examples():
    # Section 2: V(Delta^2) = s(s+1)/2 and V(Delta^3) = s(s+1)(s+2)/6 for an
    # edge of s cells.
    for n in range(0, 30):
        s = n + 1
        assert oracle.count(2, n) == s * (s + 1) // 2
        assert oracle.count(3, n) == s * (s + 1) * (s + 2) // 6


# ---------------------------------------------------------- enumeration/HITS

@pytest.mark.parametrize("m,n", [(2, 0), (2, 1), (2, 7), (3, 0), (3, 5), (4, 3), (2, 33), (3, 17)])
def test_hits_visits_simplex_exactly_once(m, n):
    out = si.sentinel_box(m, n, np.uint32)
    visited = oracle.apply(m, n, "hits", None, out)
    assert visited == math.comb(n + m, m)
    inside = si.inside_mask(m, n)
    assert np.all(out[inside] == si.SENTINEL_U32 + 1)
    assert np.all(out[~inside] == si.SENTINEL_U32)


@pytest.mark.parametrize("m,n", [(2, 6), (3, 4), (4, 3)])
def test_hits_matches_brute_force_positions(m, n):
    out = np.zeros((n + 1,) * m, dtype=np.uint32)
    oracle.apply(m, n, "hits", None, out)
    flat = out.reshape(-1)
    expect = np.zeros_like(flat)
    for x in brute.cells(m, n):
        expect[brute.flat_index(n, x)] += 1
    assert np.array_equal(flat, expect)


# ------------------------------------------------------------------ ACCUM

@pytest.mark.parametrize("m,n", [(2, 40), (3, 12), (4, 7)])
def test_accum(m, n):
    inp = si.box(m, n, "u31", seed=5 + m)
    inside = si.inside_mask(m, n)
    inp[(0,) * m] = 0xFFFFFFFF  # inside the simplex: must wrap to 0
    out = si.sentinel_box(m, n, np.uint32)
    oracle.apply(m, n, "accum", inp, out)
    want = inp.astype(np.uint64) + 1
    assert out[(0,) * m] == 0
    assert np.array_equal(out[inside], (want[inside] & 0xFFFFFFFF).astype(np.uint32))
    assert np.all(out[~inside] == si.SENTINEL_U32)


def test_accum_in_place():
    m, n = 2, 30
    buf = si.box(m, n, "u31", seed=3)
    ref = buf.copy()
    oracle.apply(m, n, "accum", buf, buf)
    inside = si.inside_mask(m, n)
    assert np.array_equal(buf[inside], ref[inside] + 1)
    assert np.array_equal(buf[~inside], ref[~inside])


# ------------------------------------------------------------------ MAP

def test_map_writes_nothing():
    m, n = 3, 9
    out = si.sentinel_box(m, n, np.uint32)
    assert oracle.apply(m, n, "map", None, out) == math.comb(n + m, m)
    assert np.all(out == si.SENTINEL_U32)


# ------------------------------------------------------------------ hash

def test_hash_published_vectors():
    rows = _golden("published_vectors.txt")
    seen = set()
    for row in rows:
        if row[0] == "fnv1a32":
            words = list(row[1].encode())
            assert oracle.fnv1a_words(words) == int(row[2], 16), row
            seen.add("fnv")
        elif row[0] == "murmur3_empty":
            assert oracle.fmix32(int(row[1], 16)) == int(row[2], 16), row
            seen.add("fmix")
    assert seen == {"fnv", "fmix"}


def _unfmix32(h):
    """Inverse of fmix32 built from the mathematics: xorshift inverses and
    modular inverses of the two odd multipliers."""
    M = 1 << 32
    h ^= h >> 16
    h = (h * pow(0xC2B2AE35, -1, M)) % M
    h ^= (h >> 13) ^ (h >> 26)
    h = (h * pow(0x85EBCA6B, -1, M)) % M
    h ^= h >> 16
    return h


def test_fmix32_is_a_bijection():
    rng = random.Random(7)
    for _ in range(2000):
        x = rng.getrandbits(32)
        assert _unfmix32(oracle.fmix32(x)) == x


def test_fnv_step_is_injective_in_last_word():
    # (h ^ w) * p with p odd is a bijection of w, so distinct last words give
    # distinct prefix hashes.
    vals = {oracle.fnv1a_words([3, 1, w]) for w in range(4096)}
    assert len(vals) == 4096


@pytest.mark.parametrize("m,n", [(2, 20), (3, 9), (4, 6)])
def test_hash_box(m, n):
    out = si.sentinel_box(m, n, np.uint32)
    oracle.apply(m, n, "hash", None, out)
    flat = out.reshape(-1)
    for x in brute.cells(m, n):
        assert flat[brute.flat_index(n, x)] == oracle.fmix32(oracle.fnv1a_words(list(x)))
    inside = si.inside_mask(m, n)
    assert np.all(out[~inside] == si.SENTINEL_U32)
    # coordinate order matters (x_1 is hashed first)
    assert oracle.hash32([1, 2]) != oracle.hash32([2, 1])


# ------------------------------------------------------------------ CA

def _ca_reference_scipy(m, n, inp, birth, survive):
    """Neighbour counts by library convolution: zero everything outside the
    simplex, convolve with a 3^m box kernel (constant-zero boundary), subtract
    the centre."""
    inside = si.inside_mask(m, n)
    live = np.where(inside, inp == 1, False).astype(np.int32)
    cnt = ndimage.convolve(live, np.ones((3,) * m, dtype=np.int32), mode="constant", cval=0) - live
    nxt = np.where(live == 1, np.isin(cnt, survive), np.isin(cnt, birth)).astype(np.uint8)
    return nxt, inside


@pytest.mark.parametrize("n,p,seed", [(0, 0.3, 1), (1, 0.5, 2), (2, 0.5, 3), (11, 0.3, 4), (64, 0.3, 5), (97, 0.45, 6)])
def test_ca2_against_library_convolution(n, p, seed):
    inp = si.box(2, n, "bern", seed, p=p)
    out = si.sentinel_box(2, n, np.uint8)
    oracle.apply(2, n, "ca2", inp, out)
    nxt, inside = _ca_reference_scipy(2, n, inp, [3], [2, 3])
    assert np.array_equal(out[inside], nxt[inside])
    assert np.all(out[~inside] == si.SENTINEL_U8)


@pytest.mark.parametrize("n,p,seed", [(0, 0.3, 1), (1, 0.5, 2), (3, 0.5, 3), (10, 0.3, 4), (33, 0.2, 5), (40, 0.5, 6)])
def test_ca3_against_library_convolution(n, p, seed):
    inp = si.box(3, n, "bern", seed, p=p)
    out = si.sentinel_box(3, n, np.uint8)
    oracle.apply(3, n, "ca3", inp, out)
    nxt, inside = _ca_reference_scipy(3, n, inp, [6], [5, 6, 7])
    assert np.array_equal(out[inside], nxt[inside])
    assert np.all(out[~inside] == si.SENTINEL_U8)


@pytest.mark.parametrize("m,n,op,birth,survive", [(2, 9, "ca2", {3}, {2, 3}), (3, 6, "ca3", {6}, {5, 6, 7})])
def test_ca_against_brute_force(m, n, op, birth, survive):
    inp = si.box(m, n, "bern", 11, p=0.5)
    out = si.sentinel_box(m, n, np.uint8)
    oracle.apply(m, n, op, inp, out)
    flat_in, flat_out = inp.reshape(-1), out.reshape(-1)
    grid = {x: int(flat_in[brute.flat_index(n, x)]) for x in brute.cells(m, n)}
    nxt = brute.life_step(m, n, grid, birth, survive)
    for x, v in nxt.items():
        assert flat_out[brute.flat_index(n, x)] == v, x


def _run(m, n, op, inp):
    out = si.sentinel_box(m, n, np.uint8)
    oracle.apply(m, n, op, inp, out)
    return out


def _pattern(m, n, cells):
    g = np.zeros((n + 1,) * m, dtype=np.uint8)
    for x in cells:  # x = (x_1, ..., x_m); numpy index is reversed
        g[tuple(reversed(x))] = 1
    si.poison_outside(g, m, n)
    return g


def _live(m, n, g):
    inside = si.inside_mask(m, n)
    return {tuple(reversed(t)) for t in zip(*np.nonzero((g == 1) & inside))}


def test_ca2_textbook_patterns():
    n = 60
    block = {(10, 10), (11, 10), (10, 11), (11, 11)}
    assert _live(2, n, _run(2, n, "ca2", _pattern(2, n, block))) == block
    blinker = {(20, 12), (21, 12), (22, 12)}
    g1 = _run(2, n, "ca2", _pattern(2, n, blinker))
    assert _live(2, n, g1) == {(21, 11), (21, 12), (21, 13)}
    g2 = _run(2, n, "ca2", np.where(si.inside_mask(2, n), g1, 1).astype(np.uint8))
    assert _live(2, n, g2) == blinker
    glider = {(11, 10), (12, 11), (10, 12), (11, 12), (12, 12)}
    g = _pattern(2, n, glider)
    for _ in range(4):
        g = np.where(si.inside_mask(2, n), _run(2, n, "ca2", g), 1).astype(np.uint8)
    assert _live(2, n, g) == {(a + 1, b + 1) for a, b in glider}


def test_ca2_outside_is_dead_not_alive():
    # Everything inside dead, everything outside poisoned "alive": a rule that
    # counted outside cells would give births along the hypotenuse.
    n = 25
    g = _pattern(2, n, set())
    assert _live(2, n, _run(2, n, "ca2", g)) == set()
    g3 = _pattern(3, 12, set())
    assert _live(3, 12, _run(3, 12, "ca3", g3)) == set()


def test_ca3_cube_still_life():
    # Under B6/S567 each cell of a 2x2x2 cube has 7 live neighbours and every
    # outside cell has at most 4, so the cube is a still life.
    n = 20
    cube = {(4 + a, 5 + b, 6 + c) for a in (0, 1) for b in (0, 1) for c in (0, 1)}
    assert _live(3, n, _run(3, n, "ca3", _pattern(3, n, cube))) == cube
    single = {(3, 3, 3)}
    assert _live(3, n, _run(3, n, "ca3", _pattern(3, n, single))) == set()


def test_ca_ignores_poison_values():
    m, n = 2, 30
    inp = si.box(m, n, "bern", 9, p=0.4)
    a = _run(m, n, "ca2", inp)
    inp2 = inp.copy()
    si.poison_outside(inp2, m, n, value=0)
    b = _run(m, n, "ca2", inp2)
    assert np.array_equal(a, b)


# ------------------------------------------------------------ slab and cell

def test_slabs_compose_to_full_run():
    m, n = 3, 14
    inp = si.box(m, n, "bern", 21, p=0.3)
    full = _run(m, n, "ca3", inp)
    part = si.sentinel_box(m, n, np.uint8)
    total = 0
    for lo in range(0, n + 1, 4):
        total += oracle.apply_slab(m, n, "ca3", inp, part, lo, lo + 4)
    assert total == math.comb(n + m, m)
    assert np.array_equal(full, part)


def test_cell_matches_full_run():
    rng = random.Random(3)
    for m, n, op in [(2, 40, "ca2"), (3, 15, "ca3"), (2, 30, "accum"), (4, 8, "hash")]:
        dist = "bern" if op.startswith("ca") else "u31"
        inp = si.box(m, n, dist, 4, p=0.35)
        if op == "hash":
            inp = np.zeros((n + 1,) * m, dtype=np.uint32)
        out = si.sentinel_box(m, n, oracle.dtype_of(op))
        oracle.apply(m, n, op, inp, out)
        flat = out.reshape(-1)
        pts = brute.cells(m, n)
        for x in rng.sample(pts, 50):
            assert oracle.cell(m, n, op, inp, x) == int(flat[brute.flat_index(n, x)])
        assert oracle.cell(m, n, op, inp, (n, 1) + (0,) * (m - 2)) == -1


def test_rejects_bad_arguments():
    inp = si.box(2, 5, "bern", 1, p=0.5)
    with pytest.raises(ValueError):
        oracle.apply(2, 5, "ca2", inp, inp)  # in place is not allowed for CA
    with pytest.raises(ValueError):
        oracle.apply(3, 5, "ca2", None, None)


# ---------------------------------------------------------- shared generator

def test_generator_published_vector():
    row = [r for r in _golden("published_vectors.txt") if r[0] == "splitmix64"][0]
    got = si.splitmix64(int(row[1]), 0, 3)
    assert [int(v) for v in got] == [int(h, 16) for h in row[2:]]


def test_generator_numpy_and_torch_agree():
    torch = pytest.importorskip("torch")
    a = si.splitmix64(22081161702, 12345, 5000)
    b = si.splitmix64_torch(22081161702, 12345, 5000).numpy().view(np.uint64)
    assert np.array_equal(a, b)
    for m, n, dist, p in [(2, 37, "bern", 0.3), (3, 11, "bern", 0.2), (2, 19, "u31", None)]:
        x = si.box(m, n, dist, 77, p=p)
        y = si.box_torch(m, n, dist, 77, p=p, device="cpu").numpy()
        assert np.array_equal(x.view(y.dtype), y)
    idx = np.array([0, 5, 999])
    assert np.array_equal(si.values_at(77, "bern", 0.3, idx),
                          si.box(2, 37, "bern", 77, p=0.3, poison=False).reshape(-1)[idx])


def test_bernoulli_thresholds():
    assert si.bern_threshold(0.3) == 1288490188
    assert si.bern_threshold(0.2) == 858993459
    assert si.bern_threshold(0.25) == 1073741824


# ---- EDM (Section 5.1, test 3): pins against closed forms and invariants ----

def _edm_pair(out, n, i, j):
    """The oracle's value for the pair (i, j), i <= j: element (x_1, x_2) = (i, n - j)."""
    return out[n - j, i]          # numpy axes (x_2, x_1)


def test_edm_collinear_points_give_index_gaps():
    n = 40
    pts = np.zeros((n + 1, 3), dtype=np.float32)
    pts[:, 0] = np.arange(n + 1)
    out = oracle.edm(n, pts)
    for i in range(n + 1):
        for j in range(i, n + 1):
            assert _edm_pair(out, n, i, j) == j - i


@pytest.mark.parametrize("step,norm", [((3, 4, 0), 5), ((2, 3, 6), 7), ((1, 4, 8), 9)])
def test_edm_pythagorean_directions(step, norm):
    n = 25
    pts = (np.arange(n + 1)[:, None] * np.array(step)[None, :]).astype(np.float32)
    out = oracle.edm(n, pts)
    for i in range(0, n + 1, 3):
        for j in range(i, n + 1, 2):
            assert _edm_pair(out, n, i, j) == norm * (j - i)


def test_edm_layout_diagonal_outside_and_symmetry_of_definition():
    n = 30
    pts = si.points(n, 77)
    out = oracle.edm(n, pts)
    x1 = np.arange(n + 1)[None, :]
    x2 = np.arange(n + 1)[:, None]
    inside = x1 + x2 <= n
    assert np.isnan(out[~inside]).all() and not np.isnan(out[inside]).any()
    assert (out[x1 + x2 == n] == 0.0).all()                   # i == j
    # d(p_i, p_j) for i < j equals the same definition with the roles swapped
    for i, j in [(0, n), (3, 17), (11, 12), (29, 30)]:
        d = np.sqrt(((pts[j].astype(np.float64) - pts[i]) ** 2).sum())
        assert abs(_edm_pair(out, n, i, j) - d) <= 1e-15


def test_edm_triangle_inequality_and_exact_scaling():
    n = 36
    pts = si.points(n, 91)
    out = oracle.edm(n, pts)
    D = np.zeros((n + 1, n + 1))
    for i in range(n + 1):
        for j in range(i, n + 1):
            D[i, j] = D[j, i] = _edm_pair(out, n, i, j)
    viol = D[:, None, :] > D[:, :, None] + D[None, :, :] + 1e-12   # d(i,k) > d(i,j) + d(j,k)
    assert not viol.any()
    out2 = oracle.edm(n, (pts * 2).astype(np.float32))        # exact in float32
    inside = ~np.isnan(out)
    assert np.array_equal(out2[inside], 2 * out[inside])
    coarse = (np.floor(pts * 4096.0) / 4096.0).astype(np.float32)   # 12-bit fractions
    shifted = (coarse + np.float32(0.5)).astype(np.float32)          # exact in float32
    assert np.array_equal(shifted - np.float32(0.5), coarse)
    assert np.array_equal(oracle.edm(n, shifted)[inside], oracle.edm(n, coarse)[inside])


def test_points_generator_is_exact_and_seeded():
    a, b = si.points(10, 5), si.points(10, 5)
    assert a.dtype == np.float32 and a.shape == (11, 3) and np.array_equal(a, b)
    assert ((a * 16777216.0) == np.round(a * 16777216.0)).all() and (a >= 0).all() and (a < 1).all()
    assert not np.array_equal(a, si.points(10, 6))
