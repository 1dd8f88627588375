"""Host-side checks of the block-space maps (no GPU).

``simplex_plan_tiles`` runs, on the host, the same decode functions the
kernels run, for every workgroup of a launch.  These tests check that the
decoded tiles are exactly the block simplex {b : sum b <= floor(n/rho)},
each hit once, and that the launched counts equal the paper's closed forms:
V(S_N^2) = N(N-1)/2 (Lemma 1, eq_m2), the packed 3-D grid
(N/2) x (N/2) x 3N/4 (Section 4.3, after Lemma 4) with its 9/8 limit, the
generic self-similar volume (N^m - beta^log2(N)) / (2^m - beta)
(Section 6, eq_generic-m with r = 1/2), and the bounding box
ceil((n+1)/rho)^m with its m! limit (Section 2).
"""
import math
import os

import numpy as np
import pytest

from paper_2208_11617_amd import binding as smap

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

TILES = {  # (m, op) -> supported rho values
    (2, "hits"): [16, 32, 64, 128],
    (3, "hits"): [8, 16, 32],
    (4, "hits"): [4, 8, 16],
    (2, "ca2"): [128, 256, 512, 1024, 2048, 4096],
    (3, "ca3"): [32, 64, 128, 256],
}


def check_exact(m, n, op, use_bb=False, beta=0):
    info = smap.plan_info(m, n, op, use_bb=use_bb, beta=beta)
    rho = info["rho"]
    M = n // rho
    valid, tiles = smap.plan_tiles(m, n, op, use_bb=use_bb, beta=beta)
    assert len(valid) == info["launched_tiles"]
    t = tiles[valid].astype(np.int64)
    assert np.all(t >= 0)
    assert np.all(t.sum(axis=1) <= M)
    keys = np.zeros(len(t), dtype=np.int64)
    for k in range(m):
        keys = keys * (M + 1) + t[:, k]
    assert len(np.unique(keys)) == len(t), "a tile is mapped twice"
    assert len(t) == math.comb(M + m, m) == info["useful_tiles"]
    return info


@pytest.mark.parametrize("m,op,nmax", [(2, "hits", 300), (3, "hits", 130), (4, "hits", 40),
                                       (2, "ca2", 300), (3, "ca3", 130)])
def test_h_covers_block_simplex_exactly_once(m, op, nmax):
    try:
        for rho in TILES[(m, op)]:
            smap.set_tile(m, op, rho)
            for n in range(0, nmax + 1):
                check_exact(m, n, op)
                if m == 4:
                    check_exact(m, n, op, beta=4)
    finally:
        smap.set_tile(m, op, 0)


@pytest.mark.parametrize("m,op", [(2, "hits"), (3, "hits"), (4, "hits"), (2, "ca2"), (3, "ca3")])
def test_bb_covers_block_simplex_exactly_once(m, op):
    for n in list(range(0, 70)) + [257, 1023]:
        if m == 4 and n == 1023:
            # 256^2 tiles would exceed the 65535 z-extent of the 3-D grid
            with pytest.raises(smap.SimplexMapError):
                smap.plan_info(m, n, op, use_bb=True)
            continue
        info = check_exact(m, n, op, use_bb=True)
        assert info["launched_tiles"] == ((n + info["rho"]) // info["rho"]) ** m


@pytest.mark.parametrize("m,n,op,beta", [(2, 1024, "accum", 0), (2, 16384, "ca2", 0),
                                         (3, 1024, "ca3", 0), (4, 128, "hash", 3),
                                         (4, 128, "hash", 4)])
def test_workload_plans_exact(m, n, op, beta):
    check_exact(m, n, op, beta=beta)


def test_large_k_sweep():
    # larger block simplices than the n-sweeps reach, odd K included
    smap.set_tile(2, "hits", 16)
    smap.set_tile(3, "hits", 8)
    try:
        for n in (16 * 254, 16 * 255, 16 * 256 + 7, 16 * 383, 16 * 511 + 15):
            check_exact(2, n, "hits")
        for n in (8 * 62, 8 * 63, 8 * 64 + 3, 8 * 95):
            check_exact(3, n, "hits")
    finally:
        smap.set_tile(2, "hits", 0)
        smap.set_tile(3, "hits", 0)


def _native_n(m, K):
    return 1 << int(math.floor(math.log2(K + 1)))


def test_native_counts_match_closed_forms():
    # K = 2^j - 1 exactly: the launch is the native map alone.
    smap.set_tile(2, "hits", 16)
    smap.set_tile(3, "hits", 8)
    smap.set_tile(4, "hits", 4)
    try:
        for j in range(1, 9):
            N = 1 << j
            n = 16 * (N - 2)
            info = smap.plan_info(2, n, "hits")
            assert info["shell_layers"] == 0 and info["native_n"] == N
            assert info["launched_tiles"] == N * (N - 1) // 2          # eq_m2
            assert info["launched_tiles"] == info["useful_tiles"]       # no waste in 2-D
        for j in range(1, 8):
            N = 1 << j
            info = smap.plan_info(3, 8 * (N - 2), "hits")
            assert info["native_n"] == N and info["shell_layers"] == 0
            assert info["launched_tiles"] == (N // 2) ** 2 * (N // 2 + N // 4)
            assert info["useful_tiles"] == (N ** 3 - N) // 6          # eq_m3
        for j in range(1, 6):
            N = 1 << j
            for beta in (3, 4):
                info = smap.plan_info(4, 4 * (N - 2), "hits", beta=beta)
                assert info["native_n"] == N and info["shell_layers"] == 0
                # eq_generic-m with r = 1/2
                assert info["launched_tiles"] * (16 - beta) == N ** 4 - beta ** j
    finally:
        for m in (2, 3, 4):
            smap.set_tile(m, "hits", 0)


def test_packed_3d_grid_ratio_tends_to_nine_eighths():
    # Section 4.3: the packed grid over the useful tiles -> 1 + 1/8.
    smap.set_tile(3, "hits", 8)
    try:
        ratios = []
        for j in (4, 6, 8):
            N = 1 << j
            info = smap.plan_info(3, 8 * (N - 2), "hits")
            ratios.append(info["launched_tiles"] / info["useful_tiles"])
        assert ratios[0] > ratios[1] > ratios[2] > 1.125
        assert abs(ratios[2] - 1.125) < 0.002
    finally:
        smap.set_tile(3, "hits", 0)


def test_bb_ratio_tends_to_m_factorial():
    # Section 2: launched / useful -> m! for the bounding box
    for m, n in ((2, 16384), (3, 1024), (4, 128)):
        smap.set_tile(m, "hits", {2: 16, 3: 8, 4: 4}[m])
        try:
            info = smap.plan_info(m, n, "hits", use_bb=True)
            ratio = info["launched_tiles"] / info["useful_tiles"]
            assert abs(ratio / math.factorial(m) - 1) < 0.25
        finally:
            smap.set_tile(m, "hits", 0)


def test_theorem1_worked_case():
    """N = 4: the six blocks of the 2 x 3 grid land on { X < Y <= 3 }."""
    rows = []
    with open(os.path.join(GOLDEN, "h2_n4_theorem1.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(v) for v in line.split()])
    smap.set_tile(2, "hits", 16)
    try:
        n = 16 * 2  # floor(n / rho) = 2, K = 3 = N - 1 with N = 4: native map only
        info = smap.plan_info(2, n, "hits")
        assert info["native_n"] == 4 and info["shell_layers"] == 0 and info["launched_tiles"] == 6
        valid, tiles = smap.plan_tiles(2, n, "hits")
        assert valid.all()
        for wx, wy, X, Y in rows:
            w = wx + 2 * wy  # grid row-major, w_x fastest
            assert tuple(tiles[w]) == (X, 4 - 1 - Y)
    finally:
        smap.set_tile(2, "hits", 0)


def test_hinge_is_used_in_3d():
    # Some 3-D workgroups of the first cube must be reflected by the hinge
    # (local sum >= 2b-1); without it coverage would fail, so check that the
    # reflected tiles exist: third coordinate >= N/2 comes only from the hinge.
    smap.set_tile(3, "hits", 8)
    try:
        n = 8 * 30  # K = 31 = N - 1, N = 32
        valid, tiles = smap.plan_tiles(3, n, "hits")
        t = tiles[valid]
        assert (t[:, 2] >= 16).sum() == math.comb(15 + 2, 3)  # corner T_3(15)
    finally:
        smap.set_tile(3, "hits", 0)


def test_m4_rejects_beta_two():
    with pytest.raises(smap.SimplexMapError) as e:
        smap.plan_info(4, 100, "hits", beta=2)
    assert e.value.status == smap.EUNSUPPORTED


def test_levels_layout_3d_covers_exactly_once_without_waste():
    """The level-ordered 3-D layout (the fully efficient variant of Section
    4.3): exactly-once coverage for every n and tile, and with no shell the
    launch is exactly the useful tiles, C(N+1, 3) = (N^3 - N) / 6."""
    smap.set_layout(3, smap.LAYOUT_LEVELS)
    try:
        for op in ("hits", "ca3"):
            for rho in TILES[(3, op)]:
                smap.set_tile(3, op, rho)
                for n in range(0, 131):
                    check_exact(3, n, op)
            smap.set_tile(3, op, 0)
        smap.set_tile(3, "hits", 8)
        for j in range(1, 9):
            N = 1 << j
            info = smap.plan_info(3, 8 * (N - 2), "hits")
            assert info["native_n"] == N and info["shell_layers"] == 0
            assert info["launched_tiles"] == info["useful_tiles"] == (N ** 3 - N) // 6
        # the 3-D workload (n = 1024, rho = 128): fewer launched tiles than packed
        lev = smap.plan_info(3, 1024, "ca3")
        smap.set_layout(3, smap.LAYOUT_PACKED)
        pk = smap.plan_info(3, 1024, "ca3")
        assert lev["useful_tiles"] == pk["useful_tiles"] and lev["launched_tiles"] < pk["launched_tiles"]
    finally:
        smap.set_tile(3, "hits", 0)
        smap.set_layout(3, smap.LAYOUT_AUTO)
    with pytest.raises(smap.SimplexMapError):
        smap.set_layout(2, smap.LAYOUT_LEVELS)
    with pytest.raises(smap.SimplexMapError):
        smap.set_layout(3, 7)
    with pytest.raises(smap.SimplexMapError):
        smap.set_layout(3, -2)
    with pytest.raises(smap.SimplexMapError):
        smap.set_layout(2, smap.LAYOUT_AUTO)


def test_concurrent_plan_queries_match_sequential():
    """The plan cache is shared and mutex-guarded: plan queries from several
    threads at once (ctypes releases the interpreter lock during the call)
    give the same answers as the same queries made one by one."""
    import threading
    keys = [(m, n, op, beta) for m, op, beta in ((2, "ca2", 0), (3, "ca3", 0), (4, "hash", 3), (4, "hash", 4),
                                                 (2, "accum", 0), (3, "hits", 0))
            for n in (7, 63, 129, 300, 1023) if m < 4 or n <= 300]
    want = {k: smap.plan_info(k[0], k[1], k[2], beta=k[3]) for k in keys}
    got, errors = {}, []

    def worker(part):
        try:
            for _ in range(20):
                for k in part:
                    got[k] = smap.plan_info(k[0], k[1], k[2], beta=k[3])
                    assert got[k] == want[k], k
        except Exception as e:   # collected and re-raised in the main thread
            errors.append(e)
    threads = [threading.Thread(target=worker, args=(keys[i::4] + keys[:3],)) for i in range(4)]
    smap.lib().simplex_autotune_reset()
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors[0]
    assert got == want


def test_auto_layout_levels_for_single_ca3_launches_only():
    """By default single CA3 launches (and their plan info) use the
    level-ordered layout at rho 256, the per-element ops the packed one."""
    assert smap.plan_info(3, 1024, "ca3")["rho"] == 256
    # the default CA3 tile: 128^3 below n = 768, 256^3 from there on (H and BB)
    for n, rho in ((0, 128), (500, 128), (767, 128), (768, 256), (2000, 256)):
        assert smap.plan_info(3, n, "ca3")["rho"] == rho, n
        assert smap.plan_info(3, n, "ca3", use_bb=True)["rho"] == rho, n
    auto_ca3, auto_hits = smap.plan_info(3, 1024, "ca3"), smap.plan_info(3, 1024, "hits")
    try:
        smap.set_layout(3, smap.LAYOUT_LEVELS)
        assert smap.plan_info(3, 1024, "ca3") == auto_ca3
        smap.set_layout(3, smap.LAYOUT_PACKED)
        assert smap.plan_info(3, 1024, "hits") == auto_hits
        assert smap.plan_info(3, 1024, "ca3")["launched_tiles"] > auto_ca3["launched_tiles"]
    finally:
        smap.set_layout(3, smap.LAYOUT_AUTO)
    for n in (0, 1, 255, 256, 511, 700):
        check_exact(3, n, "ca3")
