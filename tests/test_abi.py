"""The C-ABI library loads, exports every declared symbol, and rejects bad
arguments before launching anything (no GPU needed: every call here fails
validation or is host-only)."""
import math
import os
import re

import pytest

from paper_2208_11617_amd import binding as smap

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "simplexmap.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(simplex_\w+)\s*\(", src, re.M)))


def test_header_declares_the_binding_exports():
    assert _declared() == sorted(smap.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = smap.lib()
    for name in _declared():
        assert hasattr(lib, name), name


def test_status_strings():
    for s in (smap.OK, smap.EINVAL, smap.EUNSUPPORTED, smap.ERANGE, smap.EHIP):
        assert smap.strerror(s)
    assert smap.strerror(12345) == "unknown status"


def test_count():
    for m in (1, 2, 3, 4, 7):
        for n in (0, 1, 5, 128, 1024, 16384):
            want = math.comb(n + m, m)
            if want < 1 << 64:
                assert smap.count(m, n) == want
            else:
                with pytest.raises(smap.SimplexMapError):
                    smap.count(m, n)
    assert smap.count(4, 128) == 12082785
    with pytest.raises(smap.SimplexMapError) as e:
        smap.count(30, 1 << 40)
    assert e.value.status == smap.ERANGE
    with pytest.raises(smap.SimplexMapError):
        smap.count(2, -1)


FAKE = 0x10000000  # never dereferenced: every call below fails validation


@pytest.mark.parametrize("launch", ["h", "bb"])
def test_argument_errors(launch):
    def call(m, n, op, i, o):
        if launch == "h":
            return smap.map_launch_raw(m, n, 0, 0, op, i, o, None)
        return smap.bb_launch_raw(m, n, op, i, o, None)

    assert call(1, 10, smap.OP_ACCUM, FAKE, FAKE) == smap.EINVAL     # m = 1: no map needed
    assert call(5, 10, smap.OP_ACCUM, FAKE, FAKE) == smap.EINVAL
    assert call(2, -1, smap.OP_ACCUM, FAKE, FAKE) == smap.EINVAL
    assert call(2, 10, 7, FAKE, FAKE) == smap.EINVAL                  # unknown op
    assert call(3, 10, smap.OP_EDM, FAKE, FAKE) == smap.EINVAL         # EDM needs m = 2
    assert call(2, 10, smap.OP_EDM, None, FAKE) == smap.EINVAL         # no points
    assert call(2, 10, smap.OP_EDM, FAKE, None) == smap.EINVAL
    assert call(2, 10, smap.OP_EDM, FAKE + 4, FAKE) == smap.EINVAL     # points not 16-byte aligned
    assert call(2, 10, -1, FAKE, FAKE) == smap.EINVAL
    assert call(3, 10, smap.OP_CA2, FAKE, FAKE + 4096) == smap.EINVAL  # CA2 needs m = 2
    assert call(2, 10, smap.OP_CA3, FAKE, FAKE + 4096) == smap.EINVAL  # CA3 needs m = 3
    assert call(2, 10, smap.OP_ACCUM, None, FAKE) == smap.EINVAL
    assert call(2, 10, smap.OP_ACCUM, FAKE, None) == smap.EINVAL
    assert call(2, 10, smap.OP_HITS, FAKE, None) == smap.EINVAL
    assert call(2, 10, smap.OP_HASH, None, None) == smap.EINVAL
    assert call(2, 10, smap.OP_CA2, FAKE, FAKE) == smap.EINVAL         # in place
    assert call(2, 10, smap.OP_CA2, FAKE, FAKE + 100) == smap.EINVAL   # overlap (box = 121 B)
    assert call(3, 10, smap.OP_CA3, FAKE + 1000, FAKE) == smap.EINVAL  # overlap (box = 1331 B)
    assert call(2, 10, smap.OP_CA2, None, FAKE) == smap.EINVAL
    assert call(4, 1 << 20, smap.OP_HASH, None, FAKE) == smap.ERANGE   # box too large
    assert call(2, 1 << 31, smap.OP_ACCUM, FAKE, FAKE) == smap.ERANGE


def test_unsupported_r_beta():
    raw = smap.map_launch_raw
    assert raw(2, 10, 3, 0, smap.OP_HITS, None, FAKE, None) == smap.EUNSUPPORTED  # r = 1/3
    assert raw(2, 10, 2, 3, smap.OP_HITS, None, FAKE, None) == smap.EUNSUPPORTED  # beta 3 for m = 2
    assert raw(3, 10, 2, 4, smap.OP_HITS, None, FAKE, None) == smap.EUNSUPPORTED
    # m = 4 with the paper's (r, beta) = (1/2, 2) cannot cover the simplex
    assert raw(4, 10, 2, 2, smap.OP_HITS, None, FAKE, None) == smap.EUNSUPPORTED
    assert raw(4, 10, 2, 5, smap.OP_HITS, None, FAKE, None) == smap.EUNSUPPORTED


def test_set_tile_validation():
    with pytest.raises(smap.SimplexMapError):
        smap.set_tile(2, "accum", 24)
    with pytest.raises(smap.SimplexMapError):
        smap.set_tile(4, "hash", 8, 512)
    with pytest.raises(smap.SimplexMapError):
        smap.set_tile(2, "ca2", 256, wg_threads=512)
    with pytest.raises(smap.SimplexMapError):
        smap.set_tile(2, "ca2", 64)
    with pytest.raises(smap.SimplexMapError):
        smap.set_tile(3, "ca3", 16)
    with pytest.raises(smap.SimplexMapError):
        smap.set_tile(3, "ca3", 32, 256)
    with pytest.raises(smap.SimplexMapError):
        smap.set_tile(3, "ca3", 64, 512)
    smap.set_tile(2, "ca2", 128)
    assert smap.plan_info(2, 1000, "ca2")["rho"] == 128
    assert smap.plan_info(2, 1000, "ca2")["wg_threads"] == 128
    smap.set_tile(2, "ca2", 1024, 256)
    info = smap.plan_info(2, 16384, "ca2")
    assert info["wg_threads"] == 256 and info["wgs_per_tile"] == 16
    assert info["launched_wgs"] == 16 * info["launched_tiles"]
    smap.set_tile(2, "ca2", 0)
    info = smap.plan_info(2, 16384, "ca2")
    assert info["rho"] == 1024 and info["wg_threads"] == 64 and info["wgs_per_tile"] == 256


def test_plan_info_fields():
    info = smap.plan_info(2, 16384, "ca2")
    assert info["useful_elements"] == 134242305
    assert info["tile_side_k"] == 17 and info["native_n"] == 16 and info["shell_layers"] == 2
    bb = smap.plan_info(2, 16384, "ca2", use_bb=True)
    assert bb["launched_tiles"] == 17 * 17 and bb["use_bb"] == 1
    assert smap.plan_info(4, 128, "hash")["beta"] == 3
    assert smap.plan_info(4, 128, "hash", beta=4)["beta"] == 4


def test_batch_launch_argument_errors():
    """simplex_batch_launch validates every job before enqueueing anything."""
    E = smap.EINVAL
    assert smap.batch_launch_raw([], 0) == smap.OK            # empty batch: no-op
    assert smap.batch_launch_raw([], -1) == E
    assert smap.lib().simplex_batch_launch(None, 3, None) == E
    good = (2, "ca2", 100, 4096, 1 << 20)
    assert smap.batch_launch_raw([(2, "ca3", 10, 4096, 1 << 20)]) == E   # CA3 needs m = 3
    assert smap.batch_launch_raw([(3, "ca2", 10, 4096, 1 << 20)]) == E
    assert smap.batch_launch_raw([(2, "accum", 10, 4096, 1 << 20)]) == E  # automata only
    assert smap.batch_launch_raw([good, (2, "ca2", -1, 4096, 1 << 20)]) == E
    assert smap.batch_launch_raw([good, (2, "ca2", 100, 0, 1 << 20)]) == E  # NULL input
    assert smap.batch_launch_raw([good, (2, "ca2", 100, 4096, 4096 + 50)]) == E  # overlap


def test_queue_graph_argument_errors():
    """simplex_queue_graph_create validates before any device work."""
    import ctypes
    E = smap.EINVAL
    good = (2, "ca2", 100, 4096, 1 << 20)
    assert smap.queue_graph_create_raw([], 0) == E                       # no jobs
    assert smap.queue_graph_create_raw([good], max_workgroups=-1) == E
    assert smap.queue_graph_create_raw([(2, "hash", 10, 4096, 1 << 20)]) == E   # automata only
    assert smap.queue_graph_create_raw([good, (2, "ca2", 100, 4096, 4096 + 50)]) == E  # overlap
    assert smap.queue_graph_create_raw([good] * 4097) == smap.ERANGE     # more than one launch takes
    arr = smap._job_array([good])
    assert smap.lib().simplex_queue_graph_create(arr, 1, 0, None) == E   # NULL graph
    h = ctypes.c_void_p()
    assert smap.lib().simplex_queue_graph_create(None, 1, 0, ctypes.byref(h)) == E


def test_set_general_argument_errors():
    assert smap.lib().simplex_set_general(2) == smap.EINVAL
    assert smap.lib().simplex_set_general(-1) == smap.EINVAL
    assert smap.lib().simplex_set_general(smap.GENERAL_FUSED) == smap.OK


def test_queue_launch_argument_errors():
    """simplex_queue_launch validates every job and the workgroup cap first."""
    E = smap.EINVAL
    assert smap.queue_launch_raw([], 0) == smap.OK            # empty batch: no-op
    assert smap.queue_launch_raw([], -1) == E
    assert smap.lib().simplex_queue_launch(None, 3, 0, None) == E
    good = (2, "ca2", 100, 4096, 1 << 20)
    assert smap.queue_launch_raw([good], max_workgroups=-1) == E
    assert smap.queue_launch_raw([(2, "ca3", 10, 4096, 1 << 20)]) == E   # CA3 needs m = 3
    assert smap.queue_launch_raw([(3, "ca2", 10, 4096, 1 << 20)]) == E
    assert smap.queue_launch_raw([(3, "hash", 10, 4096, 1 << 20)]) == E  # automata only
    assert smap.queue_launch_raw([good, (3, "ca3", -1, 4096, 1 << 20)]) == E
    assert smap.queue_launch_raw([good, (2, "ca2", 100, 4096, 0)]) == E  # NULL output
    assert smap.queue_launch_raw([good, (2, "ca2", 100, 4096, 4096 + 50)]) == E  # overlap


def test_serve_run_argument_errors():
    """simplex_serve_run validates the whole job stream before any work."""
    E = smap.EINVAL
    arena, size = 1 << 12, 1 << 20
    assert smap.serve_run_raw([], 0, 0, smap.SERVE_BATCHED)[0] == smap.OK
    job = (2, "ca2", 100, 4096, 0.0)
    assert smap.serve_run_raw([job], arena, size, 7)[0] == E                    # bad mode
    assert smap.serve_run_raw([job], arena, size, smap.SERVE_BATCHED, 0)[0] == E  # max_inflight
    assert smap.serve_run_raw([job], arena, size, smap.SERVE_PERSISTENT, 0)[0] == E
    assert smap.serve_run_raw([job], 0, size, smap.SERVE_BATCHED)[0] == E       # no arena
    assert smap.serve_run_raw([(2, "ca2", 100, 4096, 1.0), (2, "ca2", 100, 4096, 0.5)],
                              arena, size, smap.SERVE_BATCHED)[0] == E          # arrivals out of order
    assert smap.serve_run_raw([(2, "ca2", 100, 4096, -1.0)], arena, size, smap.SERVE_BATCHED)[0] == E
    assert smap.serve_run_raw([(2, "ca2", 2000, 4096, 0.0)], arena, size, smap.SERVE_BATCHED)[0] == E  # never fits
    assert smap.serve_run_raw([(3, "ca2", 10, 4096, 0.0)], arena, size, smap.SERVE_BATCHED)[0] == E
    assert smap.serve_run_raw([(2, "ca2", 10, 0, 0.0)], arena, size, smap.SERVE_BATCHED)[0] == E
    # keep_outputs needs room for every output at once
    two = [(2, "ca2", 730, 4096, 0.0), (2, "ca2", 730, 4096, 0.0)]
    assert smap.serve_run_raw(two, arena, size, smap.SERVE_BATCHED, 2, True)[0] == E


def test_autotune_and_graph_argument_errors():
    """Validation happens before any device work."""
    import ctypes
    E = smap.EINVAL
    assert smap.autotune_raw(2, 100, "accum", 4096, 1 << 20, reps=0)[0] == E
    assert smap.autotune_raw(2, 100, "ca3", 4096, 1 << 20)[0] == E          # CA3 needs m = 3
    assert smap.autotune_raw(2, 100, "accum", 4096, 4096)[0] == E            # no in-place timing
    assert smap.autotune_raw(2, -1, "accum", 4096, 1 << 20)[0] == E
    assert smap.lib().simplex_autotune(2, 100, 1, 4096, 1 << 20, 5, None, None, None) == E
    assert smap.autotune_reset() is None
    L = smap.lib()
    h = ctypes.c_void_p()
    assert L.simplex_graph_create(2, 100, 0, 0, 1, 0, 4096, 1 << 20, 0, ctypes.byref(h)) == E   # steps < 1
    assert L.simplex_graph_create(2, 100, 0, 0, 1, 0, 4096, 1 << 20, 2, None) == E              # no handle
    assert L.simplex_graph_create(3, 100, 0, 0, 4, 1, 4096, 1 << 20, 2, ctypes.byref(h)) == E   # CA2 with m = 3
    assert L.simplex_graph_launch(None, None) == E
    assert L.simplex_graph_destroy(None) == smap.OK


def test_launch_steps_argument_errors():
    E, U = smap.EINVAL, smap.EUNSUPPORTED
    a, b = 4096, 1 << 24
    assert smap.launch_steps_raw(2, 100, "ca2", 0, a, b) == E          # steps < 1
    assert smap.launch_steps_raw(2, 100, "ca2", -3, a, b, use_bb=True) == E
    assert smap.launch_steps_raw(3, 40, "ca3", 0, a, b) == E          # steps < 1 (3-D)
    assert smap.launch_steps_raw(4, 40, "hash", 4, a, b) == U          # automata only
    assert smap.launch_steps_raw(3, 40, "ca2", 4, a, b) == E           # CA2 needs m = 2
    assert smap.launch_steps_raw(3, 40, "ca3", 4, a, a + 100) == E     # overlapping buffers
    assert smap.launch_steps_raw(2, 100, "accum", 4, a, b) == U
    assert smap.launch_steps_raw(2, 100, "ca3", 4, a, b) == E          # CA3 needs m = 3
    assert smap.launch_steps_raw(2, 100, "ca2", 4, a, a + 100) == E     # overlapping buffers
    assert smap.launch_steps_raw(2, 100, "ca2", 4, 0, b) == E           # NULL input


def test_accum_partial_overlap_rejected():
    """ACCUM may run in place (in == out) but not on buffers that overlap
    otherwise: lanes would read cells that others have already written."""
    for launch in (smap.map_launch_raw, smap.bb_launch_raw):
        args = (0, 0) if launch is smap.map_launch_raw else ()
        for shift in (4, 8, 100, 10 * 11 * 4 - 4, -4, -400):
            st = launch(2, 10, *args, smap.OP_ACCUM, FAKE, FAKE + shift, None)
            assert st == smap.EINVAL, shift


def test_batch_cross_job_overlap_rejected():
    """No job's output may overlap another job's output or input, in either
    batched launch kind; the check runs before anything is enqueued."""
    E = smap.EINVAL
    box = 101 * 101
    a_in, a_out = 1 << 20, 1 << 22
    b_in, b_out = 1 << 24, 1 << 26
    for raw in (smap.batch_launch_raw, smap.queue_launch_raw):
        # outputs overlap
        assert raw([(2, "ca2", 100, a_in, a_out), (2, "ca2", 100, b_in, a_out + box - 1)]) == E
        assert raw([(2, "ca2", 100, a_in, a_out + 7), (3, "ca3", 20, b_in, a_out)]) == E
        # another job's output reaches into an input
        assert raw([(2, "ca2", 100, a_in, a_out), (2, "ca2", 100, a_out + box - 1, b_out)]) == E
        assert raw([(2, "ca2", 100, b_out - 5, a_out), (2, "ca2", 100, b_in, b_out)]) == E
        # the same job set in the other order
        assert raw([(2, "ca2", 100, b_in, b_out), (2, "ca2", 100, b_out - 5, a_out)]) == E
    assert smap.queue_graph_create_raw([(2, "ca2", 100, a_in, a_out),
                                        (2, "ca2", 100, b_in, a_out + 3)]) == E


def test_copy_probe_argument_errors():
    E = smap.EINVAL
    raw = smap.copy_launch_raw
    assert raw(4, 10, FAKE, FAKE + (1 << 20)) == E          # m = 2 or 3 only
    assert raw(1, 10, FAKE, FAKE + (1 << 20)) == E
    assert raw(2, -1, FAKE, FAKE + (1 << 20)) == E
    assert raw(2, 10, None, FAKE) == E
    assert raw(3, 10, FAKE, None) == E
    assert raw(2, 10, FAKE, FAKE + 120) == E                # overlap (box = 121 B)
    assert raw(3, 10, FAKE + 1330, FAKE) == E               # overlap (box = 1331 B)
    assert raw(3, 1 << 20, FAKE, FAKE + (1 << 40)) == smap.ERANGE


def test_set_shape_validation_and_grouped_counts():
    """Tiles per workgroup: only compiled groupings are accepted; the plan
    reports ceil(units / tiles_per_wg) workgroups (BB: per row of the tile
    grid along x_1)."""
    bad = [(4, "hash", 8, 256, 3), (4, "hash", 8, 64, 8), (2, "accum", 32, 256, 4),
           (3, "ca3", 256, 256, 2), (2, "ca2", 1024, 64, 4)]
    for m, op, rho, wg, grp in bad:
        with pytest.raises(smap.SimplexMapError) as e:
            smap.set_shape(m, op, rho, wg, grp)
        assert e.value.status == smap.EUNSUPPORTED, (m, op, rho, wg, grp)
    for args in ((4, "hash", 8, -1, 4), (4, "hash", 8, 256, -1)):
        with pytest.raises(smap.SimplexMapError) as e:
            smap.set_shape(*args)
        assert e.value.status == smap.EINVAL
    try:
        smap.set_shape(3, "ca3", 256, 256, 1)        # automata: 0 or 1
        smap.set_shape(4, "hash", 8, 256, 0)          # first listed: two tiles per workgroup
        assert smap.plan_info(4, 128, "hash")["tiles_per_wg"] == 2
        smap.set_shape(4, "hash", 8, 256, 1)
        assert smap.plan_info(4, 128, "hash")["tiles_per_wg"] == 1
        for grp in (2, 4, 8):
            smap.set_shape(4, "hash", 8, 256, grp)
            h = smap.plan_info(4, 128, "hash")
            assert h["tiles_per_wg"] == grp and h["wgs_per_tile"] == 1
            assert h["launched_wgs"] == -(-h["launched_tiles"] // grp)
            bb = smap.plan_info(4, 128, "hash", use_bb=True)
            kb = -(-129 // 8)   # box tiles per axis
            assert bb["launched_tiles"] == kb ** 4
            assert bb["launched_wgs"] == -(-kb // grp) * kb ** 3
        smap.set_shape(4, "hash", 4, 256, 16)
        assert smap.plan_info(4, 128, "hash")["rho"] == 4
    finally:
        smap.set_tile(4, "hash", 0)
        smap.set_tile(3, "ca3", 0)
    assert smap.plan_info(4, 128, "hash")["tiles_per_wg"] == 2   # the default m = 4 shape
