"""ctypes binding of ``libsimplexmap.so`` (the C ABI in include/simplexmap.h).

Argument marshalling only: every step of the work runs in the HIP kernels
behind the C ABI.  Tensors provide device pointers (``data_ptr()``) and the
stream (``torch.cuda.current_stream().cuda_stream`` by default).  If the
library has not been built, loading raises -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsimplexmap.so")

OK, EINVAL, EUNSUPPORTED, ERANGE, EHIP = 0, -1, -2, -3, -4
OP_MAP, OP_ACCUM, OP_HITS, OP_HASH, OP_CA2, OP_CA3, OP_EDM = range(7)
OPS = {"map": OP_MAP, "accum": OP_ACCUM, "hits": OP_HITS, "hash": OP_HASH,
       "ca2": OP_CA2, "ca3": OP_CA3, "edm": OP_EDM}

# names declared in include/simplexmap.h
EXPORTS = ("simplex_map_launch", "simplex_bb_launch", "simplex_count",
           "simplex_plan_info", "simplex_plan_tiles", "simplex_set_tile",
           "simplex_strerror", "simplex_batch_launch", "simplex_serve_run",
           "simplex_autotune", "simplex_autotune_reset", "simplex_graph_create",
           "simplex_graph_launch", "simplex_graph_destroy", "simplex_map_launch_steps",
           "simplex_bb_launch_steps", "simplex_set_layout", "simplex_queue_launch",
           "simplex_set_general", "simplex_queue_graph_create", "simplex_copy_launch",
           "simplex_queue_launch_static", "simplex_set_shape")

LAYOUT_AUTO, LAYOUT_PACKED, LAYOUT_LEVELS = -1, 0, 1
GENERAL_FUSED, GENERAL_STREAMS = 0, 1

SERVE_SEQUENTIAL, SERVE_BATCHED, SERVE_PERSISTENT = 0, 1, 2


class SimplexMapError(RuntimeError):
    def __init__(self, status: int, what: str, detail: str | None = None):
        self.status = status
        super().__init__(f"{what}: {detail or strerror(status)} (status {status})")


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int32),
        ("use_bb", ctypes.c_int32),
        ("n", ctypes.c_int64),
        ("r", ctypes.c_int32),
        ("beta", ctypes.c_int32),
        ("rho", ctypes.c_int32),
        ("wg_threads", ctypes.c_int32),
        ("tile_side_k", ctypes.c_int32),
        ("native_n", ctypes.c_int32),
        ("shell_layers", ctypes.c_int32),
        ("n_pieces", ctypes.c_int32),
        ("wgs_per_tile", ctypes.c_int32),
        ("useful_elements", ctypes.c_uint64),
        ("useful_tiles", ctypes.c_uint64),
        ("launched_tiles", ctypes.c_uint64),
        ("launched_wgs", ctypes.c_uint64),
        ("native_wgs", ctypes.c_uint64),
        ("full_tiles", ctypes.c_uint64),
        ("tiles_per_wg", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class Job(ctypes.Structure):
    """struct simplex_job"""
    _fields_ = [("m", ctypes.c_int32), ("op", ctypes.c_int32), ("n", ctypes.c_int64),
                ("buf_in", ctypes.c_void_p), ("buf_out", ctypes.c_void_p)]


class ServeJob(ctypes.Structure):
    """struct simplex_serve_job"""
    _fields_ = [("m", ctypes.c_int32), ("op", ctypes.c_int32), ("n", ctypes.c_int64),
                ("buf_in", ctypes.c_void_p), ("arrival_s", ctypes.c_double)]


class ServeRecord(ctypes.Structure):
    """struct simplex_serve_record"""
    _fields_ = [("admit_s", ctypes.c_double), ("launch_s", ctypes.c_double),
                ("done_s", ctypes.c_double), ("release_s", ctypes.c_double),
                ("out_offset", ctypes.c_uint64),
                ("batch", ctypes.c_int32), ("status", ctypes.c_int32)]


class TuneResult(ctypes.Structure):
    """struct simplex_tune_result"""
    _fields_ = [("rho", ctypes.c_int32), ("wg_threads", ctypes.c_int32), ("beta", ctypes.c_int32),
                ("us", ctypes.c_float), ("tiles_per_wg", ctypes.c_int32)]


_lib = None


def lib():
    """Load the library (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2208_11617_amd.build` (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64
    ci = ctypes.c_int
    L.simplex_map_launch.argtypes = [ci, i64, ci, ci, ci, vp, vp, vp]
    L.simplex_map_launch.restype = ci
    L.simplex_bb_launch.argtypes = [ci, i64, ci, vp, vp, vp]
    L.simplex_bb_launch.restype = ci
    L.simplex_count.argtypes = [ci, i64, ctypes.POINTER(u64)]
    L.simplex_count.restype = ci
    L.simplex_plan_info.argtypes = [ci, i64, ci, ci, ci, ci, ctypes.POINTER(PlanInfo)]
    L.simplex_plan_info.restype = ci
    L.simplex_plan_tiles.argtypes = [ci, i64, ci, ci, ci, ci, vp, u64, ctypes.POINTER(u64)]
    L.simplex_plan_tiles.restype = ci
    L.simplex_set_tile.argtypes = [ci, ci, ci, ci]
    L.simplex_set_tile.restype = ci
    L.simplex_set_shape.argtypes = [ci, ci, ci, ci, ci]
    L.simplex_set_shape.restype = ci
    L.simplex_batch_launch.argtypes = [ctypes.POINTER(Job), ctypes.c_int32, vp]
    L.simplex_batch_launch.restype = ci
    L.simplex_queue_graph_create.argtypes = [ctypes.POINTER(Job), ctypes.c_int32, ctypes.c_int32,
                                              ctypes.POINTER(vp)]
    L.simplex_queue_graph_create.restype = ci
    L.simplex_set_general.argtypes = [ci]
    L.simplex_set_general.restype = ci
    L.simplex_queue_launch.argtypes = [ctypes.POINTER(Job), ctypes.c_int32, ctypes.c_int32, vp]
    L.simplex_queue_launch.restype = ci
    L.simplex_serve_run.argtypes = [ctypes.POINTER(ServeJob), ctypes.c_int32, vp, u64, ctypes.c_int32,
                                    ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ServeRecord)]
    L.simplex_serve_run.restype = ci
    L.simplex_autotune.argtypes = [ci, i64, ci, vp, vp, ctypes.c_int32, ctypes.c_char_p, vp,
                                   ctypes.POINTER(TuneResult)]
    L.simplex_autotune.restype = ci
    L.simplex_autotune_reset.argtypes = []
    L.simplex_autotune_reset.restype = ci
    L.simplex_graph_create.argtypes = [ci, i64, ci, ci, ci, ci, vp, vp, ctypes.c_int32, ctypes.POINTER(vp)]
    L.simplex_graph_create.restype = ci
    L.simplex_graph_launch.argtypes = [vp, vp]
    L.simplex_graph_launch.restype = ci
    L.simplex_graph_destroy.argtypes = [vp]
    L.simplex_graph_destroy.restype = ci
    L.simplex_map_launch_steps.argtypes = [ci, i64, ci, ci, ci, ctypes.c_int32, vp, vp, vp]
    L.simplex_map_launch_steps.restype = ci
    L.simplex_bb_launch_steps.argtypes = [ci, i64, ci, ctypes.c_int32, vp, vp, vp]
    L.simplex_bb_launch_steps.restype = ci
    L.simplex_set_layout.argtypes = [ci, ci]
    L.simplex_set_layout.restype = ci
    L.simplex_queue_launch_static.argtypes = [ctypes.POINTER(Job), ctypes.c_int32, ctypes.c_int32, vp]
    L.simplex_queue_launch_static.restype = ci
    L.simplex_copy_launch.argtypes = [ci, i64, vp, vp, vp]
    L.simplex_copy_launch.restype = ci
    L.simplex_strerror.argtypes = [ci]
    L.simplex_strerror.restype = ctypes.c_char_p
    _lib = L
    return L


def strerror(status: int) -> str:
    return lib().simplex_strerror(status).decode()


def _op(op) -> int:
    return OPS[op] if isinstance(op, str) else int(op)


def _check(status: int, what: str) -> None:
    if status != OK:
        raise SimplexMapError(status, what)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


# Element types the kernels read and write, per op (torch dtype names).
_U8 = ("uint8",)
_W32 = ("int32", "uint32", "float32")
_OP_DTYPES = {OP_ACCUM: (_W32, _W32), OP_HITS: (None, _W32), OP_HASH: (None, _W32),
              OP_CA2: (_U8, _U8), OP_CA3: (_U8, _U8), OP_EDM: (("float32",), _W32)}


def _need_bytes(op, m, n, which):
    """Bytes the kernels may touch in buffer `which` (0 in, 1 out)."""
    box = (n + 1) ** m
    if op in (OP_CA2, OP_CA3):
        return box
    if op == OP_EDM and which == 0:
        return 12 * (n + 1)                      # n+1 points in R^3, float32
    return 4 * box


_torch_mod = None


def _torch():
    """torch, imported on first use (the host-only calls do not need it)."""
    global _torch_mod
    if _torch_mod is None:
        import torch
        _torch_mod = torch
    return _torch_mod


def _dtype_name(t):
    return str(t.dtype)[6:]            # "torch.uint8" -> "uint8"


def _check_tensor(t, what, dtypes, nbytes, role, device=True):
    """Raise SimplexMapError(EINVAL) unless t is a contiguous device tensor of
    one of `dtypes` holding at least `nbytes` bytes.  Runs before any call
    into the library, so a wrong buffer never reaches a kernel."""
    _check_layout(t, what, dtypes, nbytes, role)
    if device and not t.is_cuda:
        raise SimplexMapError(EINVAL, what, f"{role} must be a device (cuda) tensor")


def _check_layout(t, what, dtypes, nbytes, role):
    """The type, contiguity and size checks of _check_tensor."""
    if not isinstance(t, _torch().Tensor):
        raise SimplexMapError(EINVAL, what, f"{role} must be a torch tensor, got {type(t).__name__}")
    if _dtype_name(t) not in dtypes:
        raise SimplexMapError(EINVAL, what, f"{role} has dtype {t.dtype}; expected one of {dtypes}")
    if not t.is_contiguous():
        raise SimplexMapError(EINVAL, what, f"{role} must be contiguous")
    have = t.numel() * t.element_size()
    if have < nbytes:
        raise SimplexMapError(EINVAL, what, f"{role} holds {have} bytes; the launch needs {nbytes}")


def _check_op_buffers(what, m, n, op, buf_in, buf_out):
    """Validate the tensors of one launch of `op` over Delta_n^m.  Sizes and
    arguments the library itself rejects (m, n, op) are left to it."""
    op = _op(op)
    if op not in _OP_DTYPES or not isinstance(m, int) or not isinstance(n, int) or m < 2 or m > 4 or n < 0:
        return
    din, dout = _OP_DTYPES[op]
    bufs = [(t, dt, which, role) for t, dt, which, role in
            ((buf_in, din, 0, "buf_in"), (buf_out, dout, 1, "buf_out")) if t is not None and dt is not None]
    for t, dt, which, role in bufs:     # every buffer's type and size first, then the devices
        _check_layout(t, what, dt, _need_bytes(op, m, n, which), role)
    for t, dt, which, role in bufs:
        if not t.is_cuda:
            raise SimplexMapError(EINVAL, what, f"{role} must be a device (cuda) tensor")


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    s = getattr(stream, "cuda_stream", stream)
    return ctypes.c_void_p(int(s) if s else 0)


def map_launch(m, n, op, buf_in=None, buf_out=None, r=0, beta=0, stream=None) -> None:
    """H launch of ``op`` over Delta_n^m on the given (or current) stream."""
    _check_op_buffers("simplex_map_launch", m, n, op, buf_in, buf_out)
    _check(lib().simplex_map_launch(m, n, r, beta, _op(op), _ptr(buf_in), _ptr(buf_out),
                                    _stream(stream)), "simplex_map_launch")


def bb_launch(m, n, op, buf_in=None, buf_out=None, stream=None) -> None:
    """Bounding-box launch of ``op`` over Delta_n^m."""
    _check_op_buffers("simplex_bb_launch", m, n, op, buf_in, buf_out)
    _check(lib().simplex_bb_launch(m, n, _op(op), _ptr(buf_in), _ptr(buf_out), _stream(stream)),
           "simplex_bb_launch")


def map_launch_raw(m, n, r, beta, op, in_ptr, out_ptr, stream_ptr) -> int:
    """Status-returning form with raw integer pointers (for error-path tests)."""
    return lib().simplex_map_launch(m, n, r, beta, _op(op), in_ptr, out_ptr, stream_ptr)


def bb_launch_raw(m, n, op, in_ptr, out_ptr, stream_ptr) -> int:
    return lib().simplex_bb_launch(m, n, _op(op), in_ptr, out_ptr, stream_ptr)


def count(m, n) -> int:
    out = ctypes.c_uint64(0)
    _check(lib().simplex_count(m, n, ctypes.byref(out)), "simplex_count")
    return out.value


def plan_info(m, n, op, use_bb=False, r=0, beta=0) -> dict:
    info = PlanInfo()
    _check(lib().simplex_plan_info(m, n, r, beta, _op(op), 1 if use_bb else 0,
                                   ctypes.byref(info)), "simplex_plan_info")
    return info.as_dict()


def plan_tiles(m, n, op, use_bb=False, r=0, beta=0):
    """(valid, tiles) numpy arrays: one row per launched tile (map unit), in order."""
    import numpy as np
    total = ctypes.c_uint64(0)
    L = lib()
    _check(L.simplex_plan_tiles(m, n, r, beta, _op(op), 1 if use_bb else 0, None, 0,
                                ctypes.byref(total)), "simplex_plan_tiles")
    buf = np.zeros((total.value, 5), dtype=np.int32)
    _check(L.simplex_plan_tiles(m, n, r, beta, _op(op), 1 if use_bb else 0,
                                buf.ctypes.data_as(ctypes.c_void_p), total.value,
                                ctypes.byref(total)), "simplex_plan_tiles")
    return buf[:, 0].astype(bool), buf[:, 1:1 + m]


def set_tile(m, op, rho, wg_threads=0) -> None:
    _check(lib().simplex_set_tile(m, _op(op), rho, wg_threads), "simplex_set_tile")


def set_shape(m, op, rho, wg_threads=0, tiles_per_wg=0) -> None:
    """simplex_set_shape: tile side, threads and tiles per workgroup."""
    _check(lib().simplex_set_shape(m, _op(op), rho, wg_threads, tiles_per_wg), "simplex_set_shape")


def _job_array(jobs, what="simplex_batch_launch"):
    """jobs: iterable of (m, op, n, buf_in, buf_out) with tensors or raw
    pointers (raw pointers are passed as they are; tensors are validated)."""
    def p(x):
        return None if x is None else (x if isinstance(x, int) else x.data_ptr())
    arr = (Job * max(len(jobs), 1))()
    for i, (m, op, n, a, b) in enumerate(jobs):
        if not isinstance(a, int) and not isinstance(b, int):
            _check_op_buffers(what, m, n, op, a, b)
        arr[i] = Job(m, _op(op), n, p(a), p(b))
    return arr


def batch_launch_raw(jobs, njobs=None, stream_ptr=None) -> int:
    """Status-returning batched launch (jobs as for batch_launch)."""
    arr = _job_array(jobs)
    return lib().simplex_batch_launch(arr, len(jobs) if njobs is None else njobs, stream_ptr)


def batch_launch(jobs, stream=None) -> None:
    """One step of every (m, op, n, buf_in, buf_out) job, batched by class."""
    arr = _job_array(jobs)
    _check(lib().simplex_batch_launch(arr, len(jobs), _stream(stream)), "simplex_batch_launch")


def queue_launch_raw(jobs, njobs=None, max_workgroups=0, stream_ptr=None) -> int:
    """Status-returning persistent work-queue launch (jobs as for batch_launch)."""
    arr = _job_array(jobs)
    return lib().simplex_queue_launch(arr, len(jobs) if njobs is None else njobs, max_workgroups, stream_ptr)


def queue_launch(jobs, max_workgroups=0, stream=None) -> None:
    """One step of every (m, op, n, buf_in, buf_out) job in one persistent
    launch that pulls H-mapped block ranges from a device-side work queue."""
    arr = _job_array(jobs, "simplex_queue_launch")
    _check(lib().simplex_queue_launch(arr, len(jobs), max_workgroups, _stream(stream)),
           "simplex_queue_launch")


def queue_launch_static_raw(jobs, njobs=None, max_workgroups=0, stream_ptr=None) -> int:
    """Status-returning simplex_queue_launch_static (jobs as for batch_launch)."""
    arr = _job_array(jobs, "simplex_queue_launch_static")
    return lib().simplex_queue_launch_static(arr, len(jobs) if njobs is None else njobs, max_workgroups,
                                             stream_ptr)


def queue_launch_static(jobs, max_workgroups=0, stream=None) -> None:
    """simplex_queue_launch without allocation: the job table lives in a
    fixed device array of the library (at most 256 jobs)."""
    arr = _job_array(jobs, "simplex_queue_launch_static")
    _check(lib().simplex_queue_launch_static(arr, len(jobs), max_workgroups, _stream(stream)),
           "simplex_queue_launch_static")


def serve_run_raw(jobs, arena_ptr, arena_bytes, mode, max_inflight=4, keep_outputs=False):
    """jobs: list of (m, op, n, buf_in, arrival_s).  Returns (status, records)."""
    def p(x):
        return x if isinstance(x, int) else x.data_ptr()
    arr = (ServeJob * max(len(jobs), 1))()
    for i, (m, op, n, a, t) in enumerate(jobs):
        arr[i] = ServeJob(m, _op(op), n, p(a), float(t))
    recs = (ServeRecord * max(len(jobs), 1))()
    rc = lib().simplex_serve_run(arr, len(jobs), arena_ptr, arena_bytes, mode, max_inflight,
                                 1 if keep_outputs else 0, recs)
    return rc, [dict((f, getattr(recs[i], f)) for f, _ in ServeRecord._fields_)
                for i in range(len(jobs))]


def serve_run(jobs, arena, mode, max_inflight=4, keep_outputs=False):
    """Replay a job stream (see simplex_serve_run); `arena` is a contiguous
    device tensor (its byte size is the memory budget)."""
    what = "simplex_serve_run"
    arena_types = ("uint8", "int8", "int32", "uint32", "float32")
    _check_tensor(arena, what, arena_types, 0, "arena", device=False)
    for (m, op, n, a, _t) in jobs:
        if not isinstance(a, int):
            _check_op_buffers(what, m, n, op, a, None)
    _check_tensor(arena, what, arena_types, 0, "arena")
    rc, recs = serve_run_raw(jobs, arena.data_ptr(), arena.numel() * arena.element_size(), mode,
                             max_inflight, keep_outputs)
    _check(rc, "simplex_serve_run")
    return recs


def autotune_raw(m, n, op, in_ptr, out_ptr, reps=20, cache_path=None, stream_ptr=None):
    """Status-returning autotune; returns (status, result dict)."""
    r = TuneResult()
    rc = lib().simplex_autotune(m, n, _op(op), in_ptr, out_ptr, reps,
                                None if cache_path is None else cache_path.encode(), stream_ptr,
                                ctypes.byref(r))
    return rc, {f: getattr(r, f) for f, _ in TuneResult._fields_}


def autotune(m, n, op, buf_in=None, buf_out=None, reps=20, cache_path=None, stream=None) -> dict:
    """Pick (rho, workgroup size, beta) for H launches of (m, n, op) by timing."""
    _check_op_buffers("simplex_autotune", m, n, op, buf_in, buf_out)
    r = TuneResult()
    _check(lib().simplex_autotune(m, n, _op(op), _ptr(buf_in), _ptr(buf_out), reps,
                                  None if cache_path is None else cache_path.encode(),
                                  _stream(stream), ctypes.byref(r)), "simplex_autotune")
    return {f: getattr(r, f) for f, _ in TuneResult._fields_}


def autotune_reset() -> None:
    _check(lib().simplex_autotune_reset(), "simplex_autotune_reset")


class Graph:
    """A captured run of `steps` H (or BB) launches (simplex_graph_create)."""

    def __init__(self, m, n, op, buf_in=None, buf_out=None, steps=1, r=0, beta=0, use_bb=False):
        self.handle = None
        _check_op_buffers("simplex_graph_create", m, n, op, buf_in, buf_out)
        h = ctypes.c_void_p()
        _check(lib().simplex_graph_create(m, n, r, beta, _op(op), 1 if use_bb else 0, _ptr(buf_in),
                                          _ptr(buf_out), steps, ctypes.byref(h)), "simplex_graph_create")
        self.handle = h

    def launch(self, stream=None) -> None:
        _check(lib().simplex_graph_launch(self.handle, _stream(stream)), "simplex_graph_launch")

    def close(self) -> None:
        if self.handle:
            _check(lib().simplex_graph_destroy(self.handle), "simplex_graph_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class QueueGraph(Graph):
    """One persistent work-queue launch over a fixed job set, captured as a
    graph (simplex_queue_graph_create); replay with launch(), free with close()."""

    def __init__(self, jobs, max_workgroups=0):   # pylint: disable=super-init-not-called
        self.handle = None
        h = ctypes.c_void_p()
        arr = _job_array(jobs, "simplex_queue_graph_create")
        _check(lib().simplex_queue_graph_create(arr, len(jobs), max_workgroups, ctypes.byref(h)),
               "simplex_queue_graph_create")
        self.handle = h


def queue_graph_create_raw(jobs, njobs=None, max_workgroups=0) -> int:
    """Status of simplex_queue_graph_create (the graph, if any, is destroyed)."""
    h = ctypes.c_void_p()
    arr = _job_array(jobs)
    rc = lib().simplex_queue_graph_create(arr, len(jobs) if njobs is None else njobs, max_workgroups,
                                          ctypes.byref(h))
    if rc == OK and h:
        lib().simplex_graph_destroy(h)
    return rc


def map_launch_steps(m, n, op, steps, buf_in, buf_out, r=0, beta=0, stream=None) -> None:
    """`steps` generations with the H map (several per pass; see the header)."""
    _check_op_buffers("simplex_map_launch_steps", m, n, op, buf_in, buf_out)
    _check(lib().simplex_map_launch_steps(m, n, r, beta, _op(op), steps, _ptr(buf_in), _ptr(buf_out),
                                          _stream(stream)), "simplex_map_launch_steps")


def bb_launch_steps(m, n, op, steps, buf_in, buf_out, stream=None) -> None:
    _check_op_buffers("simplex_bb_launch_steps", m, n, op, buf_in, buf_out)
    _check(lib().simplex_bb_launch_steps(m, n, _op(op), steps, _ptr(buf_in), _ptr(buf_out),
                                         _stream(stream)), "simplex_bb_launch_steps")


def launch_steps_raw(m, n, op, steps, in_ptr, out_ptr, use_bb=False) -> int:
    L = lib()
    if use_bb:
        return L.simplex_bb_launch_steps(m, n, _op(op), steps, in_ptr, out_ptr, None)
    return L.simplex_map_launch_steps(m, n, 0, 0, _op(op), steps, in_ptr, out_ptr, None)


def set_general(strategy) -> None:
    """How H launches run their plan's pieces: GENERAL_FUSED (default, one
    launch) or GENERAL_STREAMS (one launch per piece, on streams of their own)."""
    _check(lib().simplex_set_general(strategy), "simplex_set_general")


def set_layout(m, layout) -> None:
    """Native layout of the 3-D H map: LAYOUT_AUTO (default: levels for
    one-job CA3 launches, packed otherwise), LAYOUT_PACKED or LAYOUT_LEVELS."""
    _check(lib().simplex_set_layout(m, layout), "simplex_set_layout")


def copy_launch(m, n, buf_in, buf_out, stream=None) -> None:
    """The simplex-cell copy probe (simplex_copy_launch): uint8 boxes, m = 2, 3."""
    if isinstance(m, int) and isinstance(n, int) and n >= 0:
        for device in (False, True):
            for t, role in ((buf_in, "buf_in"), (buf_out, "buf_out")):
                _check_tensor(t, "simplex_copy_launch", _U8, (n + 1) ** m, role, device)
    _check(lib().simplex_copy_launch(m, n, _ptr(buf_in), _ptr(buf_out), _stream(stream)),
           "simplex_copy_launch")


def copy_launch_raw(m, n, in_ptr, out_ptr, stream_ptr=None) -> int:
    return lib().simplex_copy_launch(m, n, in_ptr, out_ptr, stream_ptr)
