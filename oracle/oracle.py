"""Python face of the CPU oracle (``oracle/simplex_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the ``cpu_baseline`` leg of ``bench.py``; the product package never
imports it and shares no code with it.

The C file holds the plain definitions (Section 1, Eq. 1 for the domain;
Section 5.1, Table tab:tests for the operations).  This wrapper only compiles
it with gcc, loads it with ctypes and marshals numpy arrays.

Arrays use the bounding-box layout: numpy shape ``(n+1,)*m`` in C order with
the LAST numpy axis being x_1, so that ``arr.reshape(-1)[i(x)]`` with
``i(x) = sum_k x_k (n+1)^(k-1)`` is the element x.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "simplex_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

OP_MAP, OP_ACCUM, OP_HITS, OP_HASH, OP_CA2, OP_CA3 = range(6)
OP_NAMES = {"map": OP_MAP, "accum": OP_ACCUM, "hits": OP_HITS, "hash": OP_HASH,
            "ca2": OP_CA2, "ca3": OP_CA3}

_lib = None


def build() -> str:
    """Compile the oracle with gcc into ``oracle/liboracle.so`` (always rebuilds)."""
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-shared", "-fPIC",
                    SRC, "-o", tmp, "-lm"], check=True)
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build()
    lib = ctypes.CDLL(LIB)
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.oracle_apply.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int,
                                 ctypes.c_void_p, ctypes.c_void_p, i64p]
    lib.oracle_apply.restype = ctypes.c_int
    lib.oracle_apply_slab.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int,
                                      ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_int64, ctypes.c_int64, i64p]
    lib.oracle_apply_slab.restype = ctypes.c_int
    lib.oracle_cell.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int,
                                ctypes.c_void_p, i64p]
    lib.oracle_cell.restype = ctypes.c_int64
    lib.oracle_row.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p,
                               i64p, ctypes.c_void_p]
    lib.oracle_row.restype = ctypes.c_int64
    lib.oracle_count.argtypes = [ctypes.c_int, ctypes.c_int64]
    lib.oracle_count.restype = ctypes.c_int64
    u32p = ctypes.POINTER(ctypes.c_uint32)
    lib.oracle_hash32.argtypes = [ctypes.c_int, u32p]
    lib.oracle_hash32.restype = ctypes.c_uint32
    lib.oracle_fnv1a_words.argtypes = [ctypes.c_int, u32p]
    lib.oracle_fnv1a_words.restype = ctypes.c_uint32
    lib.oracle_fmix32.argtypes = [ctypes.c_uint32]
    lib.oracle_fmix32.restype = ctypes.c_uint32
    lib.oracle_edm.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, i64p]
    lib.oracle_edm.restype = ctypes.c_int
    _lib = lib
    return lib


def _op(op) -> int:
    return OP_NAMES[op] if isinstance(op, str) else int(op)


def _ptr(a):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def dtype_of(op) -> np.dtype:
    return np.dtype(np.uint8) if _op(op) in (OP_CA2, OP_CA3) else np.dtype(np.uint32)


def count(m: int, n: int) -> int:
    """Number of elements the oracle's nested loops visit for Delta_n^m."""
    return int(_load().oracle_count(m, n))


def apply(m: int, n: int, op, inp, out) -> int:
    """Apply ``op`` over Delta_n^m in place on ``out`` (numpy box arrays).

    Returns the number of visited elements.  Raises ValueError on bad input.
    """
    code = _op(op)
    for a in (inp, out):
        if a is not None:
            if a.size != (n + 1) ** m or a.dtype != dtype_of(code):
                raise ValueError("buffer shape/dtype does not match the box")
    visited = ctypes.c_int64(0)
    rc = _load().oracle_apply(m, n, code, _ptr(inp), _ptr(out), ctypes.byref(visited))
    if rc != 0:
        raise ValueError(f"oracle_apply rejected arguments (rc={rc})")
    return visited.value


def apply_slab(m: int, n: int, op, inp, out, lo: int, hi: int) -> int:
    """Like :func:`apply` but only for lo <= x_m < hi (a bounded sample)."""
    code = _op(op)
    visited = ctypes.c_int64(0)
    rc = _load().oracle_apply_slab(m, n, code, _ptr(inp), _ptr(out), lo, hi,
                                   ctypes.byref(visited))
    if rc != 0:
        raise ValueError(f"oracle_apply_slab rejected arguments (rc={rc})")
    return visited.value


def cell(m: int, n: int, op, inp, x) -> int:
    """Expected output at element x (x_1 first).  ``inp`` is a full-size box
    array in which at least the cells the definition reads are filled."""
    xa = (ctypes.c_int64 * m)(*[int(v) for v in x])
    return int(_load().oracle_cell(m, n, _op(op), _ptr(inp), xa))


def row(m: int, n: int, op, inp, xhigh) -> np.ndarray:
    """Expected outputs of the row with x_2..x_m = ``xhigh`` (x_1 = 0 ..).

    ``inp`` is a full-size box array in which at least the cells the
    definition reads for this row hold their values (may be None for
    HITS/HASH/MAP)."""
    code = _op(op)
    s = sum(int(v) for v in xhigh)
    if s > n:
        raise ValueError("row outside the simplex")
    buf = np.zeros(n - s + 1, dtype=dtype_of(code))
    xa = (ctypes.c_int64 * (m - 1))(*[int(v) for v in xhigh])
    got = _load().oracle_row(m, n, code, _ptr(inp), xa, _ptr(buf))
    if got != len(buf):
        raise ValueError("oracle_row rejected arguments")
    return buf


def hash32(x) -> int:
    a = (ctypes.c_uint32 * len(x))(*[int(v) for v in x])
    return int(_load().oracle_hash32(len(x), a))


def fnv1a_words(x) -> int:
    a = (ctypes.c_uint32 * len(x))(*[int(v) for v in x])
    return int(_load().oracle_fnv1a_words(len(x), a))


def fmix32(h: int) -> int:
    return int(_load().oracle_fmix32(h & 0xFFFFFFFF))


def edm(n: int, pts) -> np.ndarray:
    """Euclidean distance matrix on Delta_n^2 (see oracle_edm): a float64
    (n+1, n+1) box, NaN outside the simplex.  pts: float32 (n+1, 3)."""
    pts = np.ascontiguousarray(pts, dtype=np.float32)
    assert pts.shape == (n + 1, 3)
    out = np.full((n + 1, n + 1), np.nan, dtype=np.float64)
    visited = ctypes.c_int64(0)
    rc = _load().oracle_edm(n, pts.ctypes.data_as(ctypes.c_void_p), out.ctypes.data_as(ctypes.c_void_p),
                            ctypes.byref(visited))
    if rc != 0:
        raise ValueError(f"oracle_edm failed: {rc}")
    assert visited.value == (n + 1) * (n + 2) // 2
    return out
