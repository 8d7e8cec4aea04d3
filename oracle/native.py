"""ctypes binding of the C oracle ``rng_oracle.c`` (oracle; test infrastructure only).

``build()`` compiles it with gcc/OpenMP into ``oracle/_build/``.  The wrappers
take float32 grid inputs plus the grid exponent q, convert them to exact grid
integers, and return numpy arrays of exact results.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

from .exact import radius_to_grid, to_grid

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rng_oracle.c")
_OUT = os.path.join(_HERE, "_build", "liboracle.so")
_lib = None

_i64p = C.POINTER(C.c_int64)
_i32p = C.POINTER(C.c_int32)


def build(force: bool = True) -> str:
    os.makedirs(os.path.dirname(_OUT), exist_ok=True)
    if force or not os.path.exists(_OUT) or os.path.getmtime(_OUT) < os.path.getmtime(_SRC):
        tmp = _OUT + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wextra", "-o", tmp, _SRC])
        os.replace(tmp, _OUT)
    return _OUT


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_OUT):
            build(force=False)
        L = C.CDLL(_OUT)
        L.oracle_rng_row.restype = C.c_int64
        L.oracle_rng_row.argtypes = [_i32p, C.c_int64, C.c_int32, C.c_int64, _i64p]
        L.oracle_query_row.restype = C.c_int64
        L.oracle_query_row.argtypes = [_i32p, C.c_int64, C.c_int32, _i32p, _i64p]
        L.oracle_rng_rows.restype = C.c_int64
        L.oracle_rng_rows.argtypes = [_i32p, C.c_int64, C.c_int32, _i64p, C.c_int64, C.c_int32, _i64p, _i64p]
        L.oracle_rng_rows_cap.restype = C.c_int64
        L.oracle_rng_rows_cap.argtypes = [_i32p, C.c_int64, C.c_int32, _i64p, C.c_int64, C.c_int32, C.c_int32,
                                          C.c_int64, _i64p, _i64p]
        L.oracle_rng_edges.restype = C.c_int64
        L.oracle_rng_edges.argtypes = [_i32p, C.c_int64, C.c_int32, C.c_int32, C.POINTER(_i64p)]
        L.oracle_grng_edges.restype = C.c_int64
        L.oracle_grng_edges.argtypes = [_i32p, C.c_int64, C.c_int32, _i64p, C.c_int32, C.POINTER(_i64p)]
        L.oracle_sqrt_plus_lt.restype = C.c_int32
        L.oracle_sqrt_plus_lt.argtypes = [C.c_int64, C.c_int64, C.c_int64]
        L.oracle_free.restype = None
        L.oracle_free.argtypes = [C.c_void_p]
        _lib = L
    return _lib


def _ints32(X, q):
    K = to_grid(X, q)
    if K.size and np.abs(K).max() >= 2 ** 24:
        raise ValueError("grid integers must be below 2**24")
    return np.ascontiguousarray(K.astype(np.int32))


def default_threads() -> int:
    """Every host core the process may run on."""
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except (AttributeError, OSError):
        return max(1, os.cpu_count() or 1)


def rng_edges(X, q: int, threads: int | None = None) -> np.ndarray:
    """All RNG edges (u < v) sorted, as int64 [E, 2]."""
    K = _ints32(X, q)
    n, d = K.shape
    p = _i64p()
    e = lib().oracle_rng_edges(K.ctypes.data_as(_i32p), n, d, threads or default_threads(), C.byref(p))
    if e < 0:
        raise MemoryError("oracle_rng_edges failed")
    out = np.ctypeslib.as_array(p, shape=(2 * e,)).copy().reshape(-1, 2) if e else np.zeros((0, 2), np.int64)
    lib().oracle_free(p)
    return out


def rng_row(X, q: int, x: int) -> np.ndarray:
    K = _ints32(X, q)
    n, d = K.shape
    out = np.empty(max(n, 1), dtype=np.int64)
    c = lib().oracle_rng_row(K.ctypes.data_as(_i32p), n, d, int(x), out.ctypes.data_as(_i64p))
    return out[:c].copy()


def rng_rows(X, q: int, xs, threads: int | None = None) -> list:
    """RNG neighbour lists of several points (each sorted ascending)."""
    K = _ints32(X, q)
    n, d = K.shape
    xs = np.ascontiguousarray(np.asarray(xs, dtype=np.int64))
    counts = np.zeros(len(xs), dtype=np.int64)
    out = np.empty(len(xs) * n, dtype=np.int64)
    rc = lib().oracle_rng_rows(K.ctypes.data_as(_i32p), n, d, xs.ctypes.data_as(_i64p), len(xs),
                               threads or default_threads(), counts.ctypes.data_as(_i64p),
                               out.ctypes.data_as(_i64p))
    if rc < 0:
        raise MemoryError("oracle_rng_rows failed")
    return [out[i * n:i * n + counts[i]].copy() for i in range(len(xs))]


def rng_rows_compact(X, q: int, xs, threads: int | None = None, upper: bool = False, cap: int = 1024,
                     K=None) -> list:
    """RNG neighbour lists of the points xs (each sorted ascending), for large N:
    memory is len(xs) * cap ids, and rows with more neighbours are redone with
    a larger cap.  upper=True decides only the neighbours y > x of each row.
    K: the grid integers of X when the caller already has them."""
    K = _ints32(X, q) if K is None else K
    n, d = K.shape
    xs = np.ascontiguousarray(np.asarray(xs, dtype=np.int64))
    out_rows = [None] * len(xs)
    todo = np.arange(len(xs))
    while len(todo):
        sub = np.ascontiguousarray(xs[todo])
        counts = np.zeros(len(sub), dtype=np.int64)
        out = np.empty(len(sub) * cap, dtype=np.int64)
        rc = lib().oracle_rng_rows_cap(K.ctypes.data_as(_i32p), n, d, sub.ctypes.data_as(_i64p), len(sub),
                                       threads or default_threads(), 1 if upper else 0, cap,
                                       counts.ctypes.data_as(_i64p), out.ctypes.data_as(_i64p))
        if rc < 0:
            raise MemoryError("oracle_rng_rows_cap failed")
        over, grow = [], cap
        for j, i in enumerate(todo):
            if counts[j] >= 0:
                out_rows[i] = out[j * cap:j * cap + counts[j]].copy()
            else:
                over.append(i)
                grow = max(grow, int(-counts[j]))
        cap = grow
        todo = np.asarray(over, dtype=np.int64)
    return out_rows


def grid_ints32(X, q: int) -> np.ndarray:
    """The int32 grid integers the C oracle takes (checked against the contract)."""
    return _ints32(X, q)


def query_row(X, q: int, qpt) -> np.ndarray:
    K = _ints32(X, q)
    n, d = K.shape
    Q = _ints32(np.asarray(qpt, dtype=np.float32).reshape(1, -1), q).reshape(-1)
    out = np.empty(max(n, 1), dtype=np.int64)
    c = lib().oracle_query_row(K.ctypes.data_as(_i32p), n, d, Q.ctypes.data_as(_i32p), out.ctypes.data_as(_i64p))
    return out[:c].copy()


def grng_edges(Xp, radii, q: int, threads: int | None = None) -> np.ndarray:
    """GRNG edges (i < j, indices into Xp) for pivot coordinates Xp with radii."""
    K = _ints32(Xp, q)
    m, d = K.shape
    R = np.ascontiguousarray(radius_to_grid(radii, q).astype(np.int64))
    p = _i64p()
    e = lib().oracle_grng_edges(K.ctypes.data_as(_i32p), m, d, R.ctypes.data_as(_i64p),
                                threads or default_threads(), C.byref(p))
    if e < 0:
        raise MemoryError("oracle_grng_edges failed")
    out = np.ctypeslib.as_array(p, shape=(2 * e,)).copy().reshape(-1, 2) if e else np.zeros((0, 2), np.int64)
    lib().oracle_free(p)
    return out


def sqrt_plus_lt(a: int, c: int, b: int) -> bool:
    return bool(lib().oracle_sqrt_plus_lt(int(a), int(c), int(b)))
