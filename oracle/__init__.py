"""CPU oracle for the scenario-batched Split -- TEST INFRASTRUCTURE ONLY.

Plain, slow and obviously correct: ``oracle.c`` follows the paper's Eq. (1) (Section 3)
scenario by scenario, plus Eq. (2) masks and Eq. (3) as a cross-check, exact rounded
Euclidean distances and exact sample-average moments. It also holds the linear-time
(monotone-deque) Split, a strong CPU baseline that the benchmark times and the tests check
against Eq. (1). Only ``tests/``,
the smoke check and the benchmark's CPU-baseline leg may import this package.
It imports nothing from the GPU library, and the GPU library imports nothing from it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
# SPLIT_ORACLE_LIB names another build of oracle.c (the sanitizer test's instrumented copy)
_LIB = os.environ.get("SPLIT_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None
_libs = {}

OK, E_INVAL, E_TOUR, E_DEMAND, E_NOMEM = 0, -1, -2, -3, -6


def compile_to(src: str, out: str) -> str:
    """Compile a C source of the oracle into a shared library (gcc, C11, -O2, no fast-math)."""
    tmp = out + ".tmp"
    subprocess.check_call(
        ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-pthread", "-o", tmp, src]
    )
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile the oracle library next to its source."""
    if force or not os.path.exists(_LIB):
        compile_to(_SRC, _LIB)
    return _LIB


def _load(path: str | None = None):
    """Load the oracle library (the default build, or another build of oracle.c at `path`)."""
    global _lib
    if path is not None:
        if path not in _libs:
            _libs[path] = _bind(ctypes.CDLL(path))
        return _libs[path]
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def _bind(lib):
    P = ctypes.c_void_p
    if True:
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        lib.or_isqrt.argtypes = [i64]
        lib.or_isqrt.restype = i64
        lib.or_nint_dist.argtypes = [i64, i64, i64, i64]
        lib.or_nint_dist.restype = i64
        lib.or_dist_from_coords.argtypes = [i32, P, P]
        lib.or_split.argtypes = [P, i32, P, i32, P, i64, i64, i32, P, P, ctypes.c_int]
        lib.or_mask.argtypes = [P, i32, i32, P]
        lib.or_split_masked.argtypes = [P, i32, P, i32, P, P]
        lib.or_moments.argtypes = [P, i64, P, P, P, P, P]
        lib.or_split_deque.argtypes = [P, i32, P, i32, P, i64, i64, i32, P, ctypes.c_int]
        for f in (lib.or_dist_from_coords, lib.or_split, lib.or_mask, lib.or_split_masked,
                  lib.or_moments, lib.or_split_deque):
            f.restype = ctypes.c_int
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: oracle status {status}")
        self.status = status


# Every function below takes `lib=None` (the default build) or the path of another build of
# oracle.c; the tests use the latter to check that deliberately broken copies fail the pins.

def isqrt(m: int, lib=None) -> int:
    return int(_load(lib).or_isqrt(int(m)))


def nint_dist(x1, y1, x2, y2, lib=None) -> int:
    return int(_load(lib).or_nint_dist(int(x1), int(y1), int(x2), int(y2)))


def dist_matrix(xy: np.ndarray, lib=None) -> np.ndarray:
    """(N+1) x (N+1) int32 rounded Euclidean distances from int32 coordinates [(N+1), 2]."""
    xy = np.ascontiguousarray(xy, dtype=np.int32)
    V = xy.shape[0]
    d = np.zeros((V, V), dtype=np.int32)
    rc = _load(lib).or_dist_from_coords(V - 1, _p(xy), _p(d))
    if rc != OK:
        raise OracleError(rc, "dist_matrix")
    return d


def split(tour, d, demand, Q, S=None, threads=1, return_work=False, lib=None):
    """Eq. (1) per scenario. demand: int16 [N, ld] (row c-1 = customer c).

    Returns int32 cost[S] (and the window work sum_i (w_i - 1) if return_work).
    Raises OracleError with the status on invalid input.
    """
    tour = np.ascontiguousarray(tour, dtype=np.int32)
    d = np.ascontiguousarray(d, dtype=np.int32)
    demand = np.asarray(demand)
    if demand.dtype != np.int16 or demand.ndim != 2 or not demand.flags.c_contiguous:
        raise ValueError("demand must be a C-contiguous int16 [N, ld] array")
    N, ld = demand.shape
    S = ld if S is None else int(S)
    if d.shape != (N + 1, N + 1):
        raise ValueError("distance matrix must be (N+1) x (N+1)")
    cost = np.zeros(max(S, 1), dtype=np.int32)
    work = ctypes.c_int64(0)
    rc = _load(lib).or_split(_p(tour), len(tour), _p(d), N, _p(demand), S, ld, int(Q), _p(cost),
                          ctypes.byref(work), int(threads))
    if rc != OK:
        raise OracleError(rc, "split")
    return (cost, int(work.value)) if return_work else cost


def split_deque(tour, d, demand, Q, S=None, threads=1, lib=None):
    """The linear-time Split (monotone deque of predecessors), scenario by scenario: the
    strong CPU baseline for timing. Same arguments, result and errors as split()."""
    tour = np.ascontiguousarray(tour, dtype=np.int32)
    d = np.ascontiguousarray(d, dtype=np.int32)
    demand = np.asarray(demand)
    if demand.dtype != np.int16 or demand.ndim != 2 or not demand.flags.c_contiguous:
        raise ValueError("demand must be a C-contiguous int16 [N, ld] array")
    N, ld = demand.shape
    S = ld if S is None else int(S)
    if d.shape != (N + 1, N + 1):
        raise ValueError("distance matrix must be (N+1) x (N+1)")
    cost = np.zeros(max(S, 1), dtype=np.int32)
    rc = _load(lib).or_split_deque(_p(tour), len(tour), _p(d), N, _p(demand), S, ld, int(Q),
                                   _p(cost), int(threads))
    if rc != OK:
        raise OracleError(rc, "split_deque")
    return cost


def mask(q_pos, Q, lib=None) -> np.ndarray:
    """Eq. (2): mask(i) for i = 1..n from demands in tour-position order (-1 = empty set)."""
    q = np.ascontiguousarray(q_pos, dtype=np.int32)
    out = np.zeros(len(q), dtype=np.int32)
    rc = _load(lib).or_mask(_p(q), len(q), int(Q), _p(out))
    if rc != OK:
        raise OracleError(rc, "mask")
    return out


def split_masked(tour, d, mask_vals, lib=None) -> int:
    """Eq. (3) for one scenario given Eq. (2)'s mask."""
    tour = np.ascontiguousarray(tour, dtype=np.int32)
    d = np.ascontiguousarray(d, dtype=np.int32)
    m = np.ascontiguousarray(mask_vals, dtype=np.int32)
    out = ctypes.c_int64(0)
    rc = _load(lib).or_split_masked(_p(tour), len(tour), _p(d), d.shape[0] - 1, _p(m),
                                 ctypes.byref(out))
    if rc != OK:
        raise OracleError(rc, "split_masked")
    return int(out.value)


def moments(cost, lib=None) -> dict:
    """Exact sum / sum of squares and the mean and sample variance of the costs."""
    c = np.ascontiguousarray(cost, dtype=np.int32)
    s = ctypes.c_int64()
    lo, hi = ctypes.c_uint64(), ctypes.c_uint64()
    mean, var = ctypes.c_double(), ctypes.c_double()
    rc = _load(lib).or_moments(_p(c), len(c), ctypes.byref(s), ctypes.byref(lo), ctypes.byref(hi),
                            ctypes.byref(mean), ctypes.byref(var))
    if rc != OK:
        raise OracleError(rc, "moments")
    return {"sum": int(s.value), "sumsq": (int(hi.value) << 64) | int(lo.value),
            "mean": float(mean.value), "var": float(var.value)}
