"""Seeded synthetic inputs for the scenario-batched Split.

A module of its own, used by both the GPU library's callers and the CPU oracle's tests.
It contains no Split arithmetic: it draws Philox4x32-10 random numbers (see ``gen.c``)
and shapes them into instance coordinates, giant tours and int16 demand matrices laid out
``demand[c - 1, s]`` (customer row, scenario index fastest).

The workload recipes below stand in for the paper's runtime experiment (Section 4.1), which
does not state n, Q or the demand law; the sizes and distributions are the ones this project
measures on.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
# SPLIT_GEN_LIB names another build of gen.c (the sanitizer test's instrumented copy)
_LIB = os.environ.get("SPLIT_GEN_LIB") or os.path.join(_HERE, "libsplitgen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the generator library with gcc (host code only)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64, u64, u32, f64 = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                                   ctypes.c_uint32, ctypes.c_double)
        lib.sg_philox4x32_10.argtypes = [P, P, P]
        lib.sg_philox4x32_10.restype = None
        lib.sg_coords.argtypes = [u64, i32, i32, P]
        lib.sg_tour.argtypes = [u64, u32, i32, i32, P]
        lib.sg_demand_uniform.argtypes = [u64, i32, i64, i64, i32, i32, P, ctypes.c_int]
        lib.sg_demand_poisson.argtypes = [u64, i32, i64, i64, f64, f64, i32, P, P, ctypes.c_int]
        lib.sg_demand_copula.argtypes = [u64, i32, i64, i64, f64, f64, f64, i32, P, ctypes.c_int]
        lib.sg_two_opt_tour.argtypes = [P, i32, i32, P]
        lib.sg_perturb.argtypes = [u64, P, i32, i64, i32, i32, P, ctypes.c_int]
        for f in (lib.sg_coords, lib.sg_tour, lib.sg_demand_uniform, lib.sg_demand_poisson,
                  lib.sg_demand_copula, lib.sg_two_opt_tour, lib.sg_perturb):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _threads(threads):
    if threads is not None:
        return int(threads)
    n = os.cpu_count() or 1
    return max(1, min(16, n))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"{what}: generator returned {rc}")


def philox4x32_10(ctr, key) -> np.ndarray:
    """One Philox4x32-10 block (exposed for known-answer tests)."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _load().sg_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def coords(seed: int, N: int, grid: int = 1000) -> np.ndarray:
    """int32 [(N + 1), 2] integer coordinates uniform on {0..grid-1}^2; row 0 is the depot."""
    xy = np.zeros((N + 1, 2), dtype=np.int32)
    _check(_load().sg_coords(seed, N, grid, _ptr(xy)), "coords")
    return xy


def tour(seed: int, N: int, n: int | None = None, variant: int = 0) -> np.ndarray:
    """Random permutation of customers 1..N (first n entries: a subset tour if n < N)."""
    n = N if n is None else n
    t = np.zeros(n, dtype=np.int32)
    _check(_load().sg_tour(seed, variant, N, n, _ptr(t)), "tour")
    return t


def _alloc(N, S, ld):
    ld = S if ld is None else ld
    return np.zeros((N, ld), dtype=np.int16), ld


def demand_uniform(seed, N, S, lo, hi, ld=None, threads=None) -> np.ndarray:
    dem, ld = _alloc(N, S, ld)
    _check(_load().sg_demand_uniform(seed, N, S, ld, lo, hi, _ptr(dem), _threads(threads)),
           "demand_uniform")
    return dem


def demand_poisson(seed, N, S, lam_lo, lam_hi, Q, ld=None, threads=None, return_lambda=False):
    dem, ld = _alloc(N, S, ld)
    lam = np.zeros(N, dtype=np.float64)
    _check(_load().sg_demand_poisson(seed, N, S, ld, lam_lo, lam_hi, Q, _ptr(dem), _ptr(lam),
                                     _threads(threads)), "demand_poisson")
    return (dem, lam) if return_lambda else dem


def demand_copula(seed, N, S, rho, mean, cv, Q, ld=None, threads=None) -> np.ndarray:
    dem, ld = _alloc(N, S, ld)
    _check(_load().sg_demand_copula(seed, N, S, ld, rho, mean, cv, Q, _ptr(dem),
                                    _threads(threads)), "demand_copula")
    return dem


@dataclass
class Workload:
    name: str
    N: int
    n: int
    S: int
    Q: int
    seed: int
    xy: np.ndarray
    tour: np.ndarray
    demand: np.ndarray  # int16 [N, S]

    def describe(self) -> dict:
        return {"workload": self.name, "n": self.n, "S": self.S, "Q": self.Q, "seed": self.seed}


# name -> (N, S, Q, seed, demand law)
RECIPES = {
    "uniform-n20": dict(N=20, S=1000, Q=100, seed=1, law=("uniform", 1, 20)),
    "poisson-n200": dict(N=200, S=100_000, Q=200, seed=2, law=("poisson", 5.0, 25.0)),
    "copula-n1000": dict(N=1000, S=1 << 20, Q=500, seed=3, law=("copula", 0.6, 20.0, 0.5)),
}


# name -> (instance size N, tours T, tour length range, S, Q, seed, demand law)
BATCH_RECIPES = {
    "batch-256": dict(N=1000, T=256, n_lo=100, n_hi=1000, S=65536, Q=500, seed=4,
                      law=("copula", 0.6, 20.0, 0.5)),
}


@dataclass
class BatchWorkload:
    name: str
    N: int
    S: int
    Q: int
    seed: int
    xy: np.ndarray
    tours: list  # T int32 arrays of distinct customer ids, uneven lengths
    demand: np.ndarray  # int16 [N, S]


def batch_lengths(seed: int, T: int, lo: int, hi: int) -> np.ndarray:
    """T tour lengths uniform on {lo..hi}, drawn from Philox (stream 7 of the seed)."""
    u = np.zeros(T, dtype=np.int32)
    for t in range(T):
        r = philox4x32_10([t, 0, 7, 0], [seed & 0xFFFFFFFF, seed >> 32])
        u[t] = lo + int(r[0]) % (hi - lo + 1)
    return u


def make_batch_workload(name: str, T: int | None = None, S: int | None = None,
                        threads=None) -> BatchWorkload:
    """Candidate tours of uneven length over one instance and one scenario matrix: tour t is
    the first n_t customers of an independent random permutation (a subset tour)."""
    r = BATCH_RECIPES[name]
    N, Q, seed = r["N"], r["Q"], r["seed"]
    T = r["T"] if T is None else int(T)
    S = r["S"] if S is None else int(S)
    xy = coords(seed, N)
    lens = batch_lengths(seed, T, r["n_lo"], r["n_hi"])
    tours = [tour(seed, N, int(lens[t]), variant=t + 1) for t in range(T)]
    law = r["law"]
    dem = demand_copula(seed, N, S, law[1], law[2], law[3], Q, threads=threads)
    return BatchWorkload(name, N, S, Q, seed, xy, tours, dem)


def make_workload(name: str, S: int | None = None, threads=None) -> Workload:
    """Build one of the named synthetic workloads (optionally with fewer scenarios)."""
    r = RECIPES[name]
    N, Q, seed = r["N"], r["Q"], r["seed"]
    S = r["S"] if S is None else int(S)
    xy = coords(seed, N)
    t = tour(seed, N)
    law = r["law"]
    if law[0] == "uniform":
        dem = demand_uniform(seed, N, S, law[1], law[2], threads=threads)
    elif law[0] == "poisson":
        dem = demand_poisson(seed, N, S, law[1], law[2], Q, threads=threads)
    else:
        dem = demand_copula(seed, N, S, law[1], law[2], law[3], Q, threads=threads)
    return Workload(name, N, N, S, Q, seed, xy, t, dem)


def two_opt_tour(xy: np.ndarray, max_passes: int = 200) -> np.ndarray:
    """A short giant tour over all customers: nearest neighbour, then 2-opt on straight-line
    distances (a starting point for perturbed candidates; no Split cost involved)."""
    xy = np.ascontiguousarray(xy, dtype=np.int32)
    N = xy.shape[0] - 1
    t = np.zeros(N, dtype=np.int32)
    _check(_load().sg_two_opt_tour(_ptr(xy), N, int(max_passes), _ptr(t)), "two_opt_tour")
    return t


def perturb(seed: int, base: np.ndarray, count: int, rmin: int, rmax: int,
            threads=None) -> np.ndarray:
    """[count, n] candidates: the base tour with rmin..rmax random segment reversals each."""
    base = np.ascontiguousarray(base, dtype=np.int32)
    out = np.empty((int(count), base.size), dtype=np.int32)
    _check(_load().sg_perturb(seed, _ptr(base), base.size, int(count), int(rmin), int(rmax),
                              _ptr(out), _threads(threads)), "perturb")
    return out


# Screening workload: one 1000-customer instance and 65,536 copula scenarios; a training set
# and a candidate set of randomly 2-opt-perturbed copies of a short base tour (independent
# streams), screened to the top 1%.
SCREEN_RECIPES = {
    "screen": dict(N=1000, S=65536, Q=500, seed=5, law=("copula", 0.6, 20.0, 0.5),
                   train=100_000, candidates=1_000_000, rmin=1, rmax=60, keep=0.01),
}


@dataclass
class ScreenWorkload:
    name: str
    N: int
    S: int
    Q: int
    seed: int
    xy: np.ndarray
    base: np.ndarray
    demand: np.ndarray
    train: np.ndarray  # [train, N] int32
    cands: np.ndarray  # [candidates, N] int32
    keep: int


def make_screen_workload(name: str = "screen", train: int | None = None,
                         candidates: int | None = None, S: int | None = None,
                         threads=None) -> ScreenWorkload:
    r = SCREEN_RECIPES[name]
    N, Q, seed = r["N"], r["Q"], r["seed"]
    S = r["S"] if S is None else int(S)
    ntrain = r["train"] if train is None else int(train)
    ncand = r["candidates"] if candidates is None else int(candidates)
    xy = coords(seed, N)
    base = two_opt_tour(xy)
    law = r["law"]
    dem = demand_copula(seed, N, S, law[1], law[2], law[3], Q, threads=threads)
    tr = perturb(seed * 1000 + 1, base, ntrain, r["rmin"], r["rmax"], threads)
    ca = perturb(seed * 1000 + 2, base, ncand, r["rmin"], r["rmax"], threads)
    keep = max(1, int(round(ncand * r["keep"])))
    return ScreenWorkload(name, N, S, Q, seed, xy, base, dem, tr, ca, keep)
