"""MI355X-native scenario-batched Split (arXiv 2511.18022, Section 3).

Thin ctypes binding of ``libsplitgpu.so`` (C ABI in ``include/split.h``). It only marshals
arguments: every step of the evaluation runs in the library's HIP kernels. PyTorch supplies
device memory (``torch.Tensor.data_ptr``) and the stream. There is no CPU fallback: if the
library is not built, or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsplitgpu.so")

SPLIT_OK, SPLIT_E_INVAL, SPLIT_E_TOUR, SPLIT_E_DEMAND = 0, -1, -2, -3
SPLIT_E_RANGE, SPLIT_E_HIP, SPLIT_E_NOMEM = -4, -5, -6
SPLIT_MAX_N = 8192  # largest instance (customers) the library accepts
FORM_AUTO, FORM_LANE, FORM_WAVE, FORM_MASK = 0, 1, 2, 3
FORMS = {"auto": FORM_AUTO, "lane": FORM_LANE, "wave": FORM_WAVE, "mask": FORM_MASK}
STATUS_NAMES = {0: "SPLIT_OK", -1: "SPLIT_E_INVAL", -2: "SPLIT_E_TOUR", -3: "SPLIT_E_DEMAND",
                -4: "SPLIT_E_RANGE", -5: "SPLIT_E_HIP", -6: "SPLIT_E_NOMEM"}

# Every function declared in include/split.h.
EXPORTED = [
    "split_ctx_create", "split_ctx_destroy", "split_last_error", "split_instance_set_coords",
    "split_instance_set_dist", "split_eval", "split_eval_noalloc", "split_stats_get",
    "split_eval_batch",
    "split_batch_stats_get", "split_set_form", "split_timing_enable", "split_timing_get",
    "split_timing_reset", "split_timing_samples", "split_tuning_set", "split_tuning_get",
    "split_autotune", "split_graph_create", "split_graph_launch", "split_graph_stats", "split_graph_destroy",
    # include/split_nn.h
    "split_nn_create", "split_nn_destroy", "split_nn_params_get", "split_nn_params_set",
    "split_nn_set_norm", "split_nn_set_scenarios", "split_nn_predict", "split_nn_gradient",
    "split_nn_train_step", "split_nn_train", "split_nn_step", "split_nn_save", "split_nn_load",
    "split_topk_smallest", "split_nn_shortlist", "split_nn_screen", "split_nn_timing_enable",
    "split_nn_timing_get", "split_nn_timing_reset",
    # include/split_search.h
    "split_search",
]
NN_PARAMS = 283393
VOID_FUNCS = ("split_ctx_destroy", "split_last_error", "split_graph_destroy", "split_nn_destroy")


class SplitError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class SplitStatsC(ctypes.Structure):
    _fields_ = [("sum", ctypes.c_int64), ("sumsq_lo", ctypes.c_uint64),
                ("sumsq_hi", ctypes.c_uint64), ("mean", ctypes.c_double),
                ("var", ctypes.c_double), ("n_fallback", ctypes.c_int64)]


class SplitTuningC(ctypes.Structure):
    _fields_ = [("form", ctypes.c_int32), ("lane_per_cu", ctypes.c_int32),
                ("order", ctypes.c_int32), ("wave_grid", ctypes.c_int32),
                ("lane_block", ctypes.c_int32)]


@dataclass
class SplitTuning:
    """Launch choices (split_tuning): none changes a result."""
    form: int = FORM_AUTO
    lane_per_cu: int = 0
    order: int = 0
    wave_grid: int = 0
    lane_block: int = 0

    def to_c(self) -> SplitTuningC:
        return SplitTuningC(self.form, self.lane_per_cu, self.order, self.wave_grid,
                            self.lane_block)

    @staticmethod
    def from_c(c: SplitTuningC) -> "SplitTuning":
        return SplitTuning(int(c.form), int(c.lane_per_cu), int(c.order), int(c.wave_grid),
                           int(c.lane_block))


class SplitSearchResultC(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("evaluated", ctypes.c_int64),
                ("predicted", ctypes.c_int64), ("improvements", ctypes.c_int64),
                ("start_mean", ctypes.c_double), ("best_mean", ctypes.c_double),
                ("seconds", ctypes.c_double)]


@dataclass
class SplitStats:
    sum: int
    sumsq: int
    mean: float
    var: float
    n_fallback: int


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libsplitgpu.so and declare its C signatures (no GPU needed to load)."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build it with `python -m paper_2511_18022_amd._build` "
            "(hipcc, gfx950); there is no CPU fallback")
    # torch carries its own HIP runtime under the soname this library links against. Loaded
    # first, it is the one the library binds to; loaded after the library, it would be a second
    # runtime in the process, and device calls would fail in one of the two.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.split_ctx_create.argtypes = [ctypes.c_int, ctypes.POINTER(P)]
    lib.split_ctx_destroy.argtypes = [P]
    lib.split_ctx_destroy.restype = None
    lib.split_last_error.argtypes = [P]
    lib.split_last_error.restype = ctypes.c_char_p
    lib.split_instance_set_coords.argtypes = [P, i32, P]
    lib.split_instance_set_dist.argtypes = [P, i32, P]
    lib.split_eval.argtypes = [P, P, i32, P, i64, i64, i32, P, P, P]
    lib.split_eval_noalloc.argtypes = [P, P, i32, P, i64, i64, i32, P, P, P]
    lib.split_stats_get.argtypes = [P, ctypes.POINTER(SplitStatsC)]
    lib.split_eval_batch.argtypes = [P, P, P, i32, P, i64, i64, i32, P, i64, P, P, P]
    lib.split_batch_stats_get.argtypes = [P, P, P]
    lib.split_set_form.argtypes = [P, ctypes.c_int]
    lib.split_timing_enable.argtypes = [P, ctypes.c_int]
    lib.split_timing_get.argtypes = [P, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(ctypes.c_char_p)]
    lib.split_timing_reset.argtypes = [P]
    lib.split_timing_samples.argtypes = [P, P, i64, ctypes.POINTER(i64)]
    lib.split_tuning_set.argtypes = [P, ctypes.POINTER(SplitTuningC)]
    lib.split_tuning_get.argtypes = [P, ctypes.POINTER(SplitTuningC)]
    lib.split_autotune.argtypes = [P, P, P, i32, P, i64, i64, i32, P, i64, i32, P,
                                   ctypes.POINTER(SplitTuningC), ctypes.POINTER(ctypes.c_double)]
    lib.split_graph_create.argtypes = [P, i32, i64, P, i64, i64, i32, P, i64, ctypes.POINTER(P)]
    lib.split_graph_launch.argtypes = [P, P, P, i32, P]
    lib.split_graph_stats.argtypes = [P, P, P]
    lib.split_graph_destroy.argtypes = [P]
    lib.split_graph_destroy.restype = None
    u64, f32, f64 = ctypes.c_uint64, ctypes.c_float, ctypes.c_double
    lib.split_nn_create.argtypes = [P, u64, f64, ctypes.POINTER(P)]
    lib.split_nn_destroy.argtypes = [P]
    lib.split_nn_destroy.restype = None
    lib.split_nn_params_get.argtypes = [P, P]
    lib.split_nn_params_set.argtypes = [P, P]
    lib.split_nn_set_norm.argtypes = [P, f64, f64]
    lib.split_nn_set_scenarios.argtypes = [P, P, i64, i64, i32]
    lib.split_nn_predict.argtypes = [P, P, i32, i32, P, P]
    lib.split_nn_gradient.argtypes = [P, P, P, i32, i32, P, ctypes.POINTER(f64), P]
    lib.split_nn_train_step.argtypes = [P, P, P, i32, i32, f32, ctypes.POINTER(f64), P]
    lib.split_nn_train.argtypes = [P, P, P, i64, i32, i32, i64, f32, u64, ctypes.POINTER(f64), P]
    lib.split_nn_step.argtypes = [P, ctypes.POINTER(i64)]
    lib.split_nn_save.argtypes = [P, ctypes.c_char_p]
    lib.split_nn_load.argtypes = [P, ctypes.c_char_p]
    lib.split_topk_smallest.argtypes = [P, P, i64, i64, P, P]
    lib.split_nn_shortlist.argtypes = [P, P, i32, i32, i32, P, P, P]
    lib.split_nn_timing_enable.argtypes = [P, ctypes.c_int]
    lib.split_nn_timing_get.argtypes = [P, ctypes.POINTER(f64), ctypes.POINTER(i64)]
    lib.split_nn_timing_reset.argtypes = [P]
    lib.split_search.argtypes = [P, P, P, i32, P, i64, i64, i32, i32, i32, f64, i64, u64, P, P,
                                 P, i32, P, P, P]
    lib.split_nn_screen.argtypes = [P, P, i64, i32, i64, P, i64, i64, i32, P, P, P,
                                    ctypes.POINTER(i64), ctypes.POINTER(f64), P]
    for name in EXPORTED:
        fn = getattr(lib, name)
        if name not in VOID_FUNCS:
            fn.restype = ctypes.c_int
    if path == LIB_PATH:
        _lib = lib
    return lib


def _np():
    import numpy as np
    return np


def _pack_tours(tours):
    """Concatenated int32 tours and their int64 offsets [T + 1]."""
    np = _np()
    parts = [np.ascontiguousarray(t, dtype=np.int32).ravel() for t in tours]
    T = len(parts)
    if T < 1:
        raise ValueError("need at least one tour")
    ptr = np.zeros(T + 1, dtype=np.int64)
    ptr[1:] = np.cumsum([p.size for p in parts])
    flat = np.ascontiguousarray(np.concatenate(parts))
    return flat, ptr, T


def _demand_shape(demand, S, flat, N):
    """(ld, S) of a CUDA int16 demand tensor [rows, ld], checked against the tours' ids."""
    import torch
    if not (isinstance(demand, torch.Tensor) and demand.is_cuda and
            demand.dtype == torch.int16 and demand.dim() == 2 and demand.stride(1) == 1):
        raise ValueError("demand must be a CUDA int16 tensor [N, ld] with unit column stride")
    ld = demand.stride(0)
    S = demand.shape[1] if S is None else int(S)
    if S > demand.shape[1]:
        raise ValueError(f"S={S} exceeds the demand tensor's {demand.shape[1]} columns")
    # ids above N are the library's to reject (SPLIT_E_TOUR)
    if flat is not None and flat.size and demand.shape[0] < int(flat.max()) <= N:
        raise ValueError("the demand tensor has fewer rows than the largest tour customer id")
    return ld, S


def _cost_matrix(cost, T, S, device):
    import torch
    if cost is None:
        return torch.empty((T, max(S, 1)), dtype=torch.int32, device=device)
    if not (cost.is_cuda and cost.dtype == torch.int32 and cost.dim() == 2 and
            cost.shape[0] >= T and cost.shape[1] >= S and cost.stride(1) == 1):
        raise ValueError("cost must be a CUDA int32 tensor [>= T, >= S] with unit column stride")
    return cost


class SplitContext:
    """One library context (device buffers, instance, timing) bound to a HIP device."""

    def __init__(self, device: int = 0):
        self._lib = load_library()
        h = ctypes.c_void_p()
        st = self._lib.split_ctx_create(int(device), ctypes.byref(h))
        if st != SPLIT_OK:
            raise SplitError(st, f"split_ctx_create(device={device}) failed")
        self._h = h
        self.device = device
        self.N = 0

    def close(self):
        if getattr(self, "_h", None):
            self._lib.split_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, st: int):
        if st != SPLIT_OK:
            msg = self._lib.split_last_error(self._h)
            raise SplitError(st, msg.decode() if msg else "")

    # -- instance
    def set_coords(self, xy):
        np = _np()
        a = np.ascontiguousarray(xy, dtype=np.int32)
        if a.ndim != 2 or a.shape[1] != 2:
            raise ValueError("xy must be [(N+1), 2]")
        self._check(self._lib.split_instance_set_coords(self._h, a.shape[0] - 1,
                                                        a.ctypes.data_as(ctypes.c_void_p)))
        self.N = a.shape[0] - 1

    def set_dist(self, d):
        np = _np()
        a = np.ascontiguousarray(d, dtype=np.int32)
        if a.ndim != 2 or a.shape[0] != a.shape[1]:
            raise ValueError("d must be square [(N+1), (N+1)]")
        self._check(self._lib.split_instance_set_dist(self._h, a.shape[0] - 1,
                                                      a.ctypes.data_as(ctypes.c_void_p)))
        self.N = a.shape[0] - 1

    def set_form(self, form):
        self._check(self._lib.split_set_form(self._h, FORMS.get(form, form)))

    # -- evaluation
    def eval(self, tour, demand, Q: int, S: int | None = None, cost=None, sync: bool = True,
             stream=None):
        """Split `tour` under every scenario of `demand` (torch.int16 CUDA tensor [N, ld]).

        Returns (cost, SplitStats) when sync, else (cost, None) with the work enqueued.
        """
        import torch
        np = _np()
        t = np.ascontiguousarray(tour, dtype=np.int32)
        ld, S = _demand_shape(demand, S, t, self.N)
        if cost is None:
            cost = torch.empty(max(S, 1), dtype=torch.int32, device=demand.device)
        elif not (cost.is_cuda and cost.dtype == torch.int32 and cost.is_contiguous() and
                  cost.numel() >= S):
            raise ValueError("cost must be a contiguous CUDA int32 tensor with >= S elements")
        if stream is None:
            stream = torch.cuda.current_stream(demand.device)
        sh = ctypes.c_void_p(stream.cuda_stream)
        out = SplitStatsC()
        self._last_T = 1
        st = self._lib.split_eval(self._h, t.ctypes.data_as(ctypes.c_void_p), len(t),
                                  ctypes.c_void_p(demand.data_ptr()), S, ld, int(Q),
                                  ctypes.c_void_p(cost.data_ptr()),
                                  ctypes.byref(out) if sync else None, sh)
        self._check(st)
        return cost, (self._stats(out) if sync else None)

    def eval_noalloc(self, tour, demand, Q: int, cost, S: int | None = None, sync: bool = True,
                     stream=None):
        """split_eval_noalloc: split_eval with every per-call device buffer taken from the GPU's
        fixed scratch (no allocation on the device). `cost` is the caller's contiguous CUDA
        int32 tensor of >= S elements. Returns the SplitStats when sync, else None."""
        import torch
        np = _np()
        t = np.ascontiguousarray(tour, dtype=np.int32)
        ld, S = _demand_shape(demand, S, t, self.N)
        if not (cost.is_cuda and cost.dtype == torch.int32 and cost.is_contiguous() and
                cost.numel() >= S):
            raise ValueError("cost must be a contiguous CUDA int32 tensor with >= S elements")
        if stream is None:
            stream = torch.cuda.current_stream(demand.device)
        out = SplitStatsC()
        st = self._lib.split_eval_noalloc(self._h, t.ctypes.data_as(ctypes.c_void_p), len(t),
                                          ctypes.c_void_p(demand.data_ptr()), S, ld, int(Q),
                                          ctypes.c_void_p(cost.data_ptr()),
                                          ctypes.byref(out) if sync else None,
                                          ctypes.c_void_p(stream.cuda_stream))
        self._check(st)
        return self._stats(out) if sync else None

    def eval_batch(self, tours, demand, Q: int, S: int | None = None, cost=None,
                   sync: bool = True, stream=None):
        """Split every tour of `tours` (a sequence of customer-id arrays of uneven length) under
        every scenario of `demand` (torch.int16 CUDA tensor [N, ld]) in one launch sequence.

        Returns (cost [T, S] int32 CUDA tensor, [SplitStats] * T, [status] * T) when sync, else
        (cost, None, None) with the work enqueued. A tour with an infeasible demand raises
        SplitError(SPLIT_E_DEMAND) when sync; batch_stats() then still gives every tour's result.
        """
        import torch
        np = _np()
        flat, ptr, T = _pack_tours(tours)
        ld, S = _demand_shape(demand, S, flat, self.N)
        cost = _cost_matrix(cost, T, S, demand.device)
        if stream is None:
            stream = torch.cuda.current_stream(demand.device)
        sh = ctypes.c_void_p(stream.cuda_stream)
        outs = (SplitStatsC * T)()
        status = np.zeros(T, dtype=np.int32)
        st = self._lib.split_eval_batch(
            self._h, flat.ctypes.data_as(ctypes.c_void_p), ptr.ctypes.data_as(ctypes.c_void_p),
            T, ctypes.c_void_p(demand.data_ptr()), S, ld, int(Q), ctypes.c_void_p(cost.data_ptr()),
            cost.stride(0), ctypes.cast(outs, ctypes.c_void_p) if sync else None,
            status.ctypes.data_as(ctypes.c_void_p) if sync else None, sh)
        self._last_T = T
        self._check(st)
        if not sync:
            return cost, None, None
        return cost, [self._stats(o) for o in outs], [int(x) for x in status]

    # -- launch choices
    def tuning(self) -> SplitTuning:
        c = SplitTuningC()
        self._check(self._lib.split_tuning_get(self._h, ctypes.byref(c)))
        return SplitTuning.from_c(c)

    def set_tuning(self, tuning: SplitTuning):
        c = tuning.to_c()
        self._check(self._lib.split_tuning_set(self._h, ctypes.byref(c)))

    def autotune(self, tours, demand, Q: int, S: int | None = None, cost=None, reps: int = 3,
                 stream=None):
        """Time the candidate launch choices on this batch, install the fastest and return
        (SplitTuning, mean ms of one evaluation, cost [T, S] of the batch under it)."""
        import torch
        flat, ptr, T = _pack_tours(tours)
        ld, S = _demand_shape(demand, S, flat, self.N)
        cost = _cost_matrix(cost, T, S, demand.device)
        if stream is None:
            stream = torch.cuda.current_stream(demand.device)
        best = SplitTuningC()
        ms = ctypes.c_double()
        self._last_T = T
        self._check(self._lib.split_autotune(
            self._h, flat.ctypes.data_as(ctypes.c_void_p), ptr.ctypes.data_as(ctypes.c_void_p),
            T, ctypes.c_void_p(demand.data_ptr()), S, ld, int(Q), ctypes.c_void_p(cost.data_ptr()),
            cost.stride(0), int(reps), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(best),
            ctypes.byref(ms)))
        return SplitTuning.from_c(best), float(ms.value), cost

    def graph(self, max_T: int, max_total_n: int, demand, Q: int, S: int | None = None,
              cost=None) -> "SplitGraph":
        """Capture the evaluation of batches of up to max_T tours and max_total_n positions
        against `demand` into a HIP graph (see SplitGraph)."""
        return SplitGraph(self, max_T, max_total_n, demand, Q, S, cost)

    def batch_stats(self):
        """Statistics and per-tour status of the latest evaluation (waits for it)."""
        np = _np()
        T = getattr(self, "_last_T", 1)
        outs = (SplitStatsC * T)()
        status = np.zeros(T, dtype=np.int32)
        st = self._lib.split_batch_stats_get(self._h, ctypes.cast(outs, ctypes.c_void_p),
                                             status.ctypes.data_as(ctypes.c_void_p))
        if st not in (SPLIT_OK, SPLIT_E_DEMAND):
            self._check(st)
        return [self._stats(o) for o in outs], [int(x) for x in status]

    def stats(self) -> SplitStats:
        out = SplitStatsC()
        self._check(self._lib.split_stats_get(self._h, ctypes.byref(out)))
        return self._stats(out)

    @staticmethod
    def _stats(c: SplitStatsC) -> SplitStats:
        return SplitStats(sum=int(c.sum), sumsq=(int(c.sumsq_hi) << 64) | int(c.sumsq_lo),
                          mean=float(c.mean), var=float(c.var), n_fallback=int(c.n_fallback))

    # -- timing of the dominant kernel
    def timing(self, enable: bool = True):
        self._check(self._lib.split_timing_enable(self._h, 1 if enable else 0))

    def timing_reset(self):
        self._check(self._lib.split_timing_reset(self._h))

    def timing_samples(self):
        """Durations (ms) of every timed launch since the last reset, in order."""
        np = _np()
        n = ctypes.c_int64()
        self._check(self._lib.split_timing_samples(self._h, None, 0, ctypes.byref(n)))
        out = np.zeros(n.value, dtype=np.float32)
        if n.value:
            self._check(self._lib.split_timing_samples(
                self._h, ctypes.c_void_p(out.ctypes.data), n.value, ctypes.byref(n)))
        return out

    def timing_get(self):
        ms, n = ctypes.c_double(), ctypes.c_int64()
        name = ctypes.c_char_p()
        self._check(self._lib.split_timing_get(self._h, ctypes.byref(ms), ctypes.byref(n),
                                               ctypes.byref(name)))
        return float(ms.value), int(n.value), (name.value.decode() if name.value else "")


class SplitGraph:
    """A captured evaluation (split_graph_*): fixed demand, cost, S, Q, instance and launch
    choices; each launch stages new tours and replays one HIP graph. The demand tensor must
    hold a row for every customer 1..N. Keep the SplitContext alive while the graph is."""

    def __init__(self, ctx: SplitContext, max_T: int, max_total_n: int, demand, Q: int,
                 S: int | None = None, cost=None):
        self._ctx = ctx
        self._lib = ctx._lib
        ld, S = _demand_shape(demand, S, None, ctx.N)
        if demand.shape[0] < ctx.N:
            raise ValueError("the demand tensor needs a row for every customer 1..N")
        self.cost = _cost_matrix(cost, max_T, S, demand.device)
        self.demand = demand  # the graph reads it at every launch: keep it alive
        self.S, self.Q, self.max_T = S, int(Q), int(max_T)
        self._T = 0
        h = ctypes.c_void_p()
        ctx._check(self._lib.split_graph_create(
            ctx._h, int(max_T), int(max_total_n), ctypes.c_void_p(demand.data_ptr()), S, ld,
            int(Q), ctypes.c_void_p(self.cost.data_ptr()), self.cost.stride(0), ctypes.byref(h)))
        self._h = h

    def launch(self, tours, stream=None):
        """Stage `tours` and replay the graph on `stream` (default: the current stream).
        Returns the cost tensor (rows 0..T-1 are this batch's once the stream reaches them)."""
        import torch
        flat, ptr, T = _pack_tours(tours)
        if stream is None:
            stream = torch.cuda.current_stream(self.cost.device)
        self._ctx._check(self._lib.split_graph_launch(
            self._h, flat.ctypes.data_as(ctypes.c_void_p), ptr.ctypes.data_as(ctypes.c_void_p),
            T, ctypes.c_void_p(stream.cuda_stream)))
        self._T = T
        return self.cost

    def stats(self):
        """([SplitStats] * T, [status] * T) of the latest launch (waits for it)."""
        np = _np()
        T = max(self._T, 1)
        outs = (SplitStatsC * T)()
        status = np.zeros(T, dtype=np.int32)
        st = self._lib.split_graph_stats(self._h, ctypes.cast(outs, ctypes.c_void_p),
                                         status.ctypes.data_as(ctypes.c_void_p))
        if st not in (SPLIT_OK, SPLIT_E_DEMAND):
            self._ctx._check(st)
        return [SplitContext._stats(o) for o in outs], [int(x) for x in status]

    def close(self):
        if getattr(self, "_h", None):
            self._lib.split_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def _cuda_i32_matrix(tours):
    import torch
    if not (isinstance(tours, torch.Tensor) and tours.is_cuda and tours.dtype == torch.int32 and
            tours.dim() == 2 and tours.is_contiguous()):
        raise ValueError("tours must be a contiguous CUDA int32 tensor [T, n]")
    return tours.shape[0], tours.shape[1]


def _cuda_f32_vector(x, T, what):
    import torch
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float32 and
            x.is_contiguous() and x.numel() >= T):
        raise ValueError(f"{what} must be a contiguous CUDA float32 tensor with >= {T} values")


class SplitNN:
    """The tour-encoder surrogate (include/split_nn.h) on a SplitContext's device and instance.
    Tours are CUDA int32 tensors [T, n]; labels are expected costs (CUDA float32 [T])."""

    def __init__(self, ctx: SplitContext, seed: int = 0, length_scale: float = 1000.0):
        self._ctx = ctx
        self._lib = ctx._lib
        h = ctypes.c_void_p()
        ctx._check(self._lib.split_nn_create(ctx._h, int(seed), float(length_scale),
                                             ctypes.byref(h)))
        self._h = h

    def _check(self, st):
        self._ctx._check(st)

    @staticmethod
    def _stream(stream, device):
        import torch
        s = torch.cuda.current_stream(device) if stream is None else stream
        return ctypes.c_void_p(s.cuda_stream)

    def params(self):
        np = _np()
        out = np.zeros(NN_PARAMS, dtype=np.float32)
        self._check(self._lib.split_nn_params_get(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def set_params(self, params):
        np = _np()
        a = np.ascontiguousarray(params, dtype=np.float32)
        if a.size != NN_PARAMS:
            raise ValueError(f"need {NN_PARAMS} parameters")
        self._check(self._lib.split_nn_params_set(self._h, a.ctypes.data_as(ctypes.c_void_p)))

    def set_norm(self, shift: float, scale: float):
        self._check(self._lib.split_nn_set_norm(self._h, float(shift), float(scale)))

    def set_scenarios(self, demand, Q: int, S: int | None = None):
        ld, S = _demand_shape(demand, S, None, self._ctx.N)
        if demand.shape[0] < self._ctx.N:
            raise ValueError("the demand tensor needs a row for every customer 1..N")
        self._check(self._lib.split_nn_set_scenarios(self._h, ctypes.c_void_p(demand.data_ptr()),
                                                     S, ld, int(Q)))

    def predict(self, tours, out=None, stream=None):
        import torch
        T, n = _cuda_i32_matrix(tours)
        if out is None:
            out = torch.empty(T, dtype=torch.float32, device=tours.device)
        _cuda_f32_vector(out, T, "out")
        self._check(self._lib.split_nn_predict(self._h, ctypes.c_void_p(tours.data_ptr()), T, n,
                                               ctypes.c_void_p(out.data_ptr()),
                                               self._stream(stream, tours.device)))
        return out

    def gradient(self, tours, labels, stream=None):
        np = _np()
        T, n = _cuda_i32_matrix(tours)
        _cuda_f32_vector(labels, T, "labels")
        g = np.zeros(NN_PARAMS, dtype=np.float32)
        loss = ctypes.c_double()
        self._check(self._lib.split_nn_gradient(
            self._h, ctypes.c_void_p(tours.data_ptr()), ctypes.c_void_p(labels.data_ptr()), T, n,
            g.ctypes.data_as(ctypes.c_void_p), ctypes.byref(loss),
            self._stream(stream, tours.device)))
        return g, float(loss.value)

    def train_step(self, tours, labels, lr: float, stream=None) -> float:
        T, n = _cuda_i32_matrix(tours)
        _cuda_f32_vector(labels, T, "labels")
        loss = ctypes.c_double()
        self._check(self._lib.split_nn_train_step(
            self._h, ctypes.c_void_p(tours.data_ptr()), ctypes.c_void_p(labels.data_ptr()), T, n,
            float(lr), ctypes.byref(loss), self._stream(stream, tours.device)))
        return float(loss.value)

    def train(self, tours, labels, batch: int, steps: int, lr: float, seed: int = 0,
              stream=None) -> float:
        """`steps` Adam steps over the training set; returns the mean batch loss."""
        count, n = _cuda_i32_matrix(tours)
        _cuda_f32_vector(labels, count, "labels")
        loss = ctypes.c_double()
        self._check(self._lib.split_nn_train(
            self._h, ctypes.c_void_p(tours.data_ptr()), ctypes.c_void_p(labels.data_ptr()), count,
            n, int(batch), int(steps), float(lr), int(seed), ctypes.byref(loss),
            self._stream(stream, tours.device)))
        return float(loss.value)

    @property
    def step(self) -> int:
        s = ctypes.c_int64()
        self._check(self._lib.split_nn_step(self._h, ctypes.byref(s)))
        return int(s.value)

    def timing(self, enable: bool = True):
        """Time the fused convolution kernel of every prediction with HIP events."""
        self._check(self._lib.split_nn_timing_enable(self._h, 1 if enable else 0))

    def timing_reset(self):
        self._check(self._lib.split_nn_timing_reset(self._h))

    def timing_get(self):
        """(milliseconds, launches) of the timed fused-kernel launches since the last reset."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        self._check(self._lib.split_nn_timing_get(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return float(ms.value), int(n.value)

    def save(self, path: str):
        self._check(self._lib.split_nn_save(self._h, os.fsencode(path)))

    def load(self, path: str):
        self._check(self._lib.split_nn_load(self._h, os.fsencode(path)))

    def shortlist(self, tours, K: int, pred=None, stream=None):
        """Indices (CUDA int32 [K], increasing) of the K tours with the lowest predictions."""
        import torch
        T, n = _cuda_i32_matrix(tours)
        idx = torch.empty(int(K), dtype=torch.int32, device=tours.device)
        if pred is not None:
            _cuda_f32_vector(pred, T, "pred")
        self._check(self._lib.split_nn_shortlist(
            self._h, ctypes.c_void_p(tours.data_ptr()), T, n, int(K),
            ctypes.c_void_p(idx.data_ptr()),
            ctypes.c_void_p(pred.data_ptr()) if pred is not None else None,
            self._stream(stream, tours.device)))
        return idx

    def screen(self, cands, K: int, demand, Q: int, S: int | None = None, pred=None,
               stream=None):
        """Predict every candidate, evaluate the K best predictions exactly, return a dict with
        best_idx, best_mean, short_idx [K], short_mean [K] and pred [C]."""
        import torch
        np = _np()
        C, n = _cuda_i32_matrix(cands)
        ld, S = _demand_shape(demand, S, None, self._ctx.N)
        if pred is None:
            pred = torch.empty(C, dtype=torch.float32, device=cands.device)
        _cuda_f32_vector(pred, C, "pred")
        sidx = np.zeros(K, dtype=np.int32)
        smean = np.zeros(K, dtype=np.float64)
        bi, bm = ctypes.c_int64(), ctypes.c_double()
        self._check(self._lib.split_nn_screen(
            self._h, ctypes.c_void_p(cands.data_ptr()), C, n, int(K),
            ctypes.c_void_p(demand.data_ptr()), S, ld, int(Q), ctypes.c_void_p(pred.data_ptr()),
            sidx.ctypes.data_as(ctypes.c_void_p), smean.ctypes.data_as(ctypes.c_void_p),
            ctypes.byref(bi), ctypes.byref(bm), self._stream(stream, cands.device)))
        return {"best_idx": int(bi.value), "best_mean": float(bm.value), "short_idx": sidx,
                "short_mean": smean, "pred": pred}

    def close(self):
        if getattr(self, "_h", None):
            self._lib.split_nn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def topk_smallest(ctx: SplitContext, scores, K: int, stream=None):
    """Indices (CUDA int32 [K], increasing) of the K smallest scores (CUDA float32 [C]); ties at
    the threshold go to the lower indices."""
    import torch
    C = scores.numel()
    _cuda_f32_vector(scores, C, "scores")
    idx = torch.empty(int(K), dtype=torch.int32, device=scores.device)
    s = torch.cuda.current_stream(scores.device) if stream is None else stream
    ctx._check(ctx._lib.split_topk_smallest(ctx._h, ctypes.c_void_p(scores.data_ptr()), C,
                                            int(K), ctypes.c_void_p(idx.data_ptr()),
                                            ctypes.c_void_p(s.cuda_stream)))
    return idx


def search(ctx: SplitContext, tour0, demand, Q: int, batch: int, budget_s: float,
           pool: int | None = None, nn: SplitNN | None = None, max_iters: int = 1 << 62,
           seed: int = 0, S: int | None = None, trace_cap: int = 100000, stream=None):
    """Local search from tour0 with the exact expected cost (split_search). Returns a dict with
    best_tour, the result fields and the (seconds, mean) trace of accepted moves."""
    import torch
    np = _np()
    t0 = np.ascontiguousarray(tour0, dtype=np.int32)
    ld, S = _demand_shape(demand, S, t0, ctx.N)
    if demand.shape[0] < ctx.N:
        raise ValueError("the demand tensor needs a row for every customer 1..N")
    pool = batch if pool is None else int(pool)
    best = np.zeros_like(t0)
    tt = np.zeros(trace_cap)
    tm = np.zeros(trace_cap)
    tl = ctypes.c_int32()
    res = SplitSearchResultC()
    s = torch.cuda.current_stream(demand.device) if stream is None else stream
    ctx._check(ctx._lib.split_search(
        ctx._h, nn._h if nn is not None else None, t0.ctypes.data_as(ctypes.c_void_p), t0.size,
        ctypes.c_void_p(demand.data_ptr()), S, ld, int(Q), int(batch), pool, float(budget_s),
        int(max_iters), int(seed), best.ctypes.data_as(ctypes.c_void_p),
        tt.ctypes.data_as(ctypes.c_void_p), tm.ctypes.data_as(ctypes.c_void_p), int(trace_cap),
        ctypes.byref(tl), ctypes.byref(res), ctypes.c_void_p(s.cuda_stream)))
    out = {f: getattr(res, f) for f, _ in SplitSearchResultC._fields_}
    out["best_tour"] = best
    out["trace"] = list(zip(tt[:tl.value].tolist(), tm[:tl.value].tolist()))
    return out
