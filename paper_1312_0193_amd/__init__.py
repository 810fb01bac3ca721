"""Python binding of libnomad.so, the MI355X NOMAD library (C ABI in include/nomad.h).

This module only marshals arguments: every step of the computation runs in the HIP
kernels of libnomad.so.  PyTorch provides device memory and the HIP stream.  There is
no fallback: if the library is missing or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
import re
from dataclasses import dataclass

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB_PATH = os.path.join(PKG, "libnomad.so")
HEADER = os.path.join(ROOT, "include", "nomad.h")

NOMAD_OK, NOMAD_EINVAL, NOMAD_ENOMEM, NOMAD_EDEVICE, NOMAD_ESTATE, NOMAD_ENOTIMPL = range(6)
SCHED = {"ring": 0, "perm": 1, "uniform": 2}
DTYPE = {"fp32": 0, "bf16": 1}
ROUND = {"rne": 0, "stochastic": 1}
T_SOURCE = {"pair": 0, "global": 1}
LOSS = {"square": 0, "logistic": 1}
_STATUS = {1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ESTATE", 5: "ENOTIMPL"}


class NomadConfig(C.Structure):
    _fields_ = [("k", C.c_int32), ("lambda_", C.c_float), ("alpha", C.c_float), ("beta", C.c_float),
                ("gamma", C.c_float), ("sched", C.c_int32), ("dtype", C.c_int32), ("rounding", C.c_int32),
                ("workers", C.c_int32), ("waves_per_worker", C.c_int32), ("item_slots", C.c_int32),
                ("window", C.c_int32),
                ("record_trace", C.c_int32), ("collect_stats", C.c_int32), ("debug_ownership", C.c_int32),
                ("t_source", C.c_int32), ("balance", C.c_int32), ("transpose", C.c_int32), ("loss", C.c_int32),
                ("seed", C.c_uint64)]


class NomadProblemDesc(C.Structure):
    _fields_ = [("m", C.c_int64), ("n", C.c_int64), ("nnz", C.c_int64), ("d_row", C.c_void_p),
                ("d_col", C.c_void_p), ("d_val", C.c_void_p), ("d_W0", C.c_void_p), ("d_H0", C.c_void_p),
                ("k", C.c_int32), ("lambda_", C.c_float), ("alpha", C.c_float), ("beta", C.c_float),
                ("gamma", C.c_float)]


class NomadStats(C.Structure):
    _fields_ = [("seconds", C.c_double), ("updates", C.c_uint64), ("epochs_done", C.c_uint64),
                ("layout_seconds", C.c_double), ("hops", C.c_uint64), ("violations", C.c_uint64)]


# nomad_tune_progress(const nomad_config *candidate, nomad_status status, double seconds, void *user)
TUNE_PROGRESS = C.CFUNCTYPE(None, C.POINTER(NomadConfig), C.c_int, C.c_double, C.c_void_p)


class NomadError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def library_path() -> str:
    return LIB_PATH


def load() -> C.CDLL:
    """Load libnomad.so (built by __graft_entry__.build() / paper_1312_0193_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1312_0193_amd/build.py")
    lib = C.CDLL(LIB_PATH)
    P, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    lib.nomad_config_default.restype = None
    lib.nomad_config_default.argtypes = [C.POINTER(NomadConfig)]
    lib.nomad_init.restype = C.c_int
    lib.nomad_init.argtypes = [C.POINTER(P), C.POINTER(NomadConfig), i64, i64, i64, P, P, P, P, P, P]
    lib.nomad_train_epochs.restype = C.c_int
    lib.nomad_train_epochs.argtypes = [P, i32, C.POINTER(NomadStats)]
    lib.nomad_eval_rmse.restype = C.c_int
    lib.nomad_eval_rmse.argtypes = [P, i64, P, P, P, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.nomad_eval_rmse_noalloc.restype = C.c_int
    lib.nomad_eval_rmse_noalloc.argtypes = [P, i64, P, P, P, P]
    lib.nomad_get_factors.restype = C.c_int
    lib.nomad_get_factors.argtypes = [P, P, P]
    lib.nomad_get_partition.restype = C.c_int
    lib.nomad_get_partition.argtypes = [P, C.POINTER(i32), P, i64]
    lib.nomad_get_trace.restype = C.c_int
    lib.nomad_get_trace.argtypes = [P, C.POINTER(i64), P, i64]
    lib.nomad_get_worker_stats.restype = C.c_int
    lib.nomad_get_worker_stats.argtypes = [P, P, i64]
    lib.nomad_init_batched.restype = C.c_int
    lib.nomad_init_batched.argtypes = [C.POINTER(P), i32, C.POINTER(NomadProblemDesc), C.POINTER(NomadConfig), P]
    lib.nomad_batch_problem.restype = C.c_int
    lib.nomad_batch_problem.argtypes = [P, i32, C.POINTER(P)]
    lib.nomad_batch_graph.restype = C.c_int
    lib.nomad_batch_graph.argtypes = [P, i32]
    lib.nomad_tune_batched.restype = C.c_int
    lib.nomad_tune_batched.argtypes = [i32, C.POINTER(NomadProblemDesc), C.POINTER(NomadConfig), P,
                                       TUNE_PROGRESS, P, C.POINTER(NomadConfig), C.POINTER(C.c_double)]
    lib.nomad_destroy.restype = None
    lib.nomad_destroy.argtypes = [P]
    lib.nomad_last_error.restype = C.c_char_p
    lib.nomad_last_error.argtypes = [P]
    _lib = lib
    return lib


def declared_functions() -> list[str]:
    """Names of the functions declared in include/nomad.h."""
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return re.findall(r"\b(nomad_[a-z_]+)\s*\(", src)


def _check(rc: int, ctx=None):
    if rc != NOMAD_OK:
        msg = load().nomad_last_error(ctx).decode()
        raise NomadError(rc, msg)


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _stream_handle():
    import torch
    return torch.cuda.current_stream().cuda_stream


def _dev_i32(t):
    import torch
    return t.to(device="cuda", dtype=torch.int32).contiguous()


def _dev_f32(t):
    import torch
    return t.to(device="cuda", dtype=torch.float32).contiguous()


@dataclass
class Stats:
    seconds: float
    updates: int
    epochs_done: int
    layout_seconds: float
    hops: int = 0
    violations: int = 0

    @property
    def updates_per_s(self) -> float:
        return self.updates / self.seconds if self.seconds > 0 else float("nan")


def make_config(k: int, lam: float, alpha: float, beta: float, gamma: float, *, sched="ring", dtype="fp32",
                rounding="rne", workers=0, waves_per_worker=0, item_slots=0, window=0, record_trace=False,
                collect_stats=False, debug_ownership=False, t_source="pair", balance=False,
                transpose=False, loss="square", seed=0) -> NomadConfig:
    cfg = NomadConfig()
    load().nomad_config_default(C.byref(cfg))
    cfg.k, cfg.lambda_, cfg.alpha, cfg.beta, cfg.gamma = k, lam, alpha, beta, gamma
    cfg.sched, cfg.dtype, cfg.rounding = SCHED[sched], DTYPE[dtype], ROUND[rounding]
    cfg.workers, cfg.waves_per_worker, cfg.item_slots = workers, waves_per_worker, item_slots
    cfg.window = window
    cfg.record_trace = int(bool(record_trace))
    cfg.collect_stats = int(bool(collect_stats))
    cfg.debug_ownership = int(bool(debug_ownership))
    cfg.t_source = T_SOURCE[t_source]
    cfg.balance = int(bool(balance))
    cfg.transpose = int(bool(transpose))
    cfg.loss = LOSS[loss]
    cfg.seed = seed
    return cfg


class Nomad:
    """One NOMAD problem resident on the GPU (wraps a nomad_ctx).

    row, col, val: training ratings (int32, int32, float32; any device, copied to the GPU);
    W0 (m x k), H0 (n x k): initial factors.
    """

    def __init__(self, m: int, n: int, row, col, val, W0, H0, *, k: int, lam: float, alpha: float,
                 beta: float, gamma: float, **kw):
        lib = load()
        self.m, self.n, self.k = int(m), int(n), int(k)
        self.cfg = make_config(k, lam, alpha, beta, gamma, **kw)
        row, col, val = _dev_i32(row), _dev_i32(col), _dev_f32(val)
        W0, H0 = _dev_f32(W0), _dev_f32(H0)
        if tuple(W0.shape) != (self.m, k) or tuple(H0.shape) != (self.n, k):
            raise ValueError("W0 must be m x k and H0 n x k")
        self.nnz = int(row.numel())
        ctx = C.c_void_p()
        _check(lib.nomad_init(C.byref(ctx), C.byref(self.cfg), self.m, self.n, self.nnz, _ptr(row), _ptr(col),
                              _ptr(val), _ptr(W0), _ptr(H0), _stream_handle()))
        self.ctx = ctx

    def _c(self):
        if self.ctx is None:
            raise NomadError(NOMAD_ESTATE, "context destroyed")
        return self.ctx

    def train(self, epochs: int) -> Stats:
        st = NomadStats()
        _check(load().nomad_train_epochs(self._c(), int(epochs), C.byref(st)), self.ctx)
        return Stats(st.seconds, st.updates, st.epochs_done, st.layout_seconds, st.hops, st.violations)

    def evaluate(self, row, col, val) -> tuple[float, float]:
        """(RMSE, objective J) over the given ratings, FP64."""
        row, col, val = _dev_i32(row), _dev_i32(col), _dev_f32(val)
        r, j = C.c_double(), C.c_double()
        _check(load().nomad_eval_rmse(self._c(), int(row.numel()), _ptr(row), _ptr(col), _ptr(val), C.byref(r),
                                      C.byref(j)), self.ctx)
        return r.value, j.value

    def evaluate_noalloc(self, row, col, val, out):
        """nomad_eval_rmse_noalloc: queue the evaluation on the context's stream; `out` is a
        float64 CUDA tensor of 3 elements that receives (RMSE, J, bad-index flag).  The
        rating tensors must already be int32/int32/float32 CUDA tensors (nothing is copied
        or allocated here)."""
        import torch
        if not (out.is_cuda and out.dtype == torch.float64 and out.numel() >= 3 and out.is_contiguous()):
            raise ValueError("out must be a contiguous CUDA float64 tensor of 3 elements")
        for t, dt in ((row, torch.int32), (col, torch.int32), (val, torch.float32)):
            if not (t.is_cuda and t.dtype == dt and t.is_contiguous()):
                raise ValueError("row, col, val must be contiguous CUDA int32, int32, float32 tensors")
        _check(load().nomad_eval_rmse_noalloc(self._c(), int(row.numel()), _ptr(row), _ptr(col), _ptr(val),
                                              _ptr(out)), self.ctx)

    def factors(self):
        import torch
        W = torch.empty(self.m, self.k, device="cuda", dtype=torch.float32)
        H = torch.empty(self.n, self.k, device="cuda", dtype=torch.float32)
        _check(load().nomad_get_factors(self._c(), _ptr(W), _ptr(H)), self.ctx)
        return W, H

    def partition(self):
        import numpy as np
        p = C.c_int32()
        _check(load().nomad_get_partition(self._c(), C.byref(p), None, 0), self.ctx)
        rs = np.zeros(p.value + 1, dtype=np.int64)
        _check(load().nomad_get_partition(self._c(), C.byref(p), rs.ctypes.data_as(C.c_void_p), rs.size), self.ctx)
        return rs

    def config(self) -> NomadConfig:
        """nomad_get_config: the configuration in use (the library's choices filled in)."""
        cfg = NomadConfig()
        _check(load().nomad_get_config(self._c(), C.byref(cfg)), self.ctx)
        return cfg

    @property
    def workers(self) -> int:
        p = C.c_int32()
        _check(load().nomad_get_partition(self._c(), C.byref(p), None, 0), self.ctx)
        return p.value

    def trace(self):
        import numpy as np
        n = C.c_int64()
        _check(load().nomad_get_trace(self._c(), C.byref(n), None, 0), self.ctx)
        buf = np.zeros((n.value, 4), dtype=np.int32)
        if n.value:
            _check(load().nomad_get_trace(self._c(), C.byref(n), buf.ctypes.data_as(C.c_void_p), n.value),
                   self.ctx)
        return buf

    def worker_stats(self):
        """(p, 16) int64 per worker for the last train() call, 100 MHz ticks unless a count
        (columns as listed in include/nomad.h)."""
        import numpy as np
        p = self.workers
        buf = np.zeros((p, 16), dtype=np.int64)
        _check(load().nomad_get_worker_stats(self._c(), buf.ctypes.data_as(C.c_void_p), buf.size), self.ctx)
        return buf

    def close(self):
        if getattr(self, "ctx", None) is not None:
            if getattr(self, "_owned", True):
                load().nomad_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def _problem_descs(problems):
    """nomad_problem_desc array for `problems` and the device tensors it points into."""
    keep = []
    descs = (NomadProblemDesc * len(problems))()
    for d, pr in zip(descs, problems):
        row, col, val = _dev_i32(pr["row"]), _dev_i32(pr["col"]), _dev_f32(pr["val"])
        W0, H0 = _dev_f32(pr["W0"]), _dev_f32(pr["H0"])
        k = int(pr["k"])
        if tuple(W0.shape) != (int(pr["m"]), k) or tuple(H0.shape) != (int(pr["n"]), k):
            raise ValueError("W0 must be m x k and H0 n x k")
        keep += [row, col, val, W0, H0]
        d.m, d.n, d.nnz = int(pr["m"]), int(pr["n"]), int(row.numel())
        d.d_row, d.d_col, d.d_val, d.d_W0, d.d_H0 = _ptr(row), _ptr(col), _ptr(val), _ptr(W0), _ptr(H0)
        d.k, d.lambda_, d.alpha, d.beta, d.gamma = k, pr["lam"], pr["alpha"], pr["beta"], pr["gamma"]
    return descs, keep


def tune_batched(problems, progress=None, **kw):
    """nomad_tune_batched: the fastest launch shape for a batch of `problems`.  Returns
    (dict(workers=, waves_per_worker=, window=), seconds of its epoch).  `progress`, if
    given, is called as progress(shape dict, status, seconds) after each candidate."""
    lib = load()
    cfg = make_config(1, 0.0, 0.0, 0.0, 0.0, **kw)
    descs, keep = _problem_descs(problems)
    best = NomadConfig()
    sec = C.c_double()

    def report(c, status, seconds, user):
        if progress is not None:
            c = c.contents
            progress(dict(workers=c.workers, waves_per_worker=c.waves_per_worker, window=c.window), status,
                     seconds)

    cb = TUNE_PROGRESS(report)
    _check(lib.nomad_tune_batched(len(problems), descs, C.byref(cfg), _stream_handle(), cb, None, C.byref(best),
                                  C.byref(sec)))
    del keep
    return dict(workers=best.workers, waves_per_worker=best.waves_per_worker, window=best.window), sec.value


class NomadBatch:
    """Several independent problems trained together by one launch per call (wraps a batch
    nomad_ctx).  `problems`: dicts with m, n, row, col, val, W0, H0, k, lam, alpha, beta,
    gamma; keyword arguments are the shared configuration (workers = total).  With
    autotune=True the launch shape (workers, compute waves, row window) left unset in the
    keywords is picked by nomad_tune_batched first (kept in .tuned)."""

    def __init__(self, problems, autotune=False, progress=None, **kw):
        lib = load()
        self.tuned = None
        if autotune:
            shape, sec = tune_batched(problems, progress=progress, **kw)
            self.tuned = dict(shape, seconds=sec)
            kw = dict(kw, **shape)
        self.cfg = make_config(1, 0.0, 0.0, 0.0, 0.0, **kw)
        descs, self._keep = _problem_descs(problems)
        ctx = C.c_void_p()
        _check(lib.nomad_init_batched(C.byref(ctx), len(problems), descs, C.byref(self.cfg), _stream_handle()))
        self._keep = []  # the inputs are copied by the call
        self.ctx = ctx
        self.problems = []
        for b, pr in enumerate(problems):
            sub = C.c_void_p()
            _check(lib.nomad_batch_problem(self.ctx, b, C.byref(sub)), self.ctx)
            view = Nomad.__new__(Nomad)
            view.m, view.n, view.k = int(pr["m"]), int(pr["n"]), int(pr["k"])
            view.ctx, view._owned, view.nnz = sub, False, int(pr["row"].numel())
            self.problems.append(view)

    def graph(self, epochs: int):
        """nomad_batch_graph: later train(epochs) calls replay a captured HIP graph (0 drops it)."""
        if self.ctx is None:
            raise NomadError(NOMAD_ESTATE, "batch destroyed")
        _check(load().nomad_batch_graph(self.ctx, int(epochs)), self.ctx)

    def train(self, epochs: int) -> Stats:
        if self.ctx is None:
            raise NomadError(NOMAD_ESTATE, "batch destroyed")
        st = NomadStats()
        _check(load().nomad_train_epochs(self.ctx, int(epochs), C.byref(st)), self.ctx)
        return Stats(st.seconds, st.updates, st.epochs_done, st.layout_seconds, st.hops, st.violations)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            for v in self.problems:
                v.ctx = None
            load().nomad_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
