"""FP64 CPU oracle for NOMAD SGD (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The HIP product path neither imports nor links it.

The arithmetic lives in ``nomad_oracle.c`` (plain C, IEEE double, single thread); this
module only builds it with gcc and marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nomad_oracle.c")
_LIB = os.path.join(_HERE, "libnomad_oracle.so")
_lib = None

OK, EINVAL, ENOMEM, EDEADLOCK = 0, -1, -2, -3


class Stats(C.Structure):
    _fields_ = [("updates", C.c_int64), ("visits", C.c_int64), ("violations", C.c_int64),
                ("hops", C.c_int64), ("max_queue", C.c_int64)]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math: IEEE semantics are part of the contract)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-pthread", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = C.CDLL(_LIB)
        i32, i64, u64, dbl = C.c_int32, C.c_int64, C.c_uint64, C.c_double
        P = C.c_void_p
        lib.orc_splitmix64.restype = u64
        lib.orc_splitmix64.argtypes = [u64]
        lib.orc_owner0.restype = i32
        lib.orc_owner0.argtypes = [u64, i64, i32]
        lib.orc_step.restype = dbl
        lib.orc_step.argtypes = [dbl, dbl, dbl, dbl]
        lib.orc_update.restype = None
        lib.orc_update.argtypes = [i32, P, P, dbl, dbl, dbl]
        lib.orc_partition.restype = C.c_int
        lib.orc_partition.argtypes = [i64, i64, P, i32, P]
        common = [i64, i64, i64, P, P, P, i32, dbl, dbl, dbl, dbl, i32, u64]
        lib.orc_train_ring.restype = C.c_int
        lib.orc_train_ring.argtypes = common + [i32, i32, P, P, P]
        lib.orc_lowbias32.restype = C.c_uint32
        lib.orc_lowbias32.argtypes = [C.c_uint32]
        lib.orc_sr_bits.restype = C.c_uint32
        lib.orc_sr_bits.argtypes = [C.c_uint32, i64, i64, i64, i32]
        lib.orc_round_bf16.restype = dbl
        lib.orc_round_bf16.argtypes = [dbl, i32, C.c_uint32]
        lib.orc_train_ring_bf16.restype = C.c_int
        lib.orc_train_ring_bf16.argtypes = common + [i32, i32, i32, C.c_uint32, P, P, P]
        lib.orc_train_ring_interleaved.restype = C.c_int
        lib.orc_train_ring_interleaved.argtypes = common + [i32, i32, u64, P, P, P]
        lib.orc_train_ring_gcount.restype = C.c_int
        lib.orc_train_ring_gcount.argtypes = common + [i64, i32, P, P, P]
        lib.orc_train_perm.restype = C.c_int
        lib.orc_train_perm.argtypes = common + [i32, i32, u64, P, P, P, P, i64, P, i32]
        lib.orc_train_uniform.restype = C.c_int
        lib.orc_train_uniform.argtypes = common + [i64, u64, P, P, P, P, P, i64, P, i32, i32, dbl, dbl]
        lib.orc_balanced_pick.restype = i32
        lib.orc_balanced_pick.argtypes = [i32, i64, i32, i64]
        lib.orc_train_threaded.restype = C.c_int
        lib.orc_train_threaded.argtypes = common + [i64, u64, P, P, P, P]
        lib.orc_replay.restype = C.c_int
        lib.orc_replay.argtypes = common + [i64, P, P, P, P, P, P, P]
        lib.orc_set_progress.restype = None
        lib.orc_set_progress.argtypes = [i64]
        lib.orc_rmse.restype = C.c_int
        lib.orc_rmse.argtypes = [i64, i64, i64, P, P, P, i32, P, P, P]
        lib.orc_objective.restype = C.c_int
        lib.orc_objective.argtypes = [i64, i64, i64, P, P, P, i32, dbl, P, P, P]
        lib.orc_objective_loss.restype = C.c_int
        lib.orc_objective_loss.argtypes = [i64, i64, i64, P, P, P, i32, dbl, P, P, P, i32]
        lib.orc_train_ring_loss.restype = C.c_int
        lib.orc_train_ring_loss.argtypes = common + [i32, i32, P, P, P, i32]
        lib.orc_replay_loss.restype = C.c_int
        lib.orc_replay_loss.argtypes = common + [i64, P, P, P, P, P, P, P, i32]
        lib.orc_residual.restype = dbl
        lib.orc_residual.argtypes = [dbl, dbl, i32]
        lib.orc_loss.restype = dbl
        lib.orc_loss.argtypes = [dbl, dbl, i32]
        lib.orc_update_loss.restype = None
        lib.orc_update_loss.argtypes = [i32, P, P, dbl, dbl, dbl, i32]
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _coo(row, col, val):
    row = np.ascontiguousarray(np.asarray(row, dtype=np.int32))
    col = np.ascontiguousarray(np.asarray(col, dtype=np.int32))
    val = np.ascontiguousarray(np.asarray(val, dtype=np.float32))
    assert row.shape == col.shape == val.shape
    return row, col, val


def _factors(X, rows, k):
    X = np.array(X, dtype=np.float64, order="C", copy=True)
    assert X.shape == (rows, k), (X.shape, rows, k)
    return X


class OracleError(RuntimeError):
    pass


def _check(rc):
    if rc != OK:
        raise OracleError({EINVAL: "invalid input", ENOMEM: "out of memory",
                           EDEADLOCK: "schedule cannot progress"}.get(rc, str(rc)))


@dataclass
class Hyper:
    k: int
    lam: float
    alpha: float
    beta: float
    gamma: float


def splitmix64(x: int) -> int:
    return int(_load().orc_splitmix64(x & 0xFFFFFFFFFFFFFFFF))


def owner0(seed: int, j: int, p: int) -> int:
    return int(_load().orc_owner0(seed, j, p))


def step(alpha, beta, gamma, t) -> float:
    return float(_load().orc_step(alpha, beta, gamma, float(t)))


def update(w, h, r, s, lam):
    """One SGD update; returns (w', h') as new float64 arrays."""
    w = np.array(w, dtype=np.float64)
    h = np.array(h, dtype=np.float64)
    _load().orc_update(w.size, _p(w), _p(h), float(r), float(s), float(lam))
    return w, h


def partition(m, row, p):
    row = np.ascontiguousarray(np.asarray(row, dtype=np.int32))
    out = np.zeros(p + 1, dtype=np.int64)
    _check(_load().orc_partition(m, row.size, _p(row), p, _p(out)))
    return out


LOSS = {"square": 0, "logistic": 1}


def residual(r, d, loss="square") -> float:
    return float(_load().orc_residual(float(r), float(d), LOSS[loss]))


def loss_value(r, d, loss="square") -> float:
    return float(_load().orc_loss(float(r), float(d), LOSS[loss]))


def update_loss(w, h, r, s, lam, loss="square"):
    """One update of copies of w and h (FP64) under the given loss."""
    w = np.array(w, dtype=np.float64, copy=True)
    h = np.array(h, dtype=np.float64, copy=True)
    _load().orc_update_loss(w.size, _p(w), _p(h), float(r), float(s), float(lam), LOSS[loss])
    return w, h


def train_ring(m, n, row, col, val, W0, H0, hp: Hyper, p, seed, epochs, epoch0=0,
               interleave_seed=None, loss="square"):
    """Fixed token-passing order; with interleave_seed, the same orders under a random
    asynchronous interleaving (square loss only).  Returns (W, H, stats)."""
    row, col, val = _coo(row, col, val)
    W = _factors(W0, m, hp.k)
    H = _factors(H0, n, hp.k)
    st = Stats()
    lib = _load()
    args = (m, n, row.size, _p(row), _p(col), _p(val), hp.k, hp.lam, hp.alpha, hp.beta, hp.gamma,
            p, seed, epoch0, epochs)
    if interleave_seed is None:
        _check(lib.orc_train_ring_loss(*args, _p(W), _p(H), C.byref(st), LOSS[loss]))
    else:
        assert loss == "square"
        _check(lib.orc_train_ring_interleaved(*args, interleave_seed, _p(W), _p(H), C.byref(st)))
    return W, H, st


def lowbias32(x: int) -> int:
    return int(_load().orc_lowbias32(x & 0xFFFFFFFF))


def sr_bits(seed: int, i: int, j: int, t: int, l: int) -> int:
    return int(_load().orc_sr_bits(seed & 0xFFFFFFFF, i, j, t, l))


def round_bf16(x: float, rounding: int = 0, bits: int = 0) -> float:
    """x rounded to FP32, then to bfloat16 (0 nearest-even, 1 stochastic with `bits`)."""
    return float(_load().orc_round_bf16(float(x), rounding, bits & 0xFFFFFFFF))


def train_ring_bf16(m, n, row, col, val, W0, H0, hp: Hyper, p, seed, epochs, rounding, sr_seed, epoch0=0):
    """Ring order with w_i stored in bfloat16 (rounding 0 nearest-even, 1 stochastic)."""
    row, col, val = _coo(row, col, val)
    W = _factors(W0, m, hp.k)
    H = _factors(H0, n, hp.k)
    st = Stats()
    _check(_load().orc_train_ring_bf16(m, n, row.size, _p(row), _p(col), _p(val), hp.k, hp.lam, hp.alpha,
                                       hp.beta, hp.gamma, p, seed, epoch0, epochs, rounding, sr_seed & 0xFFFFFFFF,
                                       _p(W), _p(H), C.byref(st)))
    return W, H, st


def train_ring_gcount(m, n, row, col, val, W0, H0, hp: Hyper, p, seed, epochs, t0=0):
    """Ring order with t = the global count of updates before each visit (from t0)."""
    row, col, val = _coo(row, col, val)
    W = _factors(W0, m, hp.k)
    H = _factors(H0, n, hp.k)
    st = Stats()
    _check(_load().orc_train_ring_gcount(m, n, row.size, _p(row), _p(col), _p(val), hp.k, hp.lam, hp.alpha,
                                         hp.beta, hp.gamma, p, seed, int(t0), epochs, _p(W), _p(H), C.byref(st)))
    return W, H, st


def _trace_buf(cap):
    return np.zeros((max(int(cap), 1), 4), dtype=np.int32), C.c_int64()


def balanced_pick(a: int, len_a: int, b: int, len_b: int) -> int:
    """Section 3.3's load-balanced choice between two workers (a on a tie)."""
    return int(_load().orc_balanced_pick(a, len_a, b, len_b))


def train_perm(m, n, row, col, val, W0, H0, hp: Hyper, p, seed, epochs, sched_seed, epoch0=0, trace=False,
               balance=False):
    """Random-permutation circulation (discrete-event emulation).  Returns (W, H, stats),
    plus the visit trace (rows: worker, item, t, visit number of the item) with trace=True.
    balance=True: section 3.3's dynamic load balancing of the next holder."""
    row, col, val = _coo(row, col, val)
    W = _factors(W0, m, hp.k)
    H = _factors(H0, n, hp.k)
    st = Stats()
    cap = epochs * min(row.size, n * p) if trace else 0
    buf, tlen = _trace_buf(cap)
    _check(_load().orc_train_perm(m, n, row.size, _p(row), _p(col), _p(val), hp.k, hp.lam, hp.alpha,
                                  hp.beta, hp.gamma, p, seed, epoch0, epochs, sched_seed, _p(W), _p(H),
                                  C.byref(st), _p(buf) if trace else None, cap, C.byref(tlen), int(bool(balance))))
    if trace:
        assert tlen.value <= cap
        return W, H, st, buf[:tlen.value].copy()
    return W, H, st


def train_uniform(m, n, row, col, val, W0, H0, hp: Hyper, p, seed, max_updates, sched_seed,
                  visit_count=None, trace=False, trace_cap=None, balance=False, timing=None):
    """Algorithm 1 with uniform recipients (discrete-event emulation).  Returns (W, H,
    stats), plus the trace of the visits that update something with trace=True.
    balance=True: the recipient is the less loaded of two uniform draws (section 3.3).
    timing=(slots, visit_cost, hop_time): turns follow time (workers serving `slots` items
    at once, costs in units of one update) instead of a uniform draw."""
    slots, vcost, hop = timing if timing is not None else (0, 0.0, 0.0)
    row, col, val = _coo(row, col, val)
    W = _factors(W0, m, hp.k)
    H = _factors(H0, n, hp.k)
    if visit_count is None:
        visit_count = np.zeros(p * n, dtype=np.int32)
    assert visit_count.dtype == np.int32 and visit_count.size == p * n
    st = Stats()
    cap = (trace_cap if trace_cap is not None else int(max_updates) + 1) if trace else 0
    buf, tlen = _trace_buf(cap)
    _check(_load().orc_train_uniform(m, n, row.size, _p(row), _p(col), _p(val), hp.k, hp.lam, hp.alpha,
                                     hp.beta, hp.gamma, p, seed, int(max_updates), sched_seed,
                                     _p(visit_count), _p(W), _p(H), C.byref(st),
                                     _p(buf) if trace else None, cap, C.byref(tlen), int(bool(balance)),
                                     int(slots), float(vcost), float(hop)))
    if trace:
        assert tlen.value <= cap
        return W, H, st, buf[:tlen.value].copy()
    return W, H, st


def train_threaded(m, n, row, col, val, W0, H0, hp: Hyper, p, seed, max_updates, sched_seed):
    """Algorithm 1 on p POSIX threads (CPU throughput baseline).  Returns (W, H, stats,
    seconds of the threaded run, layout excluded)."""
    row, col, val = _coo(row, col, val)
    W = _factors(W0, m, hp.k)
    H = _factors(H0, n, hp.k)
    st = Stats()
    sec = C.c_double()
    _check(_load().orc_train_threaded(m, n, row.size, _p(row), _p(col), _p(val), hp.k, hp.lam, hp.alpha,
                                      hp.beta, hp.gamma, p, seed, int(max_updates), sched_seed, _p(W), _p(H),
                                      C.byref(st), C.byref(sec)))
    return W, H, st, sec.value


def replay(m, n, row, col, val, W0, H0, hp: Hyper, p, seed, tq, tj, tt, tseq, loss="square"):
    row, col, val = _coo(row, col, val)
    W = _factors(W0, m, hp.k)
    H = _factors(H0, n, hp.k)
    tq, tj, tt, tseq = (np.ascontiguousarray(np.asarray(a, dtype=np.int32)) for a in (tq, tj, tt, tseq))
    st = Stats()
    _check(_load().orc_replay_loss(m, n, row.size, _p(row), _p(col), _p(val), hp.k, hp.lam, hp.alpha, hp.beta,
                                   hp.gamma, p, seed, tq.size, _p(tq), _p(tj), _p(tt), _p(tseq), _p(W), _p(H),
                                   C.byref(st), LOSS[loss]))
    return W, H, st


def set_progress(every: int) -> None:
    """Report progress on stderr every `every` updates (0 = off)."""
    _load().orc_set_progress(int(every))


def rmse(m, n, row, col, val, W, H) -> float:
    row, col, val = _coo(row, col, val)
    W = np.ascontiguousarray(W, dtype=np.float64)
    H = np.ascontiguousarray(H, dtype=np.float64)
    out = C.c_double()
    _check(_load().orc_rmse(m, n, row.size, _p(row), _p(col), _p(val), W.shape[1], _p(W), _p(H),
                            C.byref(out)))
    return out.value


def objective(m, n, row, col, val, W, H, lam, loss="square") -> float:
    row, col, val = _coo(row, col, val)
    W = np.ascontiguousarray(W, dtype=np.float64)
    H = np.ascontiguousarray(H, dtype=np.float64)
    out = C.c_double()
    _check(_load().orc_objective_loss(m, n, row.size, _p(row), _p(col), _p(val), W.shape[1], float(lam),
                                      _p(W), _p(H), C.byref(out), LOSS[loss]))
    return out.value
