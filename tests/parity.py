"""Comparison helpers of the GPU parity tests: the FP32 device path against the FP64 oracle.

Normwise: ||A - B||_F / ||B||_F (held to 1e-5 after one epoch of the ring order).

Elementwise, per vector: max_l |A_il - B_il| / max_l |B_il| for every row i of W or H.
The bound comes from the arithmetic, not from observed values.  The device repeats the
oracle's operations in FP32: every update of a variable rounds it twice (two FMAs), and
the residual's dot product adds an error of the same order scaled by the step size.
Under the probabilistic model of rounding errors (independent, mean zero: Higham and
Mary, "A new approach to probabilistic rounding error analysis", 2019), after T updates
the accumulated error stays below lambda * sqrt(2 T) * u * M with probability at least
1 - 2 exp(-lambda^2 / 2), u = 2^-24 the FP32 unit roundoff and M the vector's magnitude;
errors of coupled variables enter through the step size times the residual (of order
0.01-0.1 per update here), so T is taken as the largest number of updates any variable
receives in the run.  lambda = 10 makes a false alarm on any of 10^8 vectors impossible in
practice.  A single element wrong by 1% of its value fails the check as soon as the element
exceeds a few thousandths of its vector's largest entry.

Also reported: max |A - B| / (|B| + 1e-3), the elementwise relative error with an absolute
floor of 1e-3."""
from __future__ import annotations

import math

import numpy as np

U32 = 2.0 ** -24
LAMBDA = 10.0


def rel(a, b) -> float:
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def elem_tolerance(updates: int) -> float:
    """Per-vector bound max|delta| / max|x| after `updates` updates of the busiest variable."""
    return LAMBDA * math.sqrt(2.0 * max(int(updates), 1)) * U32


def elem_error(a, b) -> float:
    """max over rows of max_l |a - b| / max_l |b| (rows whose oracle values are all zero
    are compared absolutely)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    scale = np.max(np.abs(b), axis=1, keepdims=True)
    scale = np.where(scale > 0, scale, 1.0)
    return float(np.max(np.abs(a - b) / scale)) if a.size else 0.0


def floored_rel(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b) / (np.abs(b) + 1e-3))) if a.size else 0.0


def max_updates(row, col, epochs: int) -> int:
    """Updates received by the busiest row or column vector over `epochs` epochs."""
    row = np.asarray(row)
    col = np.asarray(col)
    if row.size == 0:
        return 1
    return int(max(np.bincount(row).max(), np.bincount(col).max())) * int(epochs)


def check(a, b, *, norm_tol: float, updates: int, what: str = "") -> dict:
    """Assert both bounds for one factor matrix; return the figures (printed by the caller)."""
    r = rel(a, b)
    e = elem_error(a, b)
    tol = elem_tolerance(updates)
    c = floored_rel(a, b)
    print(f"[parity] {what}: normwise {r:.2e} (<= {norm_tol:.0e}), per-vector max {e:.2e} (<= {tol:.2e}), "
          f"floored rel {c:.2e}", flush=True)
    assert r <= norm_tol, (what, r, norm_tol)
    assert e <= tol, (what, e, tol)
    return dict(normwise=r, elementwise=e, elem_tol=tol, floored=c)
