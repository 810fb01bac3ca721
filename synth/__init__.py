"""Seeded synthetic matrix-completion inputs shared by the oracle tests and the HIP path.

This module only *creates inputs*: observed-entry locations, rating values, the
train/test split and the initial factors.  It contains none of the NOMAD method's
arithmetic (no SGD update, no partition, no routing, no RMSE), so the oracle and the
device path can both consume it without sharing any method code.

The recipes stand in for the paper's benchmark data (Netflix, Yahoo! Music and
Hugewiki, Table "Dataset Details" in the experimental-setup section), which are not
available here.  They follow the paper's own synthetic recipe (the "scaling as both
dataset size and number of machines grow" section: planted Gaussian user/item
factors, Gaussian noise of standard deviation 0.1, nonzero locations drawn given the
row/column degree profile) with the shapes of the paper's datasets.

Planted model: u_i, v_j in R^rank with i.i.d. N(0, var = 1/sqrt(rank)) entries, so
Var <u_i, v_j> = 1 for every rank.  Locations: "uniform" draws distinct cells
uniformly; "zipf" is a capped Chung-Lu draw: rows and columns get weights
rank^-alpha over a random permutation, pairs are drawn independently from the two
weight vectors, duplicates are removed, and the draw is topped up until exactly
`nnz` distinct cells remain (a uniform subset is kept).  Heavy rows/columns thereby
saturate at the opposite dimension (the cap).

Initial factors: every entry of W and H is Uniform(0, 1/sqrt(k)) as in the
initialisation lines of the paper's NOMAD algorithm (and its experimental setup).

Everything is generated with torch on a chosen device from a seeded
``torch.Generator``; results are deterministic per (seed, device).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import torch

__all__ = [
    "Problem",
    "planted_problem",
    "init_factors",
    "tiny",
    "medium",
    "large",
    "very_tall",
    "batched_specs",
    "batched_problem",
    "small_case",
    "CONFIGS",
]


@dataclass
class Problem:
    """A matrix-completion instance in COO form (0-based int32 indices, fp32 values)."""

    m: int
    n: int
    row: torch.Tensor  # train rows, int32
    col: torch.Tensor  # train cols, int32
    val: torch.Tensor  # train ratings, float32
    test_row: torch.Tensor
    test_col: torch.Tensor
    test_val: torch.Tensor
    # hyper-parameters of the recipe (k, lambda, alpha, beta, gamma, epochs)
    hp: dict = field(default_factory=dict)
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row.numel())

    def to(self, device) -> "Problem":
        f = lambda t: t.to(device)  # noqa: E731
        return Problem(self.m, self.n, f(self.row), f(self.col), f(self.val), f(self.test_row),
                       f(self.test_col), f(self.test_val), dict(self.hp), self.name)


def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def _weights_zipf(size: int, alpha: float, g: torch.Generator, device) -> torch.Tensor:
    """Rank-frequency weights rank^-alpha placed on a random permutation of the ids."""
    ranks = torch.arange(1, size + 1, dtype=torch.float64, device=device)
    w_by_rank = ranks.pow(-alpha)
    perm = torch.randperm(size, generator=g, device=device)
    w = torch.empty(size, dtype=torch.float64, device=device)
    w[perm] = w_by_rank
    return w / w.sum()


def _draw_from(cdf: torch.Tensor, count: int, g: torch.Generator, device) -> torch.Tensor:
    u = torch.rand(count, generator=g, device=device, dtype=torch.float64)
    idx = torch.searchsorted(cdf, u, right=True)
    return idx.clamp_(max=cdf.numel() - 1)


def _sample_cells(m: int, n: int, nnz: int, degrees: str, alpha: float,
                  g: torch.Generator, device, cdf_c: Optional[torch.Tensor] = None) -> tuple[torch.Tensor, torch.Tensor]:
    """Distinct (row, col) cells, exactly nnz of them, in random order.  cdf_c: column
    weights (cumulative) to use instead of drawing them (zipf only)."""
    total = m * n
    if nnz > total:
        raise ValueError(f"nnz={nnz} exceeds m*n={total}")
    if degrees == "uniform":
        keys = torch.empty(0, dtype=torch.int64, device=device)
        while keys.numel() < nnz:
            need = nnz - keys.numel()
            draw = torch.randint(0, total, (int(need * 1.1) + 64,), generator=g, device=device,
                                 dtype=torch.int64)
            keys = torch.unique(torch.cat([keys, draw]))
    elif degrees == "zipf":
        wr = _weights_zipf(m, alpha, g, device)
        cdf_r = torch.cumsum(wr, 0)
        cdf_r[-1] = 1.0
        if cdf_c is None:
            wc = _weights_zipf(n, alpha, g, device)
            cdf_c = torch.cumsum(wc, 0)
            cdf_c[-1] = 1.0
        keys = torch.empty(0, dtype=torch.int64, device=device)
        rounds = 0
        while keys.numel() < nnz:
            need = nnz - keys.numel()
            batch = min(max(int(need * 1.5) + 1024, 1 << 16), 1 << 27)
            i = _draw_from(cdf_r, batch, g, device)
            j = _draw_from(cdf_c, batch, g, device)
            keys = torch.unique(torch.cat([keys, i * n + j]))
            rounds += 1
            if rounds > 400:
                raise RuntimeError("zipf cell sampler did not converge")
    else:
        raise ValueError(degrees)
    # a uniform subset of exactly nnz cells, in random order
    pick = torch.randperm(keys.numel(), generator=g, device=device)[:nnz]
    keys = keys[pick]
    return (keys // n).to(torch.int32), (keys % n).to(torch.int32)


def _dot_rows(U, V, row, col, chunk=1 << 23) -> torch.Tensor:
    """<U[row], V[col]> per cell, in chunks."""
    out = torch.empty(row.numel(), dtype=torch.float32, device=U.device)
    for s in range(0, row.numel(), chunk):
        e = min(s + chunk, row.numel())
        out[s:e] = (U[row[s:e].long()] * V[col[s:e].long()]).sum(1)
    return out


def _planted_values(row, col, m, n, rank, g, device) -> torch.Tensor:
    """<u_i, v_j> with u, v ~ N(0, var 1/sqrt(rank)) entries (so Var<u,v> = 1)."""
    std = rank ** -0.25
    U = torch.randn(m, rank, generator=g, device=device, dtype=torch.float32) * std
    V = torch.randn(n, rank, generator=g, device=device, dtype=torch.float32) * std
    return _dot_rows(U, V, row, col)


def planted_problem(m: int, n: int, nnz: int, rank: int, *, seed: int, degrees: str = "uniform",
                    alpha: float = 1.1, values: str = "gaussian", noise: float = 0.1,
                    n_test: Optional[int] = None, test_frac: Optional[float] = None,
                    device="cpu", hp: Optional[dict] = None, name: str = "") -> Problem:
    """Draw a planted low-rank completion problem.

    values:
      "gaussian"  r = x + N(0, noise^2)
      "int15"     r = clip(round(3 + x + N(0, noise^2)), 1, 5)   (integer star ratings)
      "scaled100" r = clip(50 + 25 (x + N(0, noise^2)), 0, 100)
      "sign"      r = +1 if x + N(0, noise^2) >= 0 else -1   (binary labels)
    where x = <u_i, v_j>.  The test set is a uniform subset of the drawn cells.
    """
    g = _gen(seed, device)
    row, col = _sample_cells(m, n, nnz, degrees, alpha, g, device)
    x = _planted_values(row, col, m, n, rank, g, device)
    eps = torch.randn(nnz, generator=g, device=device, dtype=torch.float32) * noise
    if values == "gaussian":
        val = x + eps
    elif values == "int15":
        val = torch.clamp(torch.round(3.0 + x + eps), 1.0, 5.0)
    elif values == "scaled100":
        val = torch.clamp(50.0 + 25.0 * (x + eps), 0.0, 100.0)
    elif values == "sign":
        val = torch.where(x + eps >= 0.0, 1.0, -1.0).to(torch.float32)
    else:
        raise ValueError(values)
    if n_test is None:
        n_test = int(round(nnz * (test_frac or 0.0)))
    # cells are already in random order: the first n_test are the held-out set
    te = slice(0, n_test)
    tr = slice(n_test, nnz)
    return Problem(m, n, row[tr].contiguous(), col[tr].contiguous(), val[tr].contiguous(),
                   row[te].contiguous(), col[te].contiguous(), val[te].contiguous(),
                   dict(hp or {}), name)


def init_factors(m: int, n: int, k: int, seed: int, device="cpu") -> tuple[torch.Tensor, torch.Tensor]:
    """W0 (m x k) and H0 (n x k), fp32 row-major, entries Uniform(0, 1/sqrt(k))."""
    g = _gen(seed ^ 0x5EED_F00D, device)
    hi = 1.0 / math.sqrt(k)
    W0 = torch.rand(m, k, generator=g, device=device, dtype=torch.float32) * hi
    H0 = torch.rand(n, k, generator=g, device=device, dtype=torch.float32) * hi
    return W0, H0


# ----------------------------------------------------------------------------------
# Named workloads.  Hyper-parameters: k, lambda and the step-size schedule
# s_t = alpha / (1 + beta * t^gamma).  The paper's Table of parameters gives
# (k, lambda, alpha, beta) for the three datasets with gamma = 1.5; the tiny and
# batched recipes use alpha=0.01, beta=1e-4, gamma=1.
# ----------------------------------------------------------------------------------

def tiny(device="cpu") -> Problem:
    """2,000 x 1,000, 100k uniform cells, planted rank 10 + N(0, 0.1^2), 10% held out."""
    return planted_problem(2000, 1000, 100_000, 10, seed=1, degrees="uniform", values="gaussian",
                           noise=0.1, test_frac=0.10, device=device, name="tiny",
                           hp=dict(k=16, lam=0.05, alpha=0.01, beta=1e-4, gamma=1.0, epochs=20))


def medium(device="cpu") -> Problem:
    """Netflix-shaped: 480,189 x 17,770, 100M Zipf(1.1) cells, integer 1..5 ratings, 1.4M held out."""
    return planted_problem(480_189, 17_770, 100_000_000, 30, seed=2, degrees="zipf", alpha=1.1,
                           values="int15", noise=0.5, n_test=1_400_000, device=device, name="medium",
                           hp=dict(k=100, lam=0.05, alpha=0.012, beta=0.05, gamma=1.5, epochs=10))


def large(device="cpu") -> Problem:
    """Yahoo!-Music-shaped: 1,000,990 x 624,961, 252.8M power-law cells, ratings 0..100."""
    return planted_problem(1_000_990, 624_961, 252_800_000, 50, seed=3, degrees="zipf", alpha=1.1,
                           values="scaled100", noise=0.1, test_frac=0.014, device=device, name="large",
                           hp=dict(k=100, lam=1.0, alpha=0.00075, beta=0.01, gamma=1.5, epochs=10))


VT_BLOCK_ROWS = 3_125_000
VT_BLOCK_CELLS = 171_250_000
VT_BLOCKS = 16


def very_tall(device="cpu", blocks: int = VT_BLOCKS) -> Problem:
    """Hugewiki-shaped: 50,000,000 x 39,780, 2.74 B cells, real ratings.

    Drawn as 16 row blocks of 3,125,000 rows and 171,250,000 cells each.  Every block
    follows the capped Chung-Lu recipe with Zipf(1.1) row weights over its own rows and
    column weights shared by all blocks; values are <u_i, v_j> + N(0, 0.1^2) with planted
    rank 50 (the v_j shared), 1.4% of each block held out.  `blocks` < 16 gives the first
    `blocks` blocks (rows 0 .. blocks * 3,125,000), a row sample of the full matrix.
    Blocks keep every sort below the 2^31 items one torch.unique call takes.
    """
    if not 1 <= blocks <= VT_BLOCKS:
        raise ValueError(blocks)
    n, rank, seed = 39_780, 50, 5
    gc = _gen(seed, device)
    wc = _weights_zipf(n, 1.1, gc, device)
    cdf_c = torch.cumsum(wc, 0)
    cdf_c[-1] = 1.0
    V = torch.randn(n, rank, generator=gc, device=device, dtype=torch.float32) * rank ** -0.25
    mb, cb = VT_BLOCK_ROWS, VT_BLOCK_CELLS
    n_test_b = int(round(cb * 0.014))
    n_train_b = cb - n_test_b
    row = torch.empty(blocks * n_train_b, dtype=torch.int32, device=device)
    col = torch.empty_like(row)
    val = torch.empty(blocks * n_train_b, dtype=torch.float32, device=device)
    trow = torch.empty(blocks * n_test_b, dtype=torch.int32, device=device)
    tcol = torch.empty_like(trow)
    tval = torch.empty(blocks * n_test_b, dtype=torch.float32, device=device)
    for b in range(blocks):
        g = _gen(seed * 1_000_003 + b + 1, device)
        r, c = _sample_cells(mb, n, cb, "zipf", 1.1, g, device, cdf_c=cdf_c)
        U = torch.randn(mb, rank, generator=g, device=device, dtype=torch.float32) * rank ** -0.25
        x = _dot_rows(U, V, r, c)
        v = x + torch.randn(cb, generator=g, device=device, dtype=torch.float32) * 0.1
        r = r + b * mb
        # cells come in random order: the first n_test_b of the block are held out
        trow[b * n_test_b:(b + 1) * n_test_b] = r[:n_test_b]
        tcol[b * n_test_b:(b + 1) * n_test_b] = c[:n_test_b]
        tval[b * n_test_b:(b + 1) * n_test_b] = v[:n_test_b]
        row[b * n_train_b:(b + 1) * n_train_b] = r[n_test_b:]
        col[b * n_train_b:(b + 1) * n_train_b] = c[n_test_b:]
        val[b * n_train_b:(b + 1) * n_train_b] = v[n_test_b:]
        del r, c, U, x, v
    return Problem(blocks * mb, n, row, col, val, trow, tcol, tval,
                   dict(k=100, lam=0.01, alpha=0.001, beta=0.0, gamma=1.5, epochs=5), "very_tall")


def batched_specs(count: int = 256, seed: int = 4) -> list[dict]:
    """Per-problem shapes of the batched workload: log-uniform sizes, k in {16,32,64},
    lambda in {0.01,0.05,0.1}; nnz clamped to half the cells."""
    g = torch.Generator().manual_seed(seed)
    out = []
    for b in range(count):
        u = torch.rand(3, generator=g, dtype=torch.float64)
        m = int(round(math.exp(math.log(1e3) + u[0].item() * (math.log(2e5) - math.log(1e3)))))
        n = int(round(math.exp(math.log(500) + u[1].item() * (math.log(2e4) - math.log(500)))))
        nnz = int(round(math.exp(math.log(5e4) + u[2].item() * (math.log(5e6) - math.log(5e4)))))
        nnz = min(nnz, (m * n) // 2)
        k = [16, 32, 64][int(torch.randint(0, 3, (1,), generator=g))]
        lam = [0.01, 0.05, 0.1][int(torch.randint(0, 3, (1,), generator=g))]
        out.append(dict(m=m, n=n, nnz=nnz, k=k, lam=lam, alpha=0.01, beta=1e-4, gamma=1.0,
                        seed=seed * 100_003 + b))
    return out


def batched_problem(spec: dict, device="cpu") -> Problem:
    return planted_problem(spec["m"], spec["n"], spec["nnz"], max(1, spec["k"] // 2), seed=spec["seed"],
                           degrees="uniform", values="gaussian", noise=0.1, test_frac=0.10,
                           device=device, name="batched",
                           hp=dict(k=spec["k"], lam=spec["lam"], alpha=spec["alpha"], beta=spec["beta"],
                                   gamma=spec["gamma"], epochs=5))


def small_case(m: int, n: int, nnz: int, *, seed: int, degrees="uniform", k=16, lam=0.05,
               alpha=0.01, beta=1e-4, gamma=1.0, rank=4, test_frac=0.1, device="cpu",
               values="gaussian") -> Problem:
    """Parity-test helper: an arbitrary small planted problem."""
    return planted_problem(m, n, nnz, rank, seed=seed, degrees=degrees, values=values, noise=0.1,
                           test_frac=test_frac, device=device, name=f"small{m}x{n}",
                           hp=dict(k=k, lam=lam, alpha=alpha, beta=beta, gamma=gamma, epochs=1))


CONFIGS = {"tiny": tiny, "medium": medium, "large": large, "very_tall": very_tall}
