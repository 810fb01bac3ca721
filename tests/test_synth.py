"""The seeded input generator: determinism, set semantics, shapes and value ranges."""
import math

import numpy as np
import torch

import synth


def test_deterministic_per_seed():
    a = synth.small_case(300, 200, 5000, seed=3)
    b = synth.small_case(300, 200, 5000, seed=3)
    c = synth.small_case(300, 200, 5000, seed=4)
    assert torch.equal(a.row, b.row) and torch.equal(a.val, b.val)
    assert not torch.equal(a.row, c.row)


def test_cells_distinct_and_in_range():
    for deg in ("uniform", "zipf"):
        p = synth.small_case(500, 300, 40_000, seed=5, degrees=deg, test_frac=0.2)
        r = torch.cat([p.row, p.test_row]).long()
        c = torch.cat([p.col, p.test_col]).long()
        assert r.numel() == 40_000
        assert torch.unique(r * p.n + c).numel() == 40_000
        assert r.min() >= 0 and r.max() < p.m and c.min() >= 0 and c.max() < p.n
        assert p.test_row.numel() == 8000


def test_zipf_degrees_are_skewed_and_capped():
    p = synth.planted_problem(20_000, 2_000, 400_000, 5, seed=9, degrees="zipf", test_frac=0.0)
    rdeg = torch.bincount(p.row.long(), minlength=p.m)
    cdeg = torch.bincount(p.col.long(), minlength=p.n)
    assert rdeg.max() <= p.n and cdeg.max() <= p.m
    assert rdeg.max() > 20 * rdeg.float().mean()  # heavy head
    assert cdeg.max() > 10 * cdeg.float().mean()


def test_value_recipes():
    g = synth.planted_problem(400, 300, 30_000, 10, seed=1, values="gaussian", noise=0.1, test_frac=0)
    assert 0.85 < g.val.double().var().item() < 1.2  # Var<u,v> = 1 plus noise 0.01
    i = synth.planted_problem(400, 300, 30_000, 10, seed=1, values="int15", noise=0.5, test_frac=0)
    assert set(torch.unique(i.val).tolist()) <= {1.0, 2.0, 3.0, 4.0, 5.0}
    s = synth.planted_problem(400, 300, 30_000, 10, seed=1, values="scaled100", test_frac=0)
    assert s.val.min() >= 0 and s.val.max() <= 100


def test_init_factors_range():
    W, H = synth.init_factors(100, 50, 16, 7)
    assert W.shape == (100, 16) and H.shape == (50, 16)
    assert W.min() >= 0 and W.max() < 1 / math.sqrt(16)
    assert abs(W.double().mean().item() - 0.5 / 4) < 0.01


def test_batched_specs():
    specs = synth.batched_specs()
    assert len(specs) == 256
    for s in specs:
        assert 1000 <= s["m"] <= 200_000 and 500 <= s["n"] <= 20_000
        assert s["nnz"] <= s["m"] * s["n"] // 2
        assert s["k"] in (16, 32, 64) and s["lam"] in (0.01, 0.05, 0.1)
    total = sum(s["nnz"] for s in specs)
    assert 1e8 < total < 5e8
    ks = np.array([s["k"] for s in specs])
    assert (ks == 16).any() and (ks == 32).any() and (ks == 64).any()
