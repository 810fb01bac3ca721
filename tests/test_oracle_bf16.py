"""Pins of the oracle's bfloat16 storage form (the BF16 configuration of the benchmark).

The trajectory itself has no closed form ("parity unpinned" beyond these pins); what is
pinned here is every primitive it is built from, each against something other than the
oracle: nearest-even rounding against torch's own float32 -> bfloat16 conversion,
stochastic rounding against its defining properties (one of the two neighbours, the
expected value is the input), and the training loop against a serial SGD loop written
out with torch's rounding for p = 1 (textbook order, as in the p = 1 pin of the FP64 form).
"""
import numpy as np
import pytest
import torch

import oracle


def torch_bf16(x: np.ndarray) -> np.ndarray:
    """float64 -> float32 (nearest) -> bfloat16 (torch: nearest-even) -> float64."""
    return torch.from_numpy(np.asarray(x, dtype=np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def test_rne_matches_torch_conversion():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 1, 3000), rng.normal(0, 1e-3, 1000), rng.uniform(-100, 100, 1000)])
    # exact ties: a bfloat16 value plus half a bfloat16 ulp (representable in FP32)
    b = torch_bf16(rng.normal(0, 1, 500))
    ties = b + np.ldexp(1.0, (np.floor(np.log2(np.abs(b))) - 8).astype(int)) * np.sign(b)
    x = np.concatenate([x, ties, -ties])
    got = np.array([oracle.round_bf16(v, 0) for v in x])
    assert np.array_equal(got, torch_bf16(x))


def test_rne_ties_go_to_even():
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7: nearest-even keeps 1.
    assert oracle.round_bf16(1.0 + 2.0 ** -8, 0) == 1.0
    # 1 + 3 * 2^-8 lies halfway between 1 + 2^-7 (odd mantissa) and 1 + 2^-6: goes up.
    assert oracle.round_bf16(1.0 + 3 * 2.0 ** -8, 0) == 1.0 + 2.0 ** -6
    assert oracle.round_bf16(-(1.0 + 2.0 ** -8), 0) == -1.0


def test_stochastic_rounding_neighbours_and_mean():
    rng = np.random.default_rng(1)
    for x in [0.3, -1.7, 1e-3, 123.456]:
        lo = float(torch_bf16(np.array([x]))[0])
        # the two bfloat16 neighbours of x
        f32 = np.float32(x)
        u = f32.view(np.uint32) & np.uint32(0xFFFF0000)
        down = float(u.view(np.float32))
        up = float((u + np.uint32(0x10000)).view(np.float32))
        vals = np.array([oracle.round_bf16(x, 1, int(b)) for b in rng.integers(0, 1 << 16, 4000)])
        assert set(np.unique(vals)) <= {down, up}
        assert lo in (down, up)
        frac = (float(f32) - down) / (up - down)
        p_up = np.mean(vals == up)
        assert abs(p_up - frac) < 4 * np.sqrt(frac * (1 - frac) / vals.size) + 1e-3
    # bits 0 truncates the magnitude; bits 0xFFFF rounds any inexact value away from zero
    assert oracle.round_bf16(1.0 + 2.0 ** -9, 1, 0) == 1.0
    assert oracle.round_bf16(1.0 + 2.0 ** -20, 1, 0xFFFF) == 1.0 + 2.0 ** -7
    assert oracle.round_bf16(1.0, 1, 0xFFFF) == 1.0


def test_rounding_bits_are_spread():
    # 16-bit values over many counters: every 8-bit bucket of the top byte is hit about
    # equally often (chi-square well below its 0.1% point for 255 degrees of freedom).
    vals = np.array([oracle.sr_bits(7, i, j, t, l) for i in range(20) for j in range(5) for t in range(3)
                     for l in range(20)])
    assert vals.max() < (1 << 16)
    counts = np.bincount(vals >> 8, minlength=256)
    expected = vals.size / 256
    chi2 = ((counts - expected) ** 2 / expected).sum()
    assert chi2 < 330
    # a change of any counter changes the bits
    base = oracle.sr_bits(7, 3, 4, 5, 6)
    assert len({base, oracle.sr_bits(8, 3, 4, 5, 6), oracle.sr_bits(7, 2, 4, 5, 6), oracle.sr_bits(7, 3, 5, 5, 6),
                oracle.sr_bits(7, 3, 4, 4, 6), oracle.sr_bits(7, 3, 4, 5, 7)}) == 6


def small_problem(seed=3, m=40, n=25, nnz=300, k=6):
    rng = np.random.default_rng(seed)
    cells = rng.choice(m * n, size=nnz, replace=False)
    row, col = (cells // n).astype(np.int32), (cells % n).astype(np.int32)
    val = rng.normal(3, 1, nnz).astype(np.float32)
    W0 = rng.uniform(0, 1 / np.sqrt(k), (m, k)).astype(np.float32)
    H0 = rng.uniform(0, 1 / np.sqrt(k), (n, k)).astype(np.float32)
    return m, n, row, col, val, W0, H0


@pytest.mark.parametrize("rounding", [0, 1])
def test_single_worker_is_serial_sgd_with_bf16_stores(rounding):
    """p = 1: the ring order is items ascending, rows ascending (the p = 1 reduction).
    Written out with torch's rounding for nearest-even; the stochastic form takes its bits
    from the counter hash and applies the defining truncation.  The dot product is summed
    in element order, as a plain loop does."""
    m, n, row, col, val, W0, H0 = small_problem()
    k = W0.shape[1]
    hp = oracle.Hyper(k, 0.05, 0.05, 0.1, 1.0)
    W, H, _ = oracle.train_ring_bf16(m, n, row, col, val, W0, H0, hp, 1, 11, 2, rounding, 99)
    Wr = torch_bf16(W0.astype(np.float64))
    Hr = H0.astype(np.float64).copy()
    order = np.lexsort((row, col))
    for t in range(2):
        s = hp.alpha / (1 + hp.beta * t ** hp.gamma)
        for e in order:
            i, j, r = row[e], col[e], float(val[e])
            w, h = Wr[i].copy(), Hr[j].copy()
            d = 0.0
            for l in range(k):
                d += w[l] * h[l]
            err = r - d
            wn = w + s * (err * h - hp.lam * w)
            Hr[j] = h + s * (err * w - hp.lam * h)
            if rounding == 0:
                Wr[i] = torch_bf16(wn)
            else:
                f = wn.astype(np.float32).view(np.uint32).astype(np.uint64)
                bits = np.array([oracle.sr_bits(99, i, j, t, l) for l in range(k)], dtype=np.uint64)
                Wr[i] = (((f + bits) & 0xFFFF0000).astype(np.uint32)).view(np.float32).astype(np.float64)
    assert np.array_equal(W, Wr)
    assert np.array_equal(H, Hr)


def test_stored_rows_are_bfloat16_and_close_to_fp64():
    m, n, row, col, val, W0, H0 = small_problem(seed=5, m=60, n=30, nnz=600, k=8)
    hp = oracle.Hyper(8, 0.05, 0.02, 0.0, 1.0)
    Wb, Hb, st = oracle.train_ring_bf16(m, n, row, col, val, W0, H0, hp, 3, 4, 1, 1, 5)
    assert st.updates == row.size
    assert np.array_equal(Wb, torch_bf16(Wb))
    Wd, Hd, _ = oracle.train_ring(m, n, row, col, val, W0, H0, hp, 3, 4, 1)
    # one epoch: bfloat16 keeps 8 significant bits, so rows differ by about 2^-9 relative
    assert np.linalg.norm(Wb - Wd) / np.linalg.norm(Wd) < 1e-2
    assert np.linalg.norm(Hb - Hd) / np.linalg.norm(Hd) < 1e-2
