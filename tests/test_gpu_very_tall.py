"""The very tall configuration (Hugewiki-shaped: 50,000,000 x 39,780, 2.74 B Zipf cells,
real ratings x + N(0, 0.1^2) of planted rank 50, k = 100, lambda = 0.01, alpha = 0.001,
beta = 0) on its first row block: rows 0 .. 3,124,999 with all their cells (171 M, a
sixteenth of the matrix; the generator draws the matrix block by block), where the FP64
oracle fits: one ring epoch with 256 workers.
  * FP32: within 1e-5 normwise and the per-vector rounding bound of the oracle; test RMSE
    within 1e-6 relative;
  * BF16 storage of W (stochastic rounding, the form the configuration names): test RMSE
    within 1e-3 relative of the oracle's BF16 form and within 0.5% of the FP64 oracle.
The full-size run (throughput, 64-bit layout offsets) is the benchmark's very_tall
workload."""
import numpy as np
import pytest
import torch

import oracle
import paper_1312_0193_amd as nm
import synth
from parity import check, max_updates, rel

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]


@pytest.fixture(scope="module")
def sample():
    print("[case] very tall workload, first row block: generating on the GPU", flush=True)
    prob = synth.very_tall(device="cuda", blocks=1)
    hpd = prob.hp
    W0, H0 = synth.init_factors(prob.m, prob.n, hpd["k"], 5, device="cuda")
    f = lambda x: float(np.float32(x))  # noqa: E731
    hp = oracle.Hyper(hpd["k"], f(hpd["lam"]), f(hpd["alpha"]), f(hpd["beta"]), f(hpd["gamma"]))
    host = dict(row=prob.row.cpu().numpy(), col=prob.col.cpu().numpy(), val=prob.val.cpu().numpy(),
                W0=W0.cpu().numpy(), H0=H0.cpu().numpy(), trow=prob.test_row.cpu().numpy(),
                tcol=prob.test_col.cpu().numpy(), tval=prob.test_val.cpu().numpy())
    print(f"[case] very tall, first row block: {prob.m} x {prob.n}, {prob.nnz} training and {prob.test_row.numel()} test "
          f"ratings; heaviest column {int(np.bincount(host['col']).max())}", flush=True)
    return prob, W0, H0, hp, host


@pytest.fixture(scope="module")
def oracle_epoch(sample):
    prob, W0, H0, hp, h = sample
    print("[case] oracle ring order, one epoch, FP64", flush=True)
    oracle.set_progress(20_000_000)
    Wo, Ho, _ = oracle.train_ring(prob.m, prob.n, h["row"], h["col"], h["val"], h["W0"], h["H0"], hp, 256, 5, 1)
    oracle.set_progress(0)
    r = oracle.rmse(prob.m, prob.n, h["trow"], h["tcol"], h["tval"], Wo, Ho)
    r0 = oracle.rmse(prob.m, prob.n, h["trow"], h["tcol"], h["tval"], h["W0"], h["H0"])
    print(f"[case] oracle test RMSE {r:.6f} (initial {r0:.6f})", flush=True)
    return Wo, Ho, r, r0


def gpu_epoch(prob, W0, H0, hp, **kw):
    model = nm.Nomad(prob.m, prob.n, prob.row, prob.col, prob.val, W0, H0, k=hp.k, lam=hp.lam, alpha=hp.alpha,
                     beta=hp.beta, gamma=hp.gamma, workers=256, seed=5, **kw)
    st = model.train(1)
    r, _ = model.evaluate(prob.test_row, prob.test_col, prob.test_val)
    W, H = (x.cpu().double().numpy() for x in model.factors())
    model.close()
    return W, H, r, st


def test_very_tall_fp32_one_ring_epoch_matches_oracle(sample, oracle_epoch):
    prob, W0, H0, hp, h = sample
    Wo, Ho, r_o, r0 = oracle_epoch
    print("[case] very tall 1/16, FP32, ring, 256 workers", flush=True)
    W, H, r, st = gpu_epoch(prob, W0, H0, hp)
    assert st.updates == prob.nnz
    T = max_updates(h["row"], h["col"], 1)
    check(W, Wo, norm_tol=1e-5, updates=T, what="very tall W")
    check(H, Ho, norm_tol=1e-5, updates=T, what="very tall H")
    print(f"[parity] very tall FP32 test RMSE {r:.6f}, oracle {r_o:.6f} (initial {r0:.6f})", flush=True)
    assert r < r0
    assert abs(r - r_o) <= 1e-6 * r_o


def test_very_tall_bf16_one_ring_epoch_against_oracle(sample, oracle_epoch):
    prob, W0, H0, hp, h = sample
    _, _, r64, _ = oracle_epoch
    print("[case] very tall 1/16, BF16 W (stochastic), ring, 256 workers", flush=True)
    W, H, r, _ = gpu_epoch(prob, W0, H0, hp, dtype="bf16", rounding="stochastic")
    assert np.all((W.astype(np.float32).view(np.uint32) & 0xFFFF) == 0)
    oracle.set_progress(20_000_000)
    Wb, Hb, _ = oracle.train_ring_bf16(prob.m, prob.n, h["row"], h["col"], h["val"], h["W0"], h["H0"], hp, 256, 5, 1,
                                       1, 5)
    oracle.set_progress(0)
    rbo = oracle.rmse(prob.m, prob.n, h["trow"], h["tcol"], h["tval"], Wb, Hb)
    gap = (r - r64) / r64
    print(f"[parity] very tall bf16: normwise W {rel(W, Wb):.2e} H {rel(H, Hb):.2e}; test RMSE gpu {r:.6f}, oracle "
          f"BF16 form {rbo:.6f}, FP64 {r64:.6f} (gap {gap:+.2e})", flush=True)
    assert abs(r - rbo) <= 1e-3 * rbo
    assert abs(gap) < 5e-3
