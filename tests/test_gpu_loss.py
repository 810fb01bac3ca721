"""The logistic loss (section 2: the method takes any separable loss) on the GPU: labels
+-1, residual e = r / (1 + exp(r d)) in FP32 with the fast exponential.

  * ring order against the FP64 oracle's ring order with the same loss: within 1e-5
    normwise and the per-vector rounding bound after two epochs (the fast exponential is
    within a few units in the last place, inside the bound's slack);
  * random permutation: the recorded trace replayed in the oracle with the same loss;
  * the objective J with the logistic loss against the oracle's (FP64 sums, 1e-12);
  * BF16 storage: classification accuracy on held-out labels within 1% of FP32;
  * batches use the square loss only (ENOTIMPL)."""
import numpy as np
import pytest

import oracle
import paper_1312_0193_amd as nm
import synth
from parity import check, max_updates

pytestmark = pytest.mark.gpu


def setup(m, n, nnz, k, seed, degrees="uniform"):
    prob = synth.small_case(m, n, nnz, seed=seed, degrees=degrees, k=k, rank=3, values="sign", test_frac=0.1)
    W0, H0 = synth.init_factors(m, n, k, seed)
    f = lambda x: float(np.float32(x))  # noqa: E731
    hp = oracle.Hyper(k, f(0.01), f(0.1), f(0.01), f(1.0))
    return prob, W0, H0, hp


def model(prob, W0, H0, hp, P, **kw):
    return nm.Nomad(prob.m, prob.n, prob.row, prob.col, prob.val, W0, H0, k=hp.k, lam=hp.lam, alpha=hp.alpha,
                    beta=hp.beta, gamma=hp.gamma, workers=P, seed=3, loss="logistic", **kw)


def accuracy(prob, W, H):
    d = np.einsum("ij,ij->i", W[prob.test_row.numpy()], H[prob.test_col.numpy()])
    return float(np.mean(np.sign(d) == prob.test_val.numpy()))


@pytest.mark.parametrize("case", [
    # m, n, nnz, k, P, degrees
    (1_500, 900, 60_000, 32, 16, "uniform"),
    (2_000, 1_000, 80_000, 100, 32, "zipf"),
])
def test_logistic_ring_matches_oracle(case):
    m, n, nnz, k, P, degrees = case
    prob, W0, H0, hp = setup(m, n, nnz, k, m + P, degrees)
    E = 2
    print(f"[case] logistic ring m={m} n={n} nnz={nnz} k={k} P={P}", flush=True)
    mdl = model(prob, W0, H0, hp, P)
    st = mdl.train(E)
    W, H = (x.cpu().double().numpy() for x in mdl.factors())
    _, J = mdl.evaluate(prob.row, prob.col, prob.val)
    mdl.close()
    assert st.updates == E * prob.nnz
    Wo, Ho, _ = oracle.train_ring(m, n, prob.row.numpy(), prob.col.numpy(), prob.val.numpy(), W0.numpy(), H0.numpy(),
                                  hp, P, 3, E, loss="logistic")
    T = max_updates(prob.row.numpy(), prob.col.numpy(), E)
    check(W, Wo, norm_tol=1e-5, updates=T, what="W (logistic)")
    check(H, Ho, norm_tol=1e-5, updates=T, what="H (logistic)")
    # the objective with the logistic loss, evaluated by the library (FP64) and the oracle
    Jo = oracle.objective(m, n, prob.row.numpy(), prob.col.numpy(), prob.val.numpy(), W, H, hp.lam, loss="logistic")
    assert J == pytest.approx(Jo, rel=1e-12)
    J0 = oracle.objective(m, n, prob.row.numpy(), prob.col.numpy(), prob.val.numpy(), W0.numpy(), H0.numpy(), hp.lam,
                          loss="logistic")
    print(f"[parity] logistic J {J0:.2f} -> {J:.2f}, held-out accuracy {accuracy(prob, W, H):.3f}", flush=True)
    assert J < J0


def test_logistic_perm_trace_replays():
    prob, W0, H0, hp = setup(1_200, 700, 50_000, 64, 17)
    P, E = 24, 3
    print("[case] logistic perm, trace replay", flush=True)
    mdl = model(prob, W0, H0, hp, P, sched="perm", record_trace=True)
    mdl.train(E)
    tr = mdl.trace()
    W, H = (x.cpu().double().numpy() for x in mdl.factors())
    mdl.close()
    t2 = tr[np.argsort(tr[:, 0], kind="stable")]
    Wr, Hr, _ = oracle.replay(prob.m, prob.n, prob.row.numpy(), prob.col.numpy(), prob.val.numpy(), W0.numpy(),
                              H0.numpy(), hp, P, 3, t2[:, 0], t2[:, 1], t2[:, 2], t2[:, 3], loss="logistic")
    T = max_updates(prob.row.numpy(), prob.col.numpy(), E)
    check(W, Wr, norm_tol=2e-5, updates=T, what="W (logistic replay)")
    check(H, Hr, norm_tol=2e-5, updates=T, what="H (logistic replay)")


def test_logistic_bf16_classifies_like_fp32():
    prob, W0, H0, hp = setup(3_000, 2_000, 300_000, 16, 23)
    acc = {}
    for dt in ("fp32", "bf16"):
        kw = dict(dtype=dt, rounding="stochastic") if dt == "bf16" else {}
        mdl = model(prob, W0, H0, hp, 32, sched="perm", **kw)
        mdl.train(15)
        W, H = (x.cpu().double().numpy() for x in mdl.factors())
        mdl.close()
        acc[dt] = accuracy(prob, W, H)
    print(f"[parity] logistic held-out accuracy: fp32 {acc['fp32']:.4f}, bf16 {acc['bf16']:.4f}", flush=True)
    assert acc["fp32"] > 0.8
    assert abs(acc["bf16"] - acc["fp32"]) < 0.01


def test_logistic_not_in_batches():
    prob, W0, H0, hp = setup(200, 300, 3_000, 8, 9)
    d = dict(m=prob.m, n=prob.n, row=prob.row, col=prob.col, val=prob.val, W0=W0, H0=H0, k=8, lam=hp.lam,
             alpha=hp.alpha, beta=hp.beta, gamma=hp.gamma)
    with pytest.raises(nm.NomadError):
        nm.NomadBatch([d, d], loss="logistic")
