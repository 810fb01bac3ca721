"""Dynamic load balancing (section 3.3) under the asynchronous schedules on the GPU: the
next worker is the less loaded of two candidates, a worker's load being the items waiting
in its inbound queue.

Which candidate wins depends on queue lengths at the moment of the hand-off, so the serial
order is checked through the trace (every holder still visited once per epoch under the
random permutation; replay in the oracle reproduces the factors) and the result
statistically against the oracle's emulation of the same rule (test RMSE on the tiny
workload after 100 epochs within 1e-3, for uniform routing within 1e-3 of the band its
timings span, as for the unbalanced schedules)."""
import numpy as np
import pytest
import torch

import oracle
import paper_1312_0193_amd as nm
import synth
from parity import check, max_updates
from test_gpu_perm import RMSE_EPOCHS, RMSE_TOL, UNIFORM_TIMINGS, holders, make, tiny_setup

pytestmark = pytest.mark.gpu


def replay_check(prob, W0, H0, hp, P, seed, tr, W, H, E):
    order = np.argsort(tr[:, 0], kind="stable")
    t2 = tr[order]
    Wr, Hr, _ = oracle.replay(prob.m, prob.n, prob.row.numpy(), prob.col.numpy(), prob.val.numpy(), W0.numpy(),
                              H0.numpy(), hp, P, seed, t2[:, 0], t2[:, 1], t2[:, 2], t2[:, 3])
    T = max_updates(prob.row.numpy(), prob.col.numpy(), E)
    check(W, Wr, norm_tol=2e-5, updates=T, what="W")
    check(H, Hr, norm_tol=2e-5, updates=T, what="H")


def item_orders(tr):
    """{(item, epoch): workers in visiting order} from a permutation-schedule trace."""
    tr = tr[np.lexsort((tr[:, 3], tr[:, 1]))]
    out = {}
    for (j, e) in {(int(a), int(b)) for a, b in tr[:, 1:3]}:
        sel = (tr[:, 1] == j) & (tr[:, 2] == e)
        out[(j, e)] = tuple(int(x) for x in tr[sel, 0])
    return out


@pytest.mark.parametrize("case", [
    # m, n, nnz, k, P, degrees
    (2_000, 1_000, 60_000, 100, 32, "zipf"),
    (600, 300, 12_000, 16, 6, "uniform"),
])
def test_balanced_perm_visits_every_holder_once_per_epoch_and_replays(case):
    m, n, nnz, k, P, degrees = case
    prob, W0, H0, hp = make(m, n, nnz, k=k, seed=m + P + 1, degrees=degrees)
    E, seed = 3, 5
    print(f"[case] balanced perm m={m} n={n} nnz={nnz} k={k} P={P}", flush=True)
    runs = {}
    for bal in (False, True):
        model = nm.Nomad(prob.m, prob.n, prob.row, prob.col, prob.val, W0, H0, k=hp.k, lam=hp.lam, alpha=hp.alpha,
                         beta=hp.beta, gamma=hp.gamma, workers=P, seed=seed, sched="perm", record_trace=True,
                         balance=bal, collect_stats=True, debug_ownership=True)
        st = model.train(E)
        tr = model.trace()
        W, H = (x.cpu().double().numpy() for x in model.factors())
        model.close()
        assert st.violations == 0
        runs[bal] = (st, tr, W, H)
    st, tr, W, H = runs[True]
    vis = holders(prob, P)
    assert st.updates == E * prob.nnz
    assert len(tr) == E * len(vis)
    for e in range(E):
        got = sorted((int(a), int(b)) for a, b in tr[tr[:, 2] == e][:, :2])
        assert got == sorted(vis), e  # each (worker, item) exactly once in epoch e
    # the rule changed some visiting orders (without it an item's order in an epoch is fixed
    # by seed, item and epoch)
    o_plain, o_bal = item_orders(runs[False][1]), item_orders(tr)
    assert o_plain.keys() == o_bal.keys()
    changed = sum(o_plain[key] != o_bal[key] for key in o_plain)
    print(f"[parity] balanced perm: {changed} of {len(o_plain)} (item, epoch) orders differ from the plain order",
          flush=True)
    if P > 8:
        assert changed > 0
    replay_check(prob, W0, H0, hp, P, seed, tr, W, H, E)


def test_balanced_uniform_trace_replays():
    prob, W0, H0, hp = make(700, 250, 14_000, k=32, seed=41)
    P, seed, E = 12, 6, 2
    print("[case] balanced uniform routing", flush=True)
    model = nm.Nomad(prob.m, prob.n, prob.row, prob.col, prob.val, W0, H0, k=hp.k, lam=hp.lam, alpha=hp.alpha,
                     beta=hp.beta, gamma=hp.gamma, workers=P, seed=seed, sched="uniform", record_trace=True,
                     balance=True, debug_ownership=True)
    st = model.train(E)
    tr = model.trace()
    W, H = (x.cpu().double().numpy() for x in model.factors())
    model.close()
    assert st.updates >= E * prob.nnz and st.violations == 0
    assert {(int(a), int(b)) for a, b in tr[:, :2]} <= holders(prob, P)
    replay_check(prob, W0, H0, hp, P, seed, tr, W, H, 2 * E)


def test_balanced_perm_rmse_matches_oracle_emulation():
    prob, W0, H0, hp, zero = tiny_setup()
    P, E = 16, RMSE_EPOCHS
    print("[case] balanced perm, tiny workload", flush=True)
    model = nm.Nomad(prob.m, prob.n, prob.row, prob.col, prob.val, W0, H0, k=hp.k, lam=hp.lam, alpha=hp.alpha,
                     beta=hp.beta, gamma=hp.gamma, workers=P, seed=1, sched="perm", balance=True)
    model.train(E)
    r_gpu, _ = model.evaluate(prob.test_row, prob.test_col, prob.test_val)
    model.close()
    Wo, Ho, _ = oracle.train_perm(prob.m, prob.n, prob.row.numpy(), prob.col.numpy(), prob.val.numpy(), W0.numpy(),
                                  H0.numpy(), hp, P, 1, E, 77, balance=True)
    r_orc = oracle.rmse(prob.m, prob.n, prob.test_row.numpy(), prob.test_col.numpy(), prob.test_val.numpy(), Wo, Ho)
    print(f"[parity] balanced perm test RMSE after {E} epochs: gpu {r_gpu:.6f}, oracle emulation {r_orc:.6f}, "
          f"zero predictor {zero:.6f}", flush=True)
    assert r_orc < 0.45 * zero
    assert abs(r_gpu - r_orc) < RMSE_TOL, (r_gpu, r_orc)


def test_balanced_uniform_rmse_matches_oracle_emulation():
    prob, W0, H0, hp, zero = tiny_setup()
    P, E = 16, RMSE_EPOCHS
    print("[case] balanced uniform routing, tiny workload", flush=True)
    model = nm.Nomad(prob.m, prob.n, prob.row, prob.col, prob.val, W0, H0, k=hp.k, lam=hp.lam, alpha=hp.alpha,
                     beta=hp.beta, gamma=hp.gamma, workers=P, seed=1, sched="uniform", balance=True)
    st = model.train(E)
    r_gpu, _ = model.evaluate(prob.test_row, prob.test_col, prob.test_val)
    model.close()
    band = []
    for timing in UNIFORM_TIMINGS:
        Wo, Ho, _ = oracle.train_uniform(prob.m, prob.n, prob.row.numpy(), prob.col.numpy(), prob.val.numpy(),
                                         W0.numpy(), H0.numpy(), hp, P, 1, st.updates, 77, balance=True,
                                         timing=timing)
        band.append(oracle.rmse(prob.m, prob.n, prob.test_row.numpy(), prob.test_col.numpy(), prob.test_val.numpy(),
                                Wo, Ho))
    lo, hi = min(band), max(band)
    print(f"[parity] balanced uniform test RMSE after {st.updates} updates: gpu {r_gpu:.6f}, oracle emulations "
          f"[{lo:.6f}, {hi:.6f}], zero predictor {zero:.6f}", flush=True)
    assert hi < 0.45 * zero
    assert lo - RMSE_TOL < r_gpu < hi + RMSE_TOL, (r_gpu, band)


def test_balance_needs_an_asynchronous_schedule():
    prob, W0, H0, hp = make(200, 100, 2_000, k=8, seed=43)
    with pytest.raises(nm.NomadError) as ei:
        nm.Nomad(prob.m, prob.n, prob.row, prob.col, prob.val, W0, H0, k=hp.k, lam=hp.lam, alpha=hp.alpha,
                 beta=hp.beta, gamma=hp.gamma, workers=4, sched="ring", balance=True)
    assert "balance" in str(ei.value)
