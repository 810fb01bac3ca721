"""Parity at the full size of the medium workload (480,189 x 17,770, 98.6 M training
ratings, Zipf degrees, k = 100), in the launch configuration the benchmark times.

At this size the oracle still takes the whole epoch (about a minute of FP64 on one core),
so the checks are the exact ones:
  * the row partition equals the oracle's;
  * random-permutation schedule (the benchmark's): the recorded trace shows every
    (worker, item) pair that shares ratings exactly once, each item's visits numbered
    consecutively, every rating updated once; replaying the trace in the oracle
    reproduces the GPU factors within the one-epoch FP32 tolerance;
  * ring schedule: one epoch equals the oracle's ring order within the same tolerance,
    and the factors do not depend on the number of compute waves (bitwise);
  * FP64 evaluation of the GPU factors equals the oracle's to 1e-12.

The tolerance is the one-epoch FP32 bound, 1e-5 relative (Frobenius norm) for W and for H,
and per vector the probabilistic rounding bound of the busiest variable (the heaviest
column takes about 473,000 updates in sequence); the per-column errors and those of the
heaviest columns are printed beside it.  The ownership invariant is checked on the device
for all three schedules (zero violations, hand-offs counted), and the benchmark's test
RMSE after six random-permutation epochs is compared with the oracle's emulations of the
same schedule (tests/golden/medium_perm_rmse.json, three scheduler seeds).  The benchmark
trains one epoch per call, and a launch ends only when every item has finished its epochs,
so items stay within an epoch of each other as in the emulation: its RMSE must lie within
1e-3 (the asynchronous criterion) of the band the emulations span.  Six epochs in one call
let light items run epochs ahead of the heaviest (a chain of 473,267 updates per epoch
that lasts about as long as the epoch): that RMSE is about 0.7% higher and is held within
1e-2.
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import paper_1312_0193_amd as nm
import synth
from parity import elem_error, elem_tolerance, floored_rel, max_updates

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

TOL_1EPOCH = 1e-5


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def check_factors(tag, W, H, Wo, Ho, col):
    deg = np.bincount(col, minlength=H.shape[0])
    ew, eh = rel(W, Wo), rel(H, Ho)
    per = np.linalg.norm(H - Ho, axis=1) / np.maximum(np.linalg.norm(Ho, axis=1), 1e-300)
    top = np.argsort(deg)[-3:]
    worst = np.argsort(per)[-5:]
    perw = np.linalg.norm(W - Wo, axis=1) / np.maximum(np.linalg.norm(Wo, axis=1), 1e-300)
    print(f"[case] {tag}: rel err W {ew:.2e}, H {eh:.2e}; "
          f"heaviest columns (ratings, rel err): " + ", ".join(f"({deg[j]}, {per[j]:.1e})" for j in top), flush=True)
    print(f"[case] {tag}: per-column rel err quantiles 50/90/99/100%: "
          + " ".join(f"{x:.1e}" for x in np.quantile(per, [0.5, 0.9, 0.99, 1.0]))
          + "; worst columns (ratings, err, norm): " + ", ".join(f"({deg[j]}, {per[j]:.1e}, {np.linalg.norm(Ho[j]):.2f})" for j in worst)
          + "; per-row W rel err quantiles 50/99/100%: " + " ".join(f"{x:.1e}" for x in np.quantile(perw, [0.5, 0.99, 1.0])),
          flush=True)
    assert ew < TOL_1EPOCH and eh < TOL_1EPOCH, (ew, eh)
    T = max_updates(np.zeros(1, dtype=np.int64), col, 1)
    tol = elem_tolerance(T)
    xw, xh = elem_error(W, Wo), elem_error(H, Ho)
    print(f"[parity] {tag}: per-vector max W {xw:.2e} H {xh:.2e} (<= {tol:.2e}, {T} updates of the busiest "
          f"column); floored rel W {floored_rel(W, Wo):.2e} H {floored_rel(H, Ho):.2e}", flush=True)
    assert xw <= tol and xh <= tol, (xw, xh, tol)


@pytest.fixture(scope="module")
def medium():
    print("[case] medium workload: generating on the GPU", flush=True)
    prob = synth.medium(device="cuda")
    hpd = prob.hp
    W0, H0 = synth.init_factors(prob.m, prob.n, hpd["k"], 2, device="cuda")
    f = lambda x: float(np.float32(x))  # noqa: E731
    hp = oracle.Hyper(hpd["k"], f(hpd["lam"]), f(hpd["alpha"]), f(hpd["beta"]), f(hpd["gamma"]))
    host = dict(row=prob.row.cpu().numpy(), col=prob.col.cpu().numpy(), val=prob.val.cpu().numpy(),
                W0=W0.cpu().numpy(), H0=H0.cpu().numpy(), test_row=prob.test_row.cpu().numpy(),
                test_col=prob.test_col.cpu().numpy(), test_val=prob.test_val.cpu().numpy())
    return prob, W0, H0, hp, host


def model(prob, W0, H0, hp, **kw):
    return nm.Nomad(prob.m, prob.n, prob.row, prob.col, prob.val, W0, H0, k=hp.k, lam=hp.lam, alpha=hp.alpha,
                    beta=hp.beta, gamma=hp.gamma, seed=2, **kw)


def test_medium_perm_trace_replays_in_oracle(medium):
    prob, W0, H0, hp, host = medium
    print("[case] medium, random-permutation schedule, one epoch with the visit trace", flush=True)
    mdl = model(prob, W0, H0, hp, sched="perm", record_trace=True, collect_stats=True)
    P = mdl.workers
    rs = mdl.partition()
    assert np.array_equal(rs, oracle.partition(prob.m, host["row"], P))
    st = mdl.train(1)
    assert st.updates == prob.nnz
    tr = mdl.trace()
    ws = mdl.worker_stats()
    W, H = (x.cpu().double().numpy() for x in mdl.factors())
    r_gpu, _ = mdl.evaluate(prob.test_row, prob.test_col, prob.test_val)
    mdl.close()
    assert int(ws[:, 6].sum()) == prob.nnz
    # every (worker, item) pair sharing ratings exactly once
    q_of = (np.searchsorted(rs, host["row"], "right") - 1).astype(np.int64)
    pairs = np.unique(q_of * prob.n + host["col"].astype(np.int64))
    got = np.sort(tr[:, 0].astype(np.int64) * prob.n + tr[:, 1].astype(np.int64))
    assert got.size == pairs.size and np.array_equal(got, pairs)
    # each item's visits numbered 0, 1, 2, ... in its order
    order = np.lexsort((tr[:, 3], tr[:, 1]))
    seq = tr[order, 3]
    starts = np.r_[0, np.flatnonzero(np.diff(tr[order, 1])) + 1]
    expect = np.arange(seq.size) - np.repeat(starts, np.diff(np.r_[starts, seq.size]))
    assert np.array_equal(seq, expect)
    print(f"[case] replaying {len(tr)} visits in the oracle", flush=True)
    t2 = tr[np.argsort(tr[:, 0], kind="stable")]
    Wr, Hr, _ = oracle.replay(prob.m, prob.n, host["row"], host["col"], host["val"], host["W0"], host["H0"], hp, P, 2,
                              t2[:, 0], t2[:, 1], t2[:, 2], t2[:, 3])
    check_factors("replay", W, H, Wr, Hr, host["col"])
    r_orc = oracle.rmse(prob.m, prob.n, host["test_row"], host["test_col"], host["test_val"], W, H)
    assert abs(r_gpu - r_orc) <= 1e-12 * r_orc


def test_medium_ring_matches_oracle_and_wave_count(medium):
    prob, W0, H0, hp, host = medium
    print("[case] medium, ring schedule, one epoch (8 and 4 compute waves)", flush=True)
    mdl = model(prob, W0, H0, hp, sched="ring")
    P = mdl.workers
    mdl.train(1)
    W, H = (x.cpu().double().numpy() for x in mdl.factors())
    mdl.close()
    mdl = model(prob, W0, H0, hp, sched="ring", workers=P, waves_per_worker=4)
    mdl.train(1)
    W4, H4 = (x.cpu().double().numpy() for x in mdl.factors())
    mdl.close()
    assert np.array_equal(W, W4) and np.array_equal(H, H4)
    print("[case] oracle ring order, one epoch", flush=True)
    Wo, Ho, _ = oracle.train_ring(prob.m, prob.n, host["row"], host["col"], host["val"], host["W0"], host["H0"], hp,
                                  P, 2, 1)
    check_factors("ring", W, H, Wo, Ho, host["col"])


@pytest.mark.parametrize("sched", ["ring", "perm", "uniform"])
def test_medium_ownership_holds_on_the_device(medium, sched):
    """Section 3.1's invariant at the full size: no item taken over while held elsewhere,
    none released by a worker that does not hold it, no rating updated by a wave that does
    not own its row; every visit hands its item on except each item's last."""
    prob, W0, H0, hp, host = medium
    print(f"[case] medium, {sched}, one epoch with ownership checks", flush=True)
    mdl = model(prob, W0, H0, hp, sched=sched, debug_ownership=True, collect_stats=True)
    P = mdl.workers
    st = mdl.train(1)
    ws = mdl.worker_stats()
    mdl.close()
    rs = oracle.partition(prob.m, host["row"], P)
    q_of = (np.searchsorted(rs, host["row"], "right") - 1).astype(np.int64)
    V = np.unique(q_of * prob.n + host["col"].astype(np.int64)).size
    active = np.unique(host["col"]).size
    print(f"[case] medium {sched}: violations {st.violations}, hops {st.hops}, visits per epoch {V}, "
          f"items {active}", flush=True)
    assert st.violations == 0
    if sched == "uniform":
        assert st.hops == int(ws[:, 2].sum()) - active
    else:
        assert st.hops == V - active


def test_medium_perm_rmse_matches_oracle_emulation(medium):
    """The benchmark's point: test RMSE after six epochs of the random-permutation schedule
    against the oracle's emulation of it (written by tests/golden/make_medium_perm_rmse.py
    from the same generated inputs)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "medium_perm_rmse.json")
    gold = json.load(open(path))
    prob, W0, H0, hp, host = medium
    band = list(gold.get("test_rmse_by_sched_seed", {"": gold["test_rmse"]}).values())
    lo, hi = min(band), max(band)
    res = {}
    for calls in ([1] * gold["epochs"], [gold["epochs"]]):
        mdl = model(prob, W0, H0, hp, sched="perm")
        assert mdl.workers == gold["workers"]
        for e in calls:
            mdl.train(e)
        res[len(calls)], _ = mdl.evaluate(prob.test_row, prob.test_col, prob.test_val)
        mdl.close()
    r, r1 = res[gold["epochs"]], res[1]
    print(f"[parity] medium perm test RMSE after {gold['epochs']} epochs: gpu {r:.6f} (one epoch per call, as the "
          f"benchmark), {r1:.6f} (one call); oracle emulations [{lo:.6f}, {hi:.6f}] "
          f"(initial {gold['initial_test_rmse']:.6f})", flush=True)
    assert r < 0.45 * gold["initial_test_rmse"]  # a learned point
    assert lo - 1e-3 < r < hi + 1e-3
    assert abs(r1 - lo) < 1e-2
