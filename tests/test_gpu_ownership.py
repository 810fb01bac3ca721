"""The ownership invariant of section 3.1 checked on the device (nomad_config.debug_ownership),
the hop counts of nomad_stats, and the global-count reading of t in the step size
(nomad_config.t_source = 1) against the oracle.

Every item has one holder word: a worker claims it when it takes the item over (it must
find it free) and frees it when it passes the item on (it must find its own claim); every
rating a compute wave updates must be of a row that wave owns.  A correct run reports zero
violations under every schedule.
"""
import numpy as np
import pytest

import oracle
import paper_1312_0193_amd as nm
import synth
from parity import check, max_updates

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def make(m, n, nnz, *, k, seed, degrees="uniform", lam=0.05, alpha=0.01, beta=1e-4, gamma=1.0):
    prob = synth.small_case(m, n, nnz, seed=seed, degrees=degrees, k=k, lam=lam, alpha=alpha, beta=beta,
                            gamma=gamma, test_frac=0.1)
    W0, H0 = synth.init_factors(m, n, k, seed)
    f = lambda x: float(np.float32(x))  # noqa: E731
    return prob, W0, H0, oracle.Hyper(k, f(lam), f(alpha), f(beta), f(gamma))


def holders(prob, P):
    row, col = prob.row.numpy(), prob.col.numpy()
    rs = oracle.partition(prob.m, row, P)
    q_of = np.searchsorted(rs, row, "right") - 1
    return {(int(q), int(j)) for q, j in zip(q_of, col)}


@pytest.mark.parametrize("sched", ["ring", "perm", "uniform"])
def test_no_ownership_violations_and_hop_counts(sched):
    prob, W0, H0, hp = make(2_500, 900, 70_000, k=32, seed=7, degrees="zipf")
    P, seed, E = 24, 3, 3
    print(f"[case] ownership {sched} P={P} E={E}", flush=True)
    model = nm.Nomad(prob.m, prob.n, prob.row, prob.col, prob.val, W0, H0, k=hp.k, lam=hp.lam, alpha=hp.alpha,
                     beta=hp.beta, gamma=hp.gamma, workers=P, seed=seed, sched=sched, debug_ownership=True,
                     collect_stats=True)
    st = model.train(E)
    ws = model.worker_stats()
    model.close()
    assert st.violations == 0
    V = len(holders(prob, P))
    active = len(np.unique(prob.col.numpy()))
    if sched in ("ring", "perm"):
        # every visit but an item's last of the call hands the item on
        assert st.hops == E * V - active, (st.hops, E * V, active)
    else:
        # every take-over but an item's first of the call came from a push
        assert st.hops == int(ws[:, 2].sum()) - active


@pytest.mark.parametrize("sched", ["ring", "perm"])
def test_ownership_checks_do_not_change_results(sched):
    """The checks only read and claim the holder words: the ring order's factors are
    bitwise those of a run without them (the asynchronous order depends on timing, so
    there only the counts are compared)."""
    prob, W0, H0, hp = make(800, 300, 16_000, k=16, seed=11)
    out = []
    for dbg in (False, True):
        model = nm.Nomad(prob.m, prob.n, prob.row, prob.col, prob.val, W0, H0, k=hp.k, lam=hp.lam,
                         alpha=hp.alpha, beta=hp.beta, gamma=hp.gamma, workers=8, seed=1, sched=sched,
                         debug_ownership=dbg)
        st = model.train(2)
        W, H = (x.cpu().numpy() for x in model.factors())
        model.close()
        out.append((W, H, st))
    assert out[0][2].hops == out[1][2].hops and out[1][2].violations == 0
    if sched == "ring":
        assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_ring_global_update_count_matches_oracle():
    """t_source = 1: t is the number of updates applied before the visit (ring order, so
    deterministic); one call of two epochs and a second call continue the count."""
    prob, W0, H0, hp = make(1_200, 500, 30_000, k=24, seed=21, alpha=0.02, beta=1e-3, gamma=1.0)
    P, seed = 12, 5
    print("[case] ring, global update count", flush=True)
    model = nm.Nomad(prob.m, prob.n, prob.row, prob.col, prob.val, W0, H0, k=hp.k, lam=hp.lam, alpha=hp.alpha,
                     beta=hp.beta, gamma=hp.gamma, workers=P, seed=seed, t_source="global")
    model.train(2)
    model.train(1)
    W, H = (x.cpu().double().numpy() for x in model.factors())
    model.close()
    Wo, Ho, _ = oracle.train_ring_gcount(prob.m, prob.n, prob.row.numpy(), prob.col.numpy(), prob.val.numpy(),
                                         W0.numpy(), H0.numpy(), hp, P, seed, 3)
    T = max_updates(prob.row.numpy(), prob.col.numpy(), 3)
    check(W, Wo, norm_tol=3e-5, updates=T, what="W")
    check(H, Ho, norm_tol=3e-5, updates=T, what="H")
    # the step falls with the global count: different from the per-pair reading
    Wp, Hp, _ = oracle.train_ring(prob.m, prob.n, prob.row.numpy(), prob.col.numpy(), prob.val.numpy(),
                                  W0.numpy(), H0.numpy(), hp, P, seed, 3)
    assert rel(Wp, Wo) > 1e-3


@pytest.mark.parametrize("sched", ["perm", "uniform"])
def test_async_global_update_count_replays(sched):
    """t_source = 1 under the asynchronous schedules: the trace's t is the global count
    of updates before the visit in the order the visits were taken; replaying the trace
    reproduces the factors, and the counts tile [0, updates)."""
    prob, W0, H0, hp = make(700, 250, 14_000, k=32, seed=31, alpha=0.02, beta=1e-3)
    P, seed, E = 12, 6, 2
    print(f"[case] {sched}, global update count", flush=True)
    model = nm.Nomad(prob.m, prob.n, prob.row, prob.col, prob.val, W0, H0, k=hp.k, lam=hp.lam, alpha=hp.alpha,
                     beta=hp.beta, gamma=hp.gamma, workers=P, seed=seed, sched=sched, t_source="global",
                     record_trace=True)
    st = model.train(E)
    tr = model.trace()
    W, H = (x.cpu().double().numpy() for x in model.factors())
    model.close()
    row, col = prob.row.numpy(), prob.col.numpy()
    rs = oracle.partition(prob.m, row, P)
    q_of = np.searchsorted(rs, row, "right") - 1
    cnt = {}
    for q, j in zip(q_of, col):
        cnt[(int(q), int(j))] = cnt.get((int(q), int(j)), 0) + 1
    ts = np.sort(tr[:, 2])
    sizes = np.array([cnt[(int(a), int(b))] for a, b in tr[np.argsort(tr[:, 2]), :2]])
    assert ts[0] == 0 and np.array_equal(ts[1:], np.cumsum(sizes)[:-1]) and sizes.sum() == st.updates
    order = np.argsort(tr[:, 0], kind="stable")
    t2 = tr[order]
    Wr, Hr, _ = oracle.replay(prob.m, prob.n, row, col, prob.val.numpy(), W0.numpy(), H0.numpy(), hp, P, seed,
                              t2[:, 0], t2[:, 1], t2[:, 2], t2[:, 3])
    T = max_updates(row, col, 2 * E)
    check(W, Wr, norm_tol=2e-5, updates=T, what="W")
    check(H, Hr, norm_tol=2e-5, updates=T, what="H")
