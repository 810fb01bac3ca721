"""Pins of the oracle's schedules that the GPU path is compared against statistically:
the step counter t of uniform routing (per worker-item pair), the next-holder draw of the
random-permutation circulation (uniform among the holders not yet visited in the epoch),
the global-count reading of t, the traces the emulations record, and the threaded
Algorithm 1 run used as the CPU baseline.  Every expected value here is computed by an
independent brute-force loop in the test, never by the oracle (all CPU)."""
import itertools
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import Hyper


def _np(p):
    return (p.row.numpy(), p.col.numpy(), p.val.numpy())


def _small(m=60, n=40, nnz=900, seed=7, degrees="uniform", k=4, lam=0.05, alpha=0.02, beta=0.01, gamma=1.5):
    p = synth.small_case(m, n, nnz, seed=seed, degrees=degrees, k=k, lam=lam, alpha=alpha, beta=beta,
                         gamma=gamma, test_frac=0.0)
    W0, H0 = synth.init_factors(m, n, k, seed)
    return p, W0.numpy(), H0.numpy(), Hyper(k, lam, alpha, beta, gamma)


def _scalar_sgd(w, h, r, s, lam):
    """One SGD step for k = 1, written out (section 2.3's update, simultaneous form)."""
    e = r - w * h
    return w + s * (e * h - lam * w), h + s * (e * w - lam * h)


# ---------------------------------------------------------------- uniform routing: t per pair

def test_uniform_t_counts_earlier_visits_of_the_same_worker_and_item():
    """Two workers, one item, one rating each (k = 1).  The item wanders between the two
    workers at random; a visit's step index t must be the number of earlier visits of the
    item to *that* worker (Algorithm 1's per-(i,j) count), not the item's visit count.
    The expected factors come from a hand-written scalar loop over the visit order."""
    row = np.array([0, 1], dtype=np.int32)
    col = np.array([0, 0], dtype=np.int32)
    val = np.array([2.0, -1.0], dtype=np.float32)
    W0 = np.array([[0.5], [0.25]])
    H0 = np.array([[0.75]])
    hp = Hyper(1, 0.1, 0.2, 1.0, 1.0)  # s_t = 0.2 / (1 + t): strongly t-dependent
    P, seed, sched_seed, budget = 2, 3, 11, 12
    W, H, st, tr = oracle.train_uniform(2, 1, row, col, val, W0, H0, hp, P, seed, budget, sched_seed, trace=True)
    assert st.updates == budget and len(tr) == budget
    qs = tr[:, 0].tolist()
    assert set(qs) == {0, 1}, "the item must visit both workers"
    # t = earlier visits of (q, item 0); the item's own count would differ once it has
    # visited both workers
    seen = {0: 0, 1: 0}
    for x, q in enumerate(qs):
        assert tr[x, 2] == seen[q] and tr[x, 3] == x
        seen[q] += 1
    assert any(tr[x, 2] != x for x in range(len(qs)))
    # replay the visit order by hand
    w = [0.5, 0.25]
    h = 0.75
    seen = {0: 0, 1: 0}
    for q in qs:
        s = 0.2 / (1.0 + seen[q])
        w[q], h = _scalar_sgd(w[q], h, float(val[q]), s, 0.1)
        seen[q] += 1
    assert W[0, 0] == pytest.approx(w[0], abs=1e-15) and W[1, 0] == pytest.approx(w[1], abs=1e-15)
    assert H[0, 0] == pytest.approx(h, abs=1e-15)


def test_uniform_recipients_are_uniform():
    """Algorithm 1's recipient is uniform over all p workers: the workers of consecutive
    visits of one item held everywhere are independent uniform draws."""
    P = 5
    m = P
    row = np.arange(m, dtype=np.int32)
    col = np.zeros(m, dtype=np.int32)
    val = np.ones(m, dtype=np.float32)
    hp = Hyper(1, 0.0, 0.0, 0.0, 1.0)  # s = 0: nothing changes, only the order is of interest
    n_vis = 20_000
    _, _, _, tr = oracle.train_uniform(m, 1, row, col, val, np.ones((m, 1)), np.ones((1, 1)), hp, P, 1, n_vis, 5,
                                       trace=True)
    q = tr[:, 0]
    counts = np.bincount(q, minlength=P)
    chi2 = ((counts - n_vis / P) ** 2 / (n_vis / P)).sum()
    assert chi2 < 30, counts  # 4 degrees of freedom
    pairs = np.bincount(q[:-1] * P + q[1:], minlength=P * P)
    chi2p = ((pairs - (n_vis - 1) / P**2) ** 2 / ((n_vis - 1) / P**2)).sum()
    assert chi2p < 70, pairs  # 24 degrees of freedom


# ---------------------------------------------------------------- permutation circulation

def test_perm_epoch_orders_are_uniform_random_permutations():
    """Section 3.4's random permutation: an item visits each holder once per epoch, the
    next one drawn uniformly among the holders not yet visited.  With three holders every
    epoch's order (after the first, whose start is the item's initial queue) is one of the
    3! = 6 orders with probability 1/6 each (a rule such as "lowest unvisited worker next"
    gives only three of them)."""
    P = 3
    row = np.arange(P, dtype=np.int32)
    col = np.zeros(P, dtype=np.int32)
    val = np.ones(P, dtype=np.float32)
    hp = Hyper(1, 0.0, 0.0, 0.0, 1.0)
    E = 6_000
    _, _, st, tr = oracle.train_perm(P, 1, row, col, val, np.ones((P, 1)), np.ones((1, 1)), hp, P, 2, E, 9,
                                     trace=True)
    assert len(tr) == E * P and st.updates == E * P
    orders = tr[:, 0].reshape(E, P)
    assert all(sorted(o) == [0, 1, 2] for o in orders.tolist())
    assert np.array_equal(tr[:, 2].reshape(E, P), np.repeat(np.arange(E)[:, None], P, axis=1))
    perms = list(itertools.permutations(range(P)))
    idx = [perms.index(tuple(o)) for o in orders[1:].tolist()]
    counts = np.bincount(idx, minlength=6)
    expect = (E - 1) / 6
    chi2 = ((counts - expect) ** 2 / expect).sum()
    assert chi2 < 30, counts  # 5 degrees of freedom: p < 1e-5 for a uniform draw
    # consecutive epochs are independent: the next epoch's first holder does not follow
    # from the last one of the epoch before
    last, first = orders[:-1, -1], orders[1:, 0]
    same = float(np.mean(last == first))
    assert abs(same - 1 / 3) < 0.03


@pytest.mark.parametrize("sched", ["perm", "uniform"])
def test_emulation_traces_replay_to_the_same_factors(sched):
    """The trace an emulation records (worker, item, t, item visit number) replays in
    orc_replay to exactly the emulation's factors: the trace says everything about the
    order that matters."""
    p_, W0, H0, hp = _small(seed=41, degrees="zipf")
    row, col, val = _np(p_)
    P, seed = 6, 4
    if sched == "perm":
        W, H, st, tr = oracle.train_perm(p_.m, p_.n, row, col, val, W0, H0, hp, P, seed, 3, 12, trace=True)
    else:
        W, H, st, tr = oracle.train_uniform(p_.m, p_.n, row, col, val, W0, H0, hp, P, seed, 3 * p_.nnz, 12,
                                            trace=True)
    order = np.argsort(tr[:, 0], kind="stable")
    t2 = tr[order]
    Wr, Hr, st2 = oracle.replay(p_.m, p_.n, row, col, val, W0, H0, hp, P, seed, t2[:, 0], t2[:, 1], t2[:, 2],
                                t2[:, 3])
    assert np.array_equal(W, Wr) and np.array_equal(H, Hr)
    assert st2.updates == st.updates


# ---------------------------------------------------------------- global update count

def test_ring_global_count_one_worker_by_hand():
    """t = updates applied before the visit: with one worker the visits are the items in
    ascending order, each over its ratings in ascending row order, every rating of a
    visit using the count at the visit's start."""
    p_, W0, H0, _ = _small(m=20, n=12, nnz=120, seed=43, k=3)
    hp = Hyper(3, 0.05, 0.05, 0.01, 1.0)
    row, col, val = _np(p_)
    E, t0 = 2, 37
    W, H, _ = oracle.train_ring_gcount(p_.m, p_.n, row, col, val, W0, H0, hp, 1, 0, E, t0=t0)
    Wb, Hb = W0.astype(np.float64).copy(), H0.astype(np.float64).copy()
    t = t0
    for _ in range(E):
        for j in range(p_.n):
            xs = np.nonzero(col == j)[0]
            xs = xs[np.argsort(row[xs])]
            s = hp.alpha / (1.0 + hp.beta * t)
            for x in xs:
                Wb[row[x]], Hb[j] = oracle.update(Wb[row[x]], Hb[j], val[x], s, hp.lam)
            t += len(xs)
    assert np.array_equal(W, Wb) and np.array_equal(H, Hb)


def test_ring_global_count_with_constant_step_is_the_ring():
    p_, W0, H0, hp = _small(seed=47)
    hp = Hyper(hp.k, hp.lam, hp.alpha, 0.0, hp.gamma)
    row, col, val = _np(p_)
    W, H, _ = oracle.train_ring_gcount(p_.m, p_.n, row, col, val, W0, H0, hp, 5, 2, 2)
    Wr, Hr, _ = oracle.train_ring(p_.m, p_.n, row, col, val, W0, H0, hp, 5, 2, 2)
    assert np.array_equal(W, Wr) and np.array_equal(H, Hr)


# ---------------------------------------------------------------- threaded Algorithm 1

def test_threaded_single_worker_is_the_ring_order():
    p_, W0, H0, hp = _small(m=40, n=30, nnz=500, seed=53)
    row, col, val = _np(p_)
    W, H, st, sec = oracle.train_threaded(p_.m, p_.n, row, col, val, W0, H0, hp, 1, 3, 3 * p_.nnz, 7)
    Wr, Hr, _ = oracle.train_ring(p_.m, p_.n, row, col, val, W0, H0, hp, 1, 3, 3)
    assert np.array_equal(W, Wr) and np.array_equal(H, Hr)
    assert st.updates == 3 * p_.nnz and sec >= 0.0


def test_threaded_many_workers_learns_like_the_emulation():
    """Several threads: the interleaving depends on timing, so the result is checked by
    its properties: the update budget is met (and overshot by less than one visit per
    worker), and the training objective falls about as far as under the serial emulation
    of the same routing (which ratings get the budget's updates depends on the threads'
    timing, so only roughly)."""
    p_, W0, H0, hp = _small(m=300, n=120, nnz=8_000, seed=59, k=8, alpha=0.05, beta=0.0)
    row, col, val = _np(p_)
    P, budget = 4, 5 * p_.nnz
    W, H, st, sec = oracle.train_threaded(p_.m, p_.n, row, col, val, W0, H0, hp, P, 3, budget, 7)
    assert budget <= st.updates <= budget + P * p_.nnz
    assert st.hops > 0 and sec > 0.0
    Wu, Hu, _ = oracle.train_uniform(p_.m, p_.n, row, col, val, W0, H0, hp, P, 3, budget, 7)
    J0 = oracle.objective(p_.m, p_.n, row, col, val, W0, H0, hp.lam)
    Jt = oracle.objective(p_.m, p_.n, row, col, val, W, H, hp.lam)
    Ju = oracle.objective(p_.m, p_.n, row, col, val, Wu, Hu, hp.lam)
    assert Jt < 0.4 * J0 and Ju < 0.4 * J0 and abs(Jt - Ju) < 0.5 * Ju, (J0, Jt, Ju)


# ---------------------------------------------------------------- dynamic load balancing (section 3.3)

def test_balanced_pick_prefers_the_shorter_queue():
    assert oracle.balanced_pick(3, 5, 7, 2) == 7
    assert oracle.balanced_pick(3, 2, 7, 5) == 3
    assert oracle.balanced_pick(3, 4, 7, 4) == 3  # a tie keeps the first draw
    assert oracle.balanced_pick(0, 0, 1, 0) == 0


@pytest.mark.parametrize("P", [3, 7])
def test_balanced_perm_still_visits_every_holder_once_per_epoch(P):
    """Load balancing changes the order of an item's holders, never which ones it visits:
    every (worker, item) pair that shares ratings once per epoch, and the trace replays."""
    p_, W0, H0, hp = _small(seed=61, degrees="zipf")
    row, col, val = _np(p_)
    E = 4
    W, H, st, tr = oracle.train_perm(p_.m, p_.n, row, col, val, W0, H0, hp, P, 2, E, 13, trace=True, balance=True)
    rs = oracle.partition(p_.m, row, P)
    q_of = np.searchsorted(rs, row, "right") - 1
    pairs = sorted({(int(q), int(j)) for q, j in zip(q_of, col)})
    assert st.updates == E * p_.nnz and st.violations == 0
    for e in range(E):
        assert sorted((int(a), int(b)) for a, b in tr[tr[:, 2] == e, :2]) == pairs
    order = np.argsort(tr[:, 0], kind="stable")
    t2 = tr[order]
    Wr, Hr, _ = oracle.replay(p_.m, p_.n, row, col, val, W0, H0, hp, P, 2, t2[:, 0], t2[:, 1], t2[:, 2], t2[:, 3])
    assert np.array_equal(W, Wr) and np.array_equal(H, Hr)


def _random_problem(P, n, per_row=40, seed=5):
    m = P * 30
    rng = np.random.default_rng(seed)
    row = np.repeat(np.arange(m, dtype=np.int32), per_row)
    col = rng.integers(0, n, row.size).astype(np.int32)
    key = np.unique(row.astype(np.int64) * n + col)
    row, col = (key // n).astype(np.int32), (key % n).astype(np.int32)
    val = rng.standard_normal(row.size).astype(np.float32)
    return m, row, col, val


@pytest.mark.parametrize("sched_seed", [1, 2, 3])
def test_balanced_uniform_routing_keeps_queues_short(sched_seed):
    """Section 3.3's rule in the uniform routing of Algorithm 1: the recipient is the less
    loaded of two uniform draws.  By the "power of two choices" result (Azar, Broder,
    Karlin, Upfal 1994) the longest queue then stays near the mean instead of drifting far
    above it as under one uniform draw; with 1,000 items among 16 workers (about 62 per
    worker) the longest queue over 30 epochs of updates must come out below half of the
    single-draw run's."""
    P, n = 16, 1000
    m, row, col, val = _random_problem(P, n)
    hp = Hyper(2, 0.05, 0.0, 0.0, 1.0)  # s = 0: only the routing matters
    W0, H0 = np.ones((m, 2)), np.ones((n, 2))
    budget = 30 * row.size
    _, _, st0 = oracle.train_uniform(m, n, row, col, val, W0, H0, hp, P, 1, budget, sched_seed)
    _, _, st1 = oracle.train_uniform(m, n, row, col, val, W0, H0, hp, P, 1, budget, sched_seed, balance=True)
    assert st0.updates >= budget and st1.updates >= budget
    assert st1.max_queue < 0.5 * st0.max_queue, (st0.max_queue, st1.max_queue)
    assert st1.max_queue >= n // P  # some worker holds at least the mean


# ---------------------------------------------------------------- time-driven turns

def test_timed_turns_with_one_worker_are_the_ring_order():
    """With one worker serving one item at a time, time-driven turns take the queue in
    FIFO order whatever the costs: the items cycle in ascending order, which is the ring
    order of one worker."""
    p_, W0, H0, hp = _small(m=40, n=30, nnz=500, seed=71)
    row, col, val = _np(p_)
    for timing in [(1, 0.0, 0.0), (1, 25.0, 45.0)]:
        W, H, st = oracle.train_uniform(p_.m, p_.n, row, col, val, W0, H0, hp, 1, 3, 3 * p_.nnz, 7, timing=timing)
        Wr, Hr, _ = oracle.train_ring(p_.m, p_.n, row, col, val, W0, H0, hp, 1, 3, 3)
        assert np.array_equal(W, Wr) and np.array_equal(H, Hr), timing


def test_timed_turns_follow_visit_costs():
    """One worker serving two items at once: item A has one rating, item B twenty.  With
    turns driven by time (costs in units of one update, no hand-off delay) A completes a
    visit every unit while B completes one every twenty, so A is visited about twenty times
    as often; under the uniform draw of turns the FIFO queue alternates them.  Both traces
    replay exactly."""
    m, n = 20, 2
    row = np.array([0] + list(range(20)), dtype=np.int32)
    col = np.array([0] + [1] * 20, dtype=np.int32)
    val = np.ones(row.size, dtype=np.float32)
    hp = Hyper(2, 0.05, 0.01, 0.0, 1.0)
    W0, H0 = np.full((m, 2), 0.3), np.full((n, 2), 0.3)
    budget = 400
    counts = {}
    for timing in (None, (2, 0.0, 0.0)):
        W, H, st, tr = oracle.train_uniform(m, n, row, col, val, W0, H0, hp, 1, 1, budget, 5, trace=True,
                                            timing=timing)
        counts[timing] = np.bincount(tr[:, 1], minlength=2)
        t2 = tr[np.argsort(tr[:, 0], kind="stable")]
        Wr, Hr, _ = oracle.replay(m, n, row, col, val, W0, H0, hp, 1, 1, t2[:, 0], t2[:, 1], t2[:, 2], t2[:, 3])
        assert np.array_equal(W, Wr) and np.array_equal(H, Hr)
    a, b = counts[None]
    assert abs(int(a) - int(b)) <= 1
    a, b = counts[(2, 0.0, 0.0)]
    assert 15 * b <= a <= 25 * b + 25, (a, b)
