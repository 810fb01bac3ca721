"""The batched form: several independent problems trained by one launch per call.

Pins (the batched-independence property): every problem of a batch ends bitwise equal
to the same problem trained alone with the same number of workers, and within the ring
tolerance (1e-5 after one epoch, FP32 vs FP64) of the oracle's ring order at that worker
count.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1312_0193_amd as nm
import synth
from parity import check, max_updates

pytestmark = pytest.mark.gpu

TOL_1EPOCH = 1e-5


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def f32(x):
    return float(np.float32(x))


def problems(specs, seed0=100):
    out = []
    for b, (m, n, nnz, k, lam) in enumerate(specs):
        prob = synth.small_case(m, n, nnz, seed=seed0 + b, degrees="uniform", k=k, lam=lam, alpha=0.01, beta=1e-4,
                                gamma=1.0, test_frac=0.1)
        W0, H0 = synth.init_factors(m, n, k, seed0 + b)
        out.append(dict(m=m, n=n, row=prob.row, col=prob.col, val=prob.val, W0=W0, H0=H0, k=k, lam=lam,
                        alpha=0.01, beta=1e-4, gamma=1.0, prob=prob))
    return out


SPECS = [
    # m, n, nnz, k, lambda: sizes spanning two orders of magnitude, k in {16, 32, 64}
    (2_000, 1_000, 60_000, 16, 0.05),
    (300, 500, 8_000, 32, 0.01),
    (1_500, 200, 30_000, 64, 0.1),
    (120, 90, 2_000, 16, 0.05),
    (4_000, 800, 90_000, 32, 0.05),
    (50, 40, 400, 64, 0.01),
]


def test_batch_matches_problems_alone_and_oracle():
    probs = problems(SPECS)
    print(f"[case] batch of {len(probs)} problems, 40 workers", flush=True)
    batch = nm.NomadBatch(probs, workers=40, seed=3)
    st = batch.train(1)
    assert st.updates == sum(int(p["row"].numel()) for p in probs)
    workers = [v.workers for v in batch.problems]
    assert sum(workers) == 40 and min(workers) >= 1
    # more ratings, more workers
    nnz = [p["row"].numel() for p in probs]
    assert workers[int(np.argmax(nnz))] == max(workers)
    for b, (p, view) in enumerate(zip(probs, batch.problems)):
        Wb, Hb = (x.cpu().double().numpy() for x in view.factors())
        print(f"[case] problem {b} alone, {workers[b]} workers", flush=True)
        alone = nm.Nomad(p["m"], p["n"], p["row"], p["col"], p["val"], p["W0"], p["H0"], k=p["k"], lam=p["lam"],
                         alpha=p["alpha"], beta=p["beta"], gamma=p["gamma"], workers=workers[b], seed=3)
        alone.train(1)
        Wa, Ha = (x.cpu().double().numpy() for x in alone.factors())
        alone.close()
        assert np.array_equal(Wa, Wb) and np.array_equal(Ha, Hb), b
        hp = oracle.Hyper(p["k"], f32(p["lam"]), f32(p["alpha"]), f32(p["beta"]), f32(p["gamma"]))
        Wo, Ho, _ = oracle.train_ring(p["m"], p["n"], p["row"].numpy(), p["col"].numpy(), p["val"].numpy(),
                                      p["W0"].numpy(), p["H0"].numpy(), hp, workers[b], 3, 1)
        T = max_updates(p["row"].numpy(), p["col"].numpy(), 1)
        check(Wb, Wo, norm_tol=TOL_1EPOCH, updates=T, what=f"problem {b} W")
        check(Hb, Ho, norm_tol=TOL_1EPOCH, updates=T, what=f"problem {b} H")
        # evaluation through the problem's view
        pr = p["prob"]
        r_gpu, _ = view.evaluate(pr.test_row, pr.test_col, pr.test_val)
        r_orc = oracle.rmse(p["m"], p["n"], pr.test_row.numpy(), pr.test_col.numpy(), pr.test_val.numpy(), Wb, Hb)
        assert abs(r_gpu - r_orc) <= 1e-12 * max(1.0, r_orc)
    batch.close()


@pytest.mark.timeout(900)
def test_batched_workload_256_problems():
    """The batched configuration itself: 256 problems with log-uniform sizes (rows 1k-200k,
    columns 500-20k, 50k-5M ratings), k in {16, 32, 64} and lambda in {0.01, 0.05, 0.1},
    one launch per epoch.  For a sample of problems (the largest, the smallest and four
    more) the factors after one epoch are bitwise those of the problem trained alone with
    the same worker count, and within the ring tolerance of the oracle."""
    specs = synth.batched_specs(256, seed=4)
    print("[case] batched workload: generating 256 problems on the GPU", flush=True)
    probs = []
    for s in specs:
        pr = synth.batched_problem(s, device="cuda")
        W0, H0 = synth.init_factors(s["m"], s["n"], s["k"], s["seed"], device="cuda")
        probs.append(dict(m=s["m"], n=s["n"], row=pr.row, col=pr.col, val=pr.val, W0=W0, H0=H0, k=s["k"],
                          lam=s["lam"], alpha=s["alpha"], beta=s["beta"], gamma=s["gamma"]))
    total = sum(int(p["row"].numel()) for p in probs)
    print(f"[case] batch of 256 problems, {total} ratings: layout", flush=True)
    batch = nm.NomadBatch(probs, seed=4)
    st = batch.train(1)
    assert st.updates == total
    workers = [v.workers for v in batch.problems]
    print(f"[case] one epoch {st.seconds * 1e3:.1f} ms, {sum(workers)} workers", flush=True)
    nnz = np.array([int(p["row"].numel()) for p in probs])
    rng = np.random.default_rng(0)
    sample = [int(np.argmax(nnz)), int(np.argmin(nnz))] + [int(x) for x in rng.choice(256, 4, replace=False)]
    for b in sample:
        p = probs[b]
        print(f"[case] problem {b}: {p['m']} x {p['n']}, {nnz[b]} ratings, k={p['k']}, {workers[b]} workers",
              flush=True)
        Wb, Hb = (x.cpu().double().numpy() for x in batch.problems[b].factors())
        alone = nm.Nomad(p["m"], p["n"], p["row"], p["col"], p["val"], p["W0"], p["H0"], k=p["k"], lam=p["lam"],
                         alpha=p["alpha"], beta=p["beta"], gamma=p["gamma"], workers=workers[b], seed=4)
        alone.train(1)
        Wa, Ha = (x.cpu().double().numpy() for x in alone.factors())
        alone.close()
        assert np.array_equal(Wa, Wb) and np.array_equal(Ha, Hb), b
        hp = oracle.Hyper(p["k"], f32(p["lam"]), f32(p["alpha"]), f32(p["beta"]), f32(p["gamma"]))
        row, col, val = (x.cpu().numpy() for x in (p["row"], p["col"], p["val"]))
        Wo, Ho, _ = oracle.train_ring(p["m"], p["n"], row, col, val, p["W0"].cpu().numpy(), p["H0"].cpu().numpy(),
                                      hp, workers[b], 4, 1)
        T = max_updates(row, col, 1)
        check(Wb, Wo, norm_tol=TOL_1EPOCH, updates=T, what=f"problem {b} W")
        check(Hb, Ho, norm_tol=TOL_1EPOCH, updates=T, what=f"problem {b} H")
    batch.close()


def test_batch_continues_across_calls_and_launches():
    probs = problems(SPECS[:3], seed0=200)
    print("[case] batch 3 problems, calls [2, 65]", flush=True)
    batch = nm.NomadBatch(probs, workers=24, seed=1)
    batch.train(2)
    batch.train(65)  # two launches
    workers = [v.workers for v in batch.problems]
    for b, (p, view) in enumerate(zip(probs, batch.problems)):
        Wb, Hb = (x.cpu().double().numpy() for x in view.factors())
        alone = nm.Nomad(p["m"], p["n"], p["row"], p["col"], p["val"], p["W0"], p["H0"], k=p["k"], lam=p["lam"],
                         alpha=p["alpha"], beta=p["beta"], gamma=p["gamma"], workers=workers[b], seed=1)
        alone.train(67)
        Wa, Ha = (x.cpu().double().numpy() for x in alone.factors())
        alone.close()
        assert np.array_equal(Wa, Wb) and np.array_equal(Ha, Hb), b
    batch.close()


def test_batch_bf16_and_empty_problem():
    probs = problems(SPECS[1:3], seed0=300)
    e = torch.zeros(0, dtype=torch.int32)
    W0, H0 = synth.init_factors(10, 7, 16, 9)
    probs.append(dict(m=10, n=7, row=e, col=e, val=torch.zeros(0), W0=W0, H0=H0, k=16, lam=0.05, alpha=0.01,
                      beta=1e-4, gamma=1.0))
    print("[case] batch with an empty problem, bf16", flush=True)
    batch = nm.NomadBatch(probs, workers=12, seed=2, dtype="bf16", rounding="stochastic")
    batch.train(2)
    W, H = batch.problems[2].factors()
    assert torch.equal(H.cpu(), H0)  # nothing to update
    for b, p in enumerate(probs[:2]):
        alone = nm.Nomad(p["m"], p["n"], p["row"], p["col"], p["val"], p["W0"], p["H0"], k=p["k"], lam=p["lam"],
                         alpha=p["alpha"], beta=p["beta"], gamma=p["gamma"], workers=batch.problems[b].workers,
                         seed=2, dtype="bf16", rounding="stochastic")
        alone.train(2)
        assert all(torch.equal(x, y) for x, y in zip(alone.factors(), batch.problems[b].factors())), b
        alone.close()
    batch.close()


def test_batch_errors():
    probs = problems(SPECS[:3], seed0=400)
    with pytest.raises(nm.NomadError, match="EINVAL"):
        nm.NomadBatch(probs, workers=2)  # fewer workers than problems
    bad = [dict(probs[0]), probs[1]]
    bad[0]["row"] = bad[0]["row"].clone()
    bad[0]["row"][0] = bad[0]["m"] + 5
    with pytest.raises(nm.NomadError, match="problem 0"):
        nm.NomadBatch(bad, workers=8)
    batch = nm.NomadBatch(probs, workers=8)
    lib = nm.load()
    W = torch.empty(probs[0]["m"], probs[0]["k"], device="cuda")
    H = torch.empty(probs[0]["n"], probs[0]["k"], device="cuda")
    assert lib.nomad_get_factors(batch.ctx, W.data_ptr(), H.data_ptr()) == nm.NOMAD_ESTATE
    assert lib.nomad_train_epochs(batch.problems[0].ctx, 1, None) == nm.NOMAD_ESTATE
    batch.close()


def _factors_equal(a, b):
    return all(torch.equal(x, y) for va, vb in zip(a.problems, b.problems)
               for x, y in zip(va.factors(), vb.factors()))


def test_batch_graph_replays_match_direct_launches():
    """A captured batch launch (nomad_batch_graph) gives the direct launches' factors
    bitwise, on every replay, with other GPU work between replays, after a direct call of a
    different length, and for a graph of two launches (66 epochs)."""
    probs = problems(SPECS[:4], seed0=500)
    for kw in (dict(), dict(dtype="bf16", rounding="stochastic")):
        print(f"[case] batch graph, 4 problems, {kw}", flush=True)
        g = nm.NomadBatch(probs, workers=24, seed=5, **kw)
        d = nm.NomadBatch(probs, workers=24, seed=5, **kw)
        g.graph(2)
        for r in range(3):
            g.train(2)
            d.train(2)
            # eager work and a synchronisation between replays
            pr = probs[0]["prob"]
            g.problems[0].evaluate(pr.test_row, pr.test_col, pr.test_val)
            torch.cuda.synchronize()
            assert _factors_equal(g, d), (kw, r)
        g.train(1)  # a direct launch between replays
        d.train(1)
        g.train(2)
        d.train(2)
        assert _factors_equal(g, d), kw
        g.close()
        d.close()
    print("[case] batch graph of 66 epochs (two launches)", flush=True)
    g = nm.NomadBatch(probs[:2], workers=8, seed=6)
    d = nm.NomadBatch(probs[:2], workers=8, seed=6)
    g.graph(66)
    g.train(66)
    d.train(66)
    assert _factors_equal(g, d)
    g.graph(0)  # dropped: direct launches again
    g.train(66)
    d.train(66)
    assert _factors_equal(g, d)
    g.close()
    d.close()
    with pytest.raises(nm.NomadError, match="ESTATE"):
        alone = nm.Nomad(probs[0]["m"], probs[0]["n"], probs[0]["row"], probs[0]["col"], probs[0]["val"],
                         probs[0]["W0"], probs[0]["H0"], k=probs[0]["k"], lam=0.05, alpha=0.01, beta=1e-4,
                         gamma=1.0, workers=4)
        try:
            nm._check(nm.load().nomad_batch_graph(alone.ctx, 2), alone.ctx)
        finally:
            alone.close()


def test_tune_batched_picks_a_working_shape():
    probs = problems(SPECS, seed0=600)
    print("[case] autotuner over the 6-problem batch", flush=True)
    seen = []
    shape, sec = nm.tune_batched(probs, progress=lambda c, st, t: seen.append((c, st, t)), seed=3)
    print(f"[case] candidates {seen}", flush=True)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    assert len(seen) == 4
    assert {(c["workers"], c["waves_per_worker"]) for c, _, _ in seen} == {(w, nw) for w in (cus, 2 * cus)
                                                                           for nw in (4, 8)}
    ok = [(t, c) for c, st, t in seen if st == nm.NOMAD_OK]
    assert ok and sec == min(t for t, _ in ok) and shape == min(ok, key=lambda x: x[0])[1]
    # a field that is set stays fixed
    shape2, _ = nm.tune_batched(probs, seed=3, waves_per_worker=6, window=16)
    assert shape2["waves_per_worker"] == 6 and shape2["window"] == 16
    batch = nm.NomadBatch(probs, autotune=True, seed=3)
    assert batch.tuned is not None and batch.tuned["workers"] == sum(v.workers for v in batch.problems)
    batch.train(1)
    b = int(np.argmax([v.workers for v in batch.problems]))
    p = probs[b]
    alone = nm.Nomad(p["m"], p["n"], p["row"], p["col"], p["val"], p["W0"], p["H0"], k=p["k"], lam=p["lam"],
                     alpha=p["alpha"], beta=p["beta"], gamma=p["gamma"], workers=batch.problems[b].workers, seed=3)
    alone.train(1)
    assert all(torch.equal(x, y) for x, y in zip(alone.factors(), batch.problems[b].factors()))
    alone.close()
    batch.close()
