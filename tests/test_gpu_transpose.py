"""Transposed mode (the symmetric choice noted in section 3.1): the row factors w_i travel
and the column factors stay with the worker that holds their column block.  The library
then runs NOMAD on A^T while every argument and result keeps A's orientation, so a
transposed context must give, bitwise, what an ordinary context gives on the transposed
problem (rows and columns, W0 and H0 exchanged), and both must match the FP64 oracle run on
A^T."""
import numpy as np
import pytest
import torch

import oracle
import paper_1312_0193_amd as nm
import synth
from parity import check, max_updates

pytestmark = pytest.mark.gpu


def setup(m, n, nnz, k, seed, degrees="uniform"):
    prob = synth.small_case(m, n, nnz, seed=seed, degrees=degrees, k=k, test_frac=0.1)
    W0, H0 = synth.init_factors(m, n, k, seed)
    f = lambda x: float(np.float32(x))  # noqa: E731
    hp = oracle.Hyper(k, f(0.05), f(0.01), f(1e-4), f(1.0))
    return prob, W0, H0, hp


def nomad(m, n, row, col, val, W0, H0, hp, P, **kw):
    return nm.Nomad(m, n, row, col, val, W0, H0, k=hp.k, lam=hp.lam, alpha=hp.alpha, beta=hp.beta, gamma=hp.gamma,
                    workers=P, seed=5, **kw)


@pytest.mark.parametrize("case", [
    # m, n, nnz, k, P, sched, dtype
    (300, 2_000, 40_000, 32, 16, "ring", "fp32"),
    (500, 3_000, 60_000, 100, 32, "ring", "bf16"),
    (400, 2_500, 50_000, 64, 8, "perm", "fp32"),
])
def test_transposed_equals_the_transposed_problem(case):
    m, n, nnz, k, P, sched, dtype = case
    prob, W0, H0, hp = setup(m, n, nnz, k, m + P)
    E = 2
    print(f"[case] transpose m={m} n={n} nnz={nnz} k={k} P={P} {sched} {dtype}", flush=True)
    kw = dict(sched=sched, dtype=dtype)
    if sched == "perm":
        P = 1  # with one worker the order is fixed, so the comparison can be bitwise
    t = nomad(m, n, prob.row, prob.col, prob.val, W0, H0, hp, P, transpose=True, **kw)
    t.train(E)
    Wt, Ht = t.factors()
    rt, jt = t.evaluate(prob.test_row, prob.test_col, prob.test_val)
    part_t = t.partition()
    t.close()
    # the same run, asked for on A^T directly
    u = nomad(n, m, prob.col, prob.row, prob.val, H0, W0, hp, P, **kw)
    u.train(E)
    Hu, Wu = u.factors()
    ru, ju = u.evaluate(prob.test_col, prob.test_row, prob.test_val)
    part_u = u.partition()
    u.close()
    assert torch.equal(Wt, Wu) and torch.equal(Ht, Hu)
    assert rt == ru and jt == ju
    assert np.array_equal(part_t, part_u)  # bounds of column blocks
    assert part_t[-1] == n
    if dtype == "fp32" and sched == "ring":
        Ho, Wo, _ = oracle.train_ring(n, m, prob.col.numpy(), prob.row.numpy(), prob.val.numpy(), H0.numpy(),
                                      W0.numpy(), hp, P, 5, E)
        T = max_updates(prob.row.numpy(), prob.col.numpy(), E)
        check(Wt.cpu().double().numpy(), Wo, norm_tol=1e-5, updates=T, what="W (transposed)")
        check(Ht.cpu().double().numpy(), Ho, norm_tol=1e-5, updates=T, what="H (transposed)")
        r_o = oracle.rmse(m, n, prob.test_row.numpy(), prob.test_col.numpy(), prob.test_val.numpy(), Wo, Ho)
        assert abs(rt - r_o) <= 1e-6 * r_o


def test_transposed_holds_fewer_vectors_in_flight():
    """With fewer rows than columns, making the rows nomadic means fewer travelling vectors:
    the hand-offs of one permutation epoch count the (worker, travelling index) visits."""
    m, n, nnz, k, P = 200, 4_000, 60_000, 16, 16
    prob, W0, H0, hp = setup(m, n, nnz, k, 7)
    hops = {}
    for tr in (False, True):
        mdl = nomad(m, n, prob.row, prob.col, prob.val, W0, H0, hp, P, sched="perm", transpose=tr)
        st = mdl.train(1)
        assert st.updates == prob.nnz
        hops[tr] = st.hops
        mdl.close()
    print(f"[parity] hand-offs per epoch: columns travel {hops[False]}, rows travel {hops[True]}", flush=True)
    assert hops[True] < hops[False]


def test_transpose_not_in_batches():
    prob, W0, H0, hp = setup(200, 300, 3_000, 8, 9)
    d = dict(m=prob.m, n=prob.n, row=prob.row, col=prob.col, val=prob.val, W0=W0, H0=H0, k=8, lam=hp.lam,
             alpha=hp.alpha, beta=hp.beta, gamma=hp.gamma)
    with pytest.raises(nm.NomadError):
        nm.NomadBatch([d, d], transpose=True)
