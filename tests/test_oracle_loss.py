"""Pins of the oracle's general separable loss (section 2: the method takes any separable
loss; the conclusion writes the objective as a sum of per-rating terms): the logistic loss
of labels +-1, whose update uses e = r / (1 + exp(r d)) in place of the square loss's r - d.

Pinned by a hand-worked update and objective (tests/golden/logistic_update.json), closed
forms of the loss and residual, central finite differences (the residual is minus the loss's
derivative; the update is minus the step times the gradient of the per-rating objective),
the one-worker ring order against serial SGD written out, and learning on planted labels."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth

GOLD = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "logistic_update.json")))


def test_logistic_update_hand_worked():
    for c in GOLD["cases"]:
        assert oracle.residual(c["r"], 0.5, "logistic") == pytest.approx(c["e"], rel=1e-15)
        w, h = oracle.update_loss(GOLD["w"], GOLD["h"], c["r"], GOLD["s"], GOLD["lambda"], "logistic")
        assert np.allclose(w, c["w"], rtol=1e-15, atol=1e-17)
        assert np.allclose(h, c["h"], rtol=1e-15, atol=1e-17)


def test_logistic_objective_hand_worked():
    W = np.array([GOLD["w"]], dtype=np.float64)
    H = np.array([GOLD["h"]], dtype=np.float64)
    J = oracle.objective(1, 1, [0], [0], [1.0], W, H, GOLD["lambda"], loss="logistic")
    assert J == pytest.approx(GOLD["objective_r1"], rel=1e-15)


def test_loss_and_residual_closed_forms():
    assert oracle.loss_value(1.0, 0.0, "logistic") == pytest.approx(math.log(2.0), rel=1e-15)
    for d in (-3.0, -0.2, 0.0, 0.7, 5.0):
        # log(1 + e^-d) - log(1 + e^d) = -d
        assert oracle.loss_value(1.0, d, "logistic") - oracle.loss_value(-1.0, d, "logistic") == pytest.approx(
            -d, abs=1e-14)
        assert oracle.residual(1.0, d, "logistic") + oracle.residual(-1.0, -d, "logistic") == pytest.approx(0.0,
                                                                                                             abs=1e-16)
    assert oracle.residual(1.0, 0.0, "logistic") == 0.5 and oracle.residual(-1.0, 0.0, "logistic") == -0.5
    assert 0.0 <= oracle.residual(1.0, 800.0, "logistic") < 1e-300  # exp overflows: e -> 0
    assert oracle.residual(1.0, -800.0, "logistic") == 1.0
    assert oracle.loss_value(1.0, -800.0, "logistic") == pytest.approx(800.0, rel=1e-15)  # no overflow
    assert oracle.residual(3.0, 1.25, "square") == 1.75
    assert oracle.loss_value(3.0, 1.25, "square") == 0.5 * 1.75 ** 2


@pytest.mark.parametrize("loss,r", [("logistic", 1.0), ("logistic", -1.0), ("square", 0.3)])
def test_residual_is_minus_the_loss_derivative(loss, r):
    for d in (-2.5, -0.4, 0.0, 0.9, 3.0):
        eps = 1e-6
        fd = (oracle.loss_value(r, d + eps, loss) - oracle.loss_value(r, d - eps, loss)) / (2 * eps)
        assert oracle.residual(r, d, loss) == pytest.approx(-fd, rel=1e-8, abs=1e-10)


def test_logistic_update_is_minus_step_times_gradient():
    rng = np.random.default_rng(7)
    k, s, lam = 5, 1e-3, 0.3
    for r in (1.0, -1.0):
        w = rng.normal(size=k)
        h = rng.normal(size=k)

        def f(w_, h_):
            return oracle.loss_value(r, float(w_ @ h_), "logistic") + 0.5 * lam * (w_ @ w_ + h_ @ h_)

        gw = np.zeros(k)
        gh = np.zeros(k)
        eps = 1e-6
        for l in range(k):
            dw = np.zeros(k)
            dw[l] = eps
            gw[l] = (f(w + dw, h) - f(w - dw, h)) / (2 * eps)
            gh[l] = (f(w, h + dw) - f(w, h - dw)) / (2 * eps)
        w2, h2 = oracle.update_loss(w, h, r, s, lam, "logistic")
        assert np.allclose((w2 - w) / s, -gw, rtol=1e-7, atol=1e-9)
        assert np.allclose((h2 - h) / s, -gh, rtol=1e-7, atol=1e-9)


def test_one_worker_logistic_ring_is_serial_sgd():
    prob = synth.small_case(40, 30, 400, seed=3, k=4, values="sign", test_frac=0.0)
    row, col, val = prob.row.numpy(), prob.col.numpy(), prob.val.numpy()
    assert set(np.unique(val)) <= {-1.0, 1.0}
    W0, H0 = synth.init_factors(40, 30, 4, 3)
    hp = oracle.Hyper(4, 0.05, 0.1, 0.01, 1.0)
    Wo, Ho, _ = oracle.train_ring(40, 30, row, col, val, W0.numpy(), H0.numpy(), hp, 1, 0, 3, loss="logistic")
    # serial SGD written out: one worker takes the items in ascending order, each item's
    # ratings in ascending row; t = epochs done
    W = W0.numpy().astype(np.float64).tolist()
    H = H0.numpy().astype(np.float64).tolist()
    order = sorted(range(len(row)), key=lambda x: (int(col[x]), int(row[x])))
    for t in range(3):
        s = hp.alpha / (1.0 + hp.beta * t ** hp.gamma)
        for x in order:
            w, h, r = W[int(row[x])], H[int(col[x])], float(val[x])
            d = 0.0
            for l in range(4):
                d += w[l] * h[l]
            e = r / (1.0 + math.exp(r * d))
            for l in range(4):
                wl, hl = w[l], h[l]
                w[l] = wl + s * (e * hl - hp.lam * wl)
                h[l] = hl + s * (e * wl - hp.lam * hl)
    assert np.allclose(Wo, np.array(W), rtol=1e-13, atol=1e-15)
    assert np.allclose(Ho, np.array(H), rtol=1e-13, atol=1e-15)


def test_logistic_learns_planted_labels():
    prob = synth.small_case(400, 300, 30_000, seed=11, k=8, rank=3, values="sign", test_frac=0.2)
    W0, H0 = synth.init_factors(400, 300, 8, 11)
    hp = oracle.Hyper(8, 0.01, 0.1, 0.0, 1.0)
    row, col, val = prob.row.numpy(), prob.col.numpy(), prob.val.numpy()
    J0 = oracle.objective(400, 300, row, col, val, W0.numpy(), H0.numpy(), hp.lam, loss="logistic")
    W, H, _ = oracle.train_ring(400, 300, row, col, val, W0.numpy(), H0.numpy(), hp, 4, 1, 30, loss="logistic")
    J = oracle.objective(400, 300, row, col, val, W, H, hp.lam, loss="logistic")
    d = np.einsum("ij,ij->i", W[prob.test_row.numpy()], H[prob.test_col.numpy()])
    acc = float(np.mean(np.sign(d) == prob.test_val.numpy()))
    print(f"logistic: J {J0:.1f} -> {J:.1f}, test accuracy {acc:.3f}")
    assert J < 0.6 * J0
    assert acc > 0.8
