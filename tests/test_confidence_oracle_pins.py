"""Pins of the confidence-head oracle (Sec. 4.2, Eq. (6)) to facts the paper
and the mathematics fix, not to the oracle itself:

* the optimum of Eq. (6) over C is C* = alpha / L_task (the paper states it):
  with the network's output set to log(alpha / L - 1), every gradient is zero
  and moving the output either way raises the objective;
* for L_task >= alpha the optimum over C > 1 is at the floor (the paper:
  the confidence saturates at 1), so the gradient pushes g down;
* C > 1 for every output, and C -> 1 as g -> -inf;
* alpha = 0 reduces Eq. (6) to C * L_task;
* every analytic gradient matches central finite differences of the loss.
"""
import numpy as np
import pytest

from oracle import confidence_ref as cr


def params(seed, scale=0.5):
    r = np.random.default_rng(seed)
    return (r.normal(0, scale, (32, 3)), r.normal(0, scale, 32), r.normal(0, scale, 32), float(r.normal(0, scale)))


def total(x, L, W1, b1, w2, b2, alpha):
    _, _, C = cr.forward(x, W1, b1, w2, b2)
    return float(cr.loss(L, C, alpha).sum())


def test_gradients_match_finite_differences():
    r = np.random.default_rng(1)
    x = r.normal(0, 2, (5, 3))
    L = r.uniform(0.01, 0.6, 5)
    W1, b1, w2, b2 = params(2)
    g = cr.backward(x, L, W1, b1, w2, b2, 0.3)
    eps = 1e-6
    for name, arr in (("dW1", W1), ("db1", b1), ("dw2", w2)):
        num = np.zeros_like(arr)
        for idx in np.ndindex(arr.shape):
            a = arr.copy(); a[idx] += eps
            b = arr.copy(); b[idx] -= eps
            args_p = {"dW1": (a, b1, w2, b2), "db1": (W1, a, w2, b2), "dw2": (W1, b1, a, b2)}[name]
            args_m = {"dW1": (b, b1, w2, b2), "db1": (W1, b, w2, b2), "dw2": (W1, b1, b, b2)}[name]
            num[idx] = (total(x, L, *args_p, 0.3) - total(x, L, *args_m, 0.3)) / (2 * eps)
        assert np.allclose(g[name], num, rtol=1e-6, atol=1e-8), name
    num = (total(x, L, W1, b1, w2, b2 + eps, 0.3) - total(x, L, W1, b1, w2, b2 - eps, 0.3)) / (2 * eps)
    assert abs(g["db2"] - num) <= 1e-6 * max(1.0, abs(num))
    # dL/dL_task = C: perturb one sample's task loss
    for i in range(5):
        Lp = L.copy(); Lp[i] += eps
        Lm = L.copy(); Lm[i] -= eps
        num = (total(x, Lp, W1, b1, w2, b2, 0.3) - total(x, Lm, W1, b1, w2, b2, 0.3)) / (2 * eps)
        assert abs(g["dL_dtask"][i] - num) <= 1e-6 * num


@pytest.mark.parametrize("L", [0.01, 0.1, 0.29])
def test_optimum_is_alpha_over_task_loss(L):
    alpha = 0.3
    W1, b1, _, _ = params(3)
    w2 = np.zeros(32)
    b2 = float(np.log(alpha / L - 1.0))     # g = b2, so C = alpha / L
    x = np.array([[0.3, -1.2, 2.0]])
    g = cr.backward(x, [L], W1, b1, w2, b2, alpha)
    assert abs(g["C"][0] - alpha / L) <= 1e-12 * alpha / L
    for k in ("dW1", "db1", "dw2"):
        assert np.abs(g[k]).max() <= 1e-12
    assert abs(g["db2"]) <= 1e-12
    f0 = total(x, [L], W1, b1, w2, b2, alpha)
    for d in (-1e-3, 1e-3):
        assert total(x, [L], W1, b1, w2, b2 + d, alpha) > f0


@pytest.mark.parametrize("seed", range(4))
def test_hard_samples_push_confidence_to_the_floor(seed):
    # L_task >= alpha: dL/dC = L - alpha / C > 0 for every C > 1, so the
    # gradient with respect to the output bias is positive (g decreases)
    W1, b1, w2, b2 = params(10 + seed)
    x = np.random.default_rng(seed).normal(0, 1, (1, 3))
    for L in (0.3, 0.5, 2.0):
        assert cr.backward(x, [L], W1, b1, w2, b2, 0.3)["db2"] > 0.0


def test_confidence_above_one_and_floor_limit():
    W1, b1, w2, b2 = params(4)
    x = np.random.default_rng(5).normal(0, 3, (100, 3))
    _, _, C = cr.forward(x, W1, b1, w2, b2)
    assert (C > 1.0).all()
    _, _, C = cr.forward(x, W1, b1, np.zeros(32), -50.0)
    assert np.abs(C - 1.0).max() <= 1e-21 + 2e-22 and (C >= 1.0).all()


def test_alpha_zero_is_the_weighted_task_loss():
    W1, b1, w2, b2 = params(6)
    x = np.random.default_rng(7).normal(0, 1, (4, 3))
    L = np.array([0.1, 0.2, 0.3, 0.4])
    g = cr.backward(x, L, W1, b1, w2, b2, 0.0)
    assert np.allclose(g["loss"], g["C"] * L, rtol=0, atol=1e-15)


def test_hand_computed_head():
    # x = (0.5, -1, 2); unit j < 8 reads input j mod 3 with weight 1:
    #   z = (0.75, -0.5, -1, 1.5, -1, 1, -0.5, 1), h = (0.75, 0, 0, 1.5, 0, 1, 0, 1)
    # units 8..31 read (1, 1, 1) with bias -10 (dead) and output weight 7,
    # which only a missing ReLU would let through.
    # g = 0.75*1 + 1.5*0.5 + 1*(-1) + 1*(-0.25) + b2 = 0.25 + 0.5 = 0.75
    W1 = np.zeros((32, 3))
    b1 = np.full(32, -10.0)
    for j in range(8):
        W1[j, j % 3] = 1.0
    W1[8:] = 1.0
    b1[:8] = [0.25, 0.5, -3.0, 1.0, 0.0, -1.0, -1.0, 2.0]
    w2 = np.full(32, 7.0)
    w2[:8] = [1.0, -2.0, 3.0, 0.5, 2.0, -1.0, 4.0, -0.25]
    h, g, C = cr.forward(np.array([[0.5, -1.0, 2.0]]), W1, b1, w2, 0.5)
    assert np.allclose(h[0, :8], [0.75, 0, 0, 1.5, 0, 1, 0, 1], rtol=0, atol=1e-15)
    assert abs(g[0] - 0.75) <= 1e-15
    assert abs(C[0] - (1.0 + np.exp(0.75))) <= 1e-15
    # Eq. (6) at L_task = 0.2, alpha = 0.3: C L - alpha log C
    Lc = cr.loss([0.2], C, 0.3)[0]
    assert abs(Lc - ((1.0 + np.exp(0.75)) * 0.2 - 0.3 * np.log(1.0 + np.exp(0.75)))) <= 1e-15
    # the output-bias gradient by hand: (L - alpha / C) (C - 1)
    d = cr.backward(np.array([[0.5, -1.0, 2.0]]), [0.2], W1, b1, w2, 0.5, 0.3)
    c = 1.0 + np.exp(0.75)
    assert abs(d["db2"] - (0.2 - 0.3 / c) * (c - 1.0)) <= 1e-15
    # hidden-unit gradients reach the live units only: dw2 = dg h
    assert np.allclose(d["dw2"][:8], (0.2 - 0.3 / c) * (c - 1.0) * np.array([0.75, 0, 0, 1.5, 0, 1, 0, 1]),
                       rtol=0, atol=1e-15)
    assert np.all(d["dW1"][8:] == 0) and np.all(d["db1"][[1, 2, 4, 6]] == 0)
