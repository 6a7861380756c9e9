"""The confidence-weighted objective of Eq. (6) inside the training step
(LearnedScene(confidence=True)), against the same step without it and
against the confidence oracle.

With one receiver shared by the batch's sets, C = 1 + exp(g(x_rx)) is one
number per step; the objective (1/S) sum_b [C L_b - alpha log C] then has
model gradients C times the task-loss gradients, and the head's gradients of
the batch sum.  From identical states:
* C equals the FP64 oracle's head at the receiver (2e-6 relative);
* the task losses equal the plain step's (the scale touches no loss);
* every geometric gradient is C times the plain step's (the backward tests'
  tolerance), the network gradients within the BF16 flip bound (2e-2 of the
  tensor's max: a scaled upstream can round a BF16 intermediate the other
  way);
* the head's gradients equal the oracle's for the step's task losses
  (1e-4 of the largest entry);
* Adam moved the head's weights.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import confidence_ref as cr
from paper_2511_22793_amd import train
from test_gpu_backward import compare

pytestmark = pytest.mark.gpu

LO, HI = [-5.0, -5.0, 0.0], [5.0, 5.0, 3.0]


def _head(seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    return {"W1": torch.randn(32, 3, generator=g) * 0.8, "b1": torch.randn(32, generator=g) * 0.5,
            "w2": torch.randn(32, generator=g) * 0.2, "b2": torch.full((1,), 0.6)}


def test_confidence_weighted_step():
    n, B = 4000, 4
    rx = [0.3, -0.2, 0.5]
    sc = synth.scene(n, seed=71, lo=[-3, -3, 0.1], hi=[3, 3, 2.5])
    emb = synth.embeddings(n, seed=72)
    w = train.init_weights(73)
    head = _head(74)
    tx = torch.from_numpy(synth.points(B, seed=75)).cuda()
    target = torch.from_numpy(synth.normal((B, train.F, 90, 360, 2), 0.05, seed=76)).cuda()
    tmean = train.spatial_mean(target, True)
    plain = train.LearnedScene(sc, emb, w, rx, B, LO, HI)
    conf = train.LearnedScene(sc, emb, w, rx, B, LO, HI, confidence=True, conf_weights=head)
    plain.train_step(tx, target, target_mean=tmean)
    conf.train_step(tx, target, target_mean=tmean)
    torch.cuda.synchronize()

    x = np.tile(np.asarray(rx, np.float64), (B, 1))
    hw = {k: v.double().numpy() for k, v in head.items()}
    L = conf.loss.double().cpu().numpy()
    ref = cr.backward(x, L, hw["W1"], hw["b1"], hw["w2"], float(hw["b2"][0]), conf.conf_alpha)
    C = conf.conf_c.double().cpu().numpy()
    assert np.allclose(C, ref["C"], rtol=2e-6, atol=0), (C, ref["C"])
    assert np.allclose(L, plain.loss.double().cpu().numpy(), rtol=1e-5, atol=0)
    assert np.allclose(conf.conf_loss.double().cpu().numpy(), ref["loss"], rtol=2e-6, atol=1e-7)
    c = float(C[0])
    assert c > 1.5, "a scale away from 1 (the test would not see it otherwise)"
    for k, v in plain.ggrads.items():
        if k == "d_attr":
            continue
        compare(conf.ggrads[k].double().cpu().numpy(), c * v.double().cpu().numpy(), "scaled " + k)
    for k, v in plain.mgrads.items():
        a, b = conf.mgrads[k].double().cpu().numpy(), c * v.double().cpu().numpy()
        assert np.abs(a - b).max() <= 2e-2 * np.abs(b).max() + 1e-30, "network gradient %s" % k
    for k, rk in (("W1", "dW1"), ("b1", "db1"), ("w2", "dw2"), ("b2", "db2")):
        want = np.atleast_1d(np.asarray(ref[rk], np.float64))
        got = conf.conf_grads[k].double().cpu().numpy().reshape(want.shape)
        assert np.abs(got - want).max() <= 1e-4 * np.abs(want).max() + 1e-7, k
    for k in head:
        assert not torch.equal(conf.conf_w[k].cpu(), head[k]), "Adam moved the head's %s" % k


def test_confidence_requires_the_fused_pass():
    sc = synth.scene(100, seed=1)
    with pytest.raises(ValueError):
        train.LearnedScene(sc, synth.embeddings(100, seed=2), train.init_weights(3), [0, 0, 0], 2, LO, HI,
                           loss_mode="two_pass", confidence=True)
