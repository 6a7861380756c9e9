"""Confidence head and confidence-weighted loss (Sec. 4.2, Eq. (6)) on the GPU
against the FP64 oracle (oracle/confidence_ref.py) through the C ABI.

Inputs are FP32-rounded before both sides see them; samples whose hidden
pre-activations come within 1e-3 of the ReLU kink are redrawn, so the two
sides take the same ReLU decisions.  Tolerance: C and the per-sample loss to
2e-6 relative (a few FP32 roundings of exp and log); the weight gradients,
FP32 sums over the samples, to 1e-4 of their largest magnitude (2e-3 at
65536 samples).
"""
import numpy as np
import pytest
import torch

import paper_2511_22793_amd as gs
from paper_2511_22793_amd._lib import GS_ERR_CAPACITY, GS_ERR_INVALID_ARG, GsError
from oracle import confidence_ref as cr

pytestmark = pytest.mark.gpu


def case(n, seed):
    r = np.random.default_rng(seed)
    W1 = r.normal(0, 0.5, (32, 3)).astype(np.float32)
    b1 = r.normal(0, 0.5, 32).astype(np.float32)
    w2 = r.normal(0, 0.3, 32).astype(np.float32)
    b2 = np.array([r.normal(0, 0.3)], np.float32)
    x = r.normal(0, 2.0, (n, 3)).astype(np.float32)
    while True:
        z = x.astype(np.float64) @ W1.T.astype(np.float64) + b1
        bad = (np.abs(z) < 1e-3).any(1)
        if not bad.any():
            break
        x[bad] = r.normal(0, 2.0, (int(bad.sum()), 3)).astype(np.float32)
    L = r.uniform(0.005, 0.6, n).astype(np.float32)
    return x, L, dict(W1=W1, b1=b1, w2=w2, b2=b2)


def run(x, L, w, alpha):
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    conf, loss, g = gs.confidence_loss(d(x), d(L), {k: d(v) for k, v in w.items()}, alpha)
    torch.cuda.synchronize()
    return conf.cpu().numpy(), loss.cpu().numpy(), {k: v.cpu().numpy() for k, v in g.items()}


@pytest.mark.parametrize("n,seed,alpha", [(1, 1, 0.3), (7, 2, 0.3), (16, 3, 0.3), (1000, 4, 0.3), (777, 5, 0.0),
                                          (4096, 10, 0.3),
                                          # the multi-workgroup path: one chunk past the single
                                          # workgroup's limit, a ragged last chunk, and more chunks
                                          # than workgroups (1024 x 256 = 262144)
                                          (4097, 11, 0.3), (65536, 6, 0.3), (300_001, 12, 0.3)])
def test_confidence_matches_oracle(n, seed, alpha):
    x, L, w = case(n, seed)
    conf, loss, g = run(x, L, w, alpha)
    ref = cr.backward(x, L, w["W1"], w["b1"], w["w2"], float(w["b2"][0]), alpha)
    assert np.allclose(conf, ref["C"], rtol=2e-6, atol=0)
    assert np.allclose(loss, ref["loss"], rtol=2e-6, atol=2e-6 * np.abs(ref["loss"]).max())
    frac = 2e-3 if n > 10000 else 1e-4
    for k, rk in (("W1", "dW1"), ("b1", "db1"), ("w2", "dw2"), ("b2", "db2")):
        want = np.atleast_1d(np.asarray(ref[rk], np.float64))
        got = g[k].astype(np.float64).reshape(want.shape)
        assert np.abs(got - want).max() <= frac * np.abs(want).max() + 1e-7, k


def test_deterministic_and_input_checks():
    x, L, w = case(300, 9)
    a = run(x, L, w, 0.3)
    b = run(x, L, w, 0.3)
    for k in a[2]:
        assert np.array_equal(a[2][k], b[2][k])
    d = lambda arr: torch.from_numpy(np.ascontiguousarray(arr)).cuda()  # noqa: E731
    wt = {k: d(v) for k, v in w.items()}
    # the multi-workgroup path is deterministic too
    x2, L2, w2 = case(20_000, 13)
    a = run(x2, L2, w2, 0.3)
    b = run(x2, L2, w2, 0.3)
    for k in a[2]:
        assert np.array_equal(a[2][k], b[2][k])
    with pytest.raises(GsError) as e:
        gs.confidence_loss(d(x), d(L), wt, alpha=-0.1)
    assert e.value.status == GS_ERR_INVALID_ARG
    with pytest.raises(GsError) as e:
        gs.confidence_loss(d(x), d(L), wt, alpha=float("nan"))
    assert e.value.status == GS_ERR_INVALID_ARG
