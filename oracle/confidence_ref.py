"""FP64 oracle of the confidence head and the confidence-weighted loss.

TEST INFRASTRUCTURE ONLY (see the package docstring): the product path never
imports this module.

Sec. 4.2 (the paragraph on confidence-weighted optimization), Eq. (6): a
small network g maps the receiver position x_rx (3 values) to a scalar, the
confidence is C = 1 + exp(g(x_rx)) (always above 1), and the objective of
one sample is

    L_conf = C * L_task - alpha * log C.

The training hyper-parameter table gives g the shape 3 -> 32 -> 1 and
alpha = 0.3.  Reading (the paper does not name the hidden activation): ReLU, as in the
attribute network, h = relu(W1 x + b1), g = w2 . h + b2.  A batch of n
samples is the sum of the per-sample objectives, so the weight gradients are
sums over the samples.

Derivatives, from the definitions above:
    dL_conf / dL_task = C
    dL_conf / dC      = L_task - alpha / C        (zero at C* = alpha / L_task)
    dC / dg           = exp(g) = C - 1
"""
from __future__ import annotations

import numpy as np

ALPHA = 0.3      # hyper-parameter table
HIDDEN = 32      # 3 -> 32 -> 1


def forward(x, W1, b1, w2, b2):
    """x: (n, 3); W1: (32, 3); b1: (32,); w2: (32,); b2: scalar.
    Returns (h (n, 32), g (n,), C (n,))."""
    x = np.asarray(x, np.float64)
    z = x @ np.asarray(W1, np.float64).T + np.asarray(b1, np.float64)
    h = np.maximum(z, 0.0)
    g = h @ np.asarray(w2, np.float64) + float(b2)
    C = 1.0 + np.exp(g)
    return h, g, C


def loss(task_loss, C, alpha=ALPHA):
    """Eq. (6) per sample."""
    return np.asarray(C, np.float64) * np.asarray(task_loss, np.float64) - alpha * np.log(C)


def backward(x, task_loss, W1, b1, w2, b2, alpha=ALPHA):
    """Per-sample C and L_conf, dL/dL_task (= C) and the gradients of the
    batch sum of L_conf with respect to W1, b1, w2, b2."""
    x = np.asarray(x, np.float64)
    L = np.asarray(task_loss, np.float64)
    h, g, C = forward(x, W1, b1, w2, b2)
    Lc = loss(L, C, alpha)
    dg = (L - alpha / C) * (C - 1.0)                 # chain: dL/dC * dC/dg
    dw2 = dg @ h
    db2 = float(dg.sum())
    dh = np.outer(dg, np.asarray(w2, np.float64)) * (h > 0.0)
    dW1 = dh.T @ x
    db1 = dh.sum(0)
    return dict(C=C, loss=Lc, dL_dtask=C.copy(), dW1=dW1, db1=db1, dw2=dw2, db2=db2)
