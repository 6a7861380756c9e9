"""FP64 oracle of the paper's own emission form: one small network per
Gaussian (Sec. 4.1, the directional neural predictor, Eq. (1)).

TEST INFRASTRUCTURE ONLY (see the package docstring): the product path never
imports this module.

Gaussian i owns a network f_i: R^3 -> R^2 of shape 3 -> 16 -> 2 (98
parameters: the implementation details and the hyper-parameter table; the
ablation on the hidden width also uses 8 and 64, and every function here
takes the width from the parameter count 6 H + 2) that
takes the receiver position; the transmitter enters through the path-loss
bias log d_i, d_i = |x_tx - mu_i|, and the emission is
    s_i = sigmoid(f_i(x_rx) - log d_i)
applied to the real and to the imaginary output separately.

Readings: the hidden activation is ReLU (not named in the paper); d_i is
floored at r_near (0.2 m), as for the attenuation of the renderer, so that log d_i
stays finite.  Parameter order per Gaussian: W1 [H][3] row-major, b1 [H],
W2 [2][H] row-major, b2 [2].
"""
from __future__ import annotations

import numpy as np

HIDDEN = 16                                     # the paper's width; 8 and 64 for the width sweep
NPARAM = 3 * HIDDEN + HIDDEN + 2 * HIDDEN + 2   # 98
R_NEAR = 0.2


def nparam(hidden):
    return 6 * hidden + 2


def unpack(P):
    """Parameter order per Gaussian, for a hidden width H = (len - 2) / 6:
    W1 [H][3], b1 [H], W2 [2][H], b2 [2]."""
    P = np.asarray(P, np.float64)
    n, k = P.shape
    H = (k - 2) // 6
    assert 6 * H + 2 == k
    W1 = P[:, :3 * H].reshape(n, H, 3)
    b1 = P[:, 3 * H:4 * H]
    W2 = P[:, 4 * H:6 * H].reshape(n, 2, H)
    b2 = P[:, 6 * H:6 * H + 2]
    return W1, b1, W2, b2


def forward(P, mean, rx, tx, r_near=R_NEAR):
    """P [n][98], mean [n][3], rx [Q][3], tx [Q][3] -> s [Q][n][2] (Re, Im)."""
    W1, b1, W2, b2 = unpack(P)
    mean = np.asarray(mean, np.float64)
    out = []
    for q in range(len(rx)):
        z = np.einsum("nij,j->ni", W1, np.asarray(rx[q], np.float64)) + b1
        h = np.maximum(z, 0.0)
        f = np.einsum("nki,ni->nk", W2, h) + b2
        d = np.maximum(np.linalg.norm(np.asarray(tx[q], np.float64) - mean, axis=1), r_near)
        out.append(1.0 / (1.0 + np.exp(-(f - np.log(d)[:, None]))))
    return np.stack(out)


def backward(P, mean, rx, tx, ds, r_near=R_NEAR):
    """Gradients of sum(ds * s) with respect to P [n][98] and mean [n][3]
    (ds [Q][n][2]); summed over the queries."""
    W1, b1, W2, b2 = unpack(P)
    mean = np.asarray(mean, np.float64)
    ds = np.asarray(ds, np.float64)
    n, H = W1.shape[0], W1.shape[1]
    dP = np.zeros((n, 6 * H + 2))
    dmean = np.zeros((n, 3))
    for q in range(len(rx)):
        x = np.asarray(rx[q], np.float64)
        z = np.einsum("nij,j->ni", W1, x) + b1
        h = np.maximum(z, 0.0)
        f = np.einsum("nki,ni->nk", W2, h) + b2
        v = np.asarray(tx[q], np.float64) - mean
        dist = np.linalg.norm(v, axis=1)
        d = np.maximum(dist, r_near)
        s = 1.0 / (1.0 + np.exp(-(f - np.log(d)[:, None])))
        du = ds[q] * s * (1.0 - s)                    # d/d(f - log d)
        dP[:, 6 * H:6 * H + 2] += du
        dP[:, 4 * H:6 * H] += np.einsum("nk,ni->nki", du, h).reshape(n, 2 * H)
        dz = np.einsum("nk,nki->ni", du, W2) * (z > 0.0)
        dP[:, 3 * H:4 * H] += dz
        dP[:, :3 * H] += np.einsum("ni,j->nij", dz, x).reshape(n, 3 * H)
        # -log d: d/dmean of log|tx - mean| = -(tx - mean)/|.|^2 (zero where floored)
        dlogd = -du.sum(1)
        live = dist > r_near
        dmean[live] += (dlogd[live] / dist[live] ** 2)[:, None] * (-v[live])
    return dP, dmean
