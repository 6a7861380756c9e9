"""FP64 oracle of the paper's own emission form: one small network per
Gaussian (Sec. 4.1, the directional neural predictor, Eq. (1)).

TEST INFRASTRUCTURE ONLY (see the package docstring): the product path never
imports this module.

Gaussian i owns a network f_i: R^3 -> R^2 of shape 3 -> 16 -> 2 (98
parameters: the implementation details and the hyper-parameter table) that
takes the receiver position; the transmitter enters through the path-loss
bias log d_i, d_i = |x_tx - mu_i|, and the emission is
    s_i = sigmoid(f_i(x_rx) - log d_i)
applied to the real and to the imaginary output separately.

Readings: the hidden activation is ReLU (not named in the paper); d_i is
floored at r_near (0.2 m), as for the attenuation of the renderer, so that log d_i
stays finite.  Parameter order per Gaussian: W1 [16][3] row-major, b1 [16],
W2 [2][16] row-major, b2 [2].
"""
from __future__ import annotations

import numpy as np

HIDDEN = 16
NPARAM = 3 * HIDDEN + HIDDEN + 2 * HIDDEN + 2   # 98
R_NEAR = 0.2


def unpack(P):
    P = np.asarray(P, np.float64)
    n = P.shape[0]
    W1 = P[:, :48].reshape(n, HIDDEN, 3)
    b1 = P[:, 48:64]
    W2 = P[:, 64:96].reshape(n, 2, HIDDEN)
    b2 = P[:, 96:98]
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
    n = W1.shape[0]
    dP = np.zeros((n, NPARAM))
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
        dP[:, 96:98] += du
        dP[:, 64:96] += np.einsum("nk,ni->nki", du, h).reshape(n, 32)
        dz = np.einsum("nk,nki->ni", du, W2) * (z > 0.0)
        dP[:, 48:64] += dz
        dP[:, :48] += np.einsum("ni,j->nij", dz, x).reshape(n, 48)
        # -log d: d/dmean of log|tx - mean| = -(tx - mean)/|.|^2 (zero where floored)
        dlogd = -du.sum(1)
        live = dist > r_near
        dmean[live] += (dlogd[live] / dist[live] ** 2)[:, None] * (-v[live])
    return dP, dmean
