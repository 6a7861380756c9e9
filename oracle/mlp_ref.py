"""Attribute network, losses and Adam: FP64 reference with BF16 rounding.

TEST INFRASTRUCTURE ONLY.

The network maps a Gaussian's embedding e_i (32-d) and the Fourier encoding
of the moving endpoint (the transmitter, 51-d) to per-subcarrier amplitude
and phase, as a shared form of the emission predictor of Eq. (1):
    x   = [e_i, gamma(x_tx)]                      (83-d, zero-padded to 96)
    h1  = relu(W1 x + b1)                         (64)
    h2  = relu(W2 h1 + b2)                        (64)
    o   = W3 h2 + b3                              (128 = 64 amplitudes, 64 phases)
    A_f = sigmoid(o_f - ln d),  phi_f = o_{64+f}, s_f = A_f exp(j phi_f)
with d = max(|x_tx - mu_i|, r_near): the log-distance bias of Eq. (1) kept
inside the sigmoid, applied to an amplitude instead of to Re/Im separately.
gamma(x) = (u, sin(2^k pi u), cos(2^k pi u)) for k = 0..7, u = x scaled to
[-1, 1] by the scene box (the order is u(3), then for each k: sin(3), cos(3)).

BF16 rounding (round to nearest even) is applied at the points where the GPU
feeds a BF16 matrix unit: e, gamma, the weights W1..W3, h1 and h2 after the
ReLU, and in the backward the gradients entering each product (d_o, dZ2,
dZ1).  Accumulation is FP64.  ``round_bf16=False`` turns every rounding off
(plain FP64 network), which is what the autograd pin compares against.
"""
from __future__ import annotations

import numpy as np

N_FREQ_BANDS = 8
EMB = 32
ENC = 3 + 6 * N_FREQ_BANDS  # 51
IN_PAD = 96
HID = 64


def bf16(x):
    """Round float64/float32 values to the nearest bfloat16 (ties to even),
    returned as float64.  Goes through the float32 bit pattern."""
    x32 = np.asarray(x, dtype=np.float32)
    b = x32.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = (b + 0x7FFF + lsb) >> 16
    out = (r << 16).astype(np.uint32).view(np.float32)
    # NaN stays NaN
    out = np.where(np.isnan(x32), np.float32(np.nan), out)
    return out.astype(np.float64)


def fourier(x, lo, hi):
    """gamma(x) for points x [..., 3] in the box [lo, hi]: [..., 51]."""
    x = np.asarray(x, np.float64)
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    u = 2.0 * (x - lo) / (hi - lo) - 1.0
    parts = [u]
    for k in range(N_FREQ_BANDS):
        parts.append(np.sin((2.0 ** k) * np.pi * u))
        parts.append(np.cos((2.0 ** k) * np.pi * u))
    return np.concatenate(parts, axis=-1)


def _r(x, on):
    return bf16(x) if on else np.asarray(x, np.float64)


def forward(W1, b1, W2, b2, W3, b3, E, tx, mean, r_near, lo, hi, round_bf16=True, F=64):
    """Attributes for every (query, Gaussian): E [n,32], tx [S,3], mean [3,n].
    Returns dict with attr [S,n,F,2] and the intermediates."""
    on = round_bf16
    W1r, W2r, W3r = _r(W1, on), _r(W2, on), _r(W3, on)
    Er = _r(E, on)
    g = _r(fourier(tx, lo, hi), on)                        # [S, 51]
    S, n = g.shape[0], Er.shape[0]
    x = np.zeros((S, n, IN_PAD))
    x[:, :, :EMB] = Er[None]
    x[:, :, EMB:EMB + ENC] = g[:, None, :]
    z1 = x @ W1r.T + b1                                    # [S, n, 64]
    h1 = _r(np.maximum(z1, 0.0), on)
    z2 = h1 @ W2r.T + b2
    h2 = _r(np.maximum(z2, 0.0), on)
    o = h2 @ W3r.T + b3                                    # [S, n, 2F]
    m = np.asarray(mean, np.float64).T                     # [n, 3]
    d = np.linalg.norm(m[None, :, :] - np.asarray(tx, np.float64)[:, None, :], axis=-1)
    d = np.maximum(d, r_near)
    amp = 1.0 / (1.0 + np.exp(-(o[..., :F] - np.log(d)[..., None])))
    ph = o[..., F:]
    attr = np.stack([amp * np.cos(ph), amp * np.sin(ph)], axis=-1)
    return dict(attr=attr, x=x, z1=z1, h1=h1, z2=z2, h2=h2, o=o, amp=amp, ph=ph, d=d,
                W1r=W1r, W2r=W2r, W3r=W3r, g=g)


def backward(fw, d_attr, round_bf16=True, F=64):
    """Gradients of sum(d_attr * attr) with respect to W1..b3 and E.
    d_attr [S,n,F,2]."""
    on = round_bf16
    amp, ph = fw["amp"], fw["ph"]
    gre, gim = d_attr[..., 0], d_attr[..., 1]
    dA = gre * np.cos(ph) + gim * np.sin(ph)
    dphi = amp * (-gre * np.sin(ph) + gim * np.cos(ph))
    do = np.concatenate([dA * amp * (1.0 - amp), dphi], axis=-1)   # [S,n,2F]
    dor = _r(do, on)
    dW3 = np.einsum("sno,snh->oh", dor, fw["h2"])
    db3 = do.sum(axis=(0, 1))
    dh2 = dor @ fw["W3r"]
    dz2 = dh2 * (fw["z2"] > 0)
    dz2r = _r(dz2, on)
    dW2 = np.einsum("sno,snh->oh", dz2r, fw["h1"])
    db2 = dz2.sum(axis=(0, 1))
    dh1 = dz2r @ fw["W2r"]
    dz1 = dh1 * (fw["z1"] > 0)
    dz1r = _r(dz1, on)
    dW1 = np.zeros_like(fw["W1r"])
    # embedding columns: products with the rounded dZ1; encoding columns and
    # bias: sums of the unrounded per-query dZ1
    dW1[:, :EMB] = np.einsum("snh,sne->he", dz1r, fw["x"][..., :EMB])
    dcs = dz1.sum(axis=1)                                          # [S, 64]
    dW1[:, EMB:EMB + ENC] = dcs.T @ fw["g"]
    db1 = dcs.sum(axis=0)
    dE = (dz1r @ fw["W1r"][:, :EMB]).sum(axis=0)                   # [n, 32]
    return dict(W1=dW1, b1=db1, W2=dW2, b2=db2, W3=dW3, b3=db3, E=dE)


def init(seed=0):
    """He-normal weights in [out, in] layout; W1 is [64, 96] with zero
    columns beyond the 83 inputs."""
    rng = np.random.default_rng(seed)
    W1 = np.zeros((HID, IN_PAD))
    W1[:, :EMB + ENC] = rng.normal(0, np.sqrt(2.0 / (EMB + ENC)), size=(HID, EMB + ENC))
    W2 = rng.normal(0, np.sqrt(2.0 / HID), size=(HID, HID))
    W3 = rng.normal(0, np.sqrt(2.0 / HID), size=(128, HID))
    return dict(W1=W1, b1=np.zeros(HID), W2=W2, b2=np.zeros(HID), W3=W3, b3=np.zeros(128))


def adam(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-15):
    """One textbook Adam step (Kingma and Ba), t >= 1; returns (p, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
