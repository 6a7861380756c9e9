"""Dense FP64 PyTorch-CPU renderer, differentiated by autograd.

TEST INFRASTRUCTURE ONLY (gradient reference). A second, independent
implementation of the forward in ``oracle.c``: it evaluates every
(pixel, Gaussian) pair as a dense [H*W, n] tensor instead of looping, so it is
meant for small n (tens to a few hundred Gaussians).

Discrete decisions (alpha >= alpha_min, the T_min stop, the azimuth wrap,
the alpha_max clamp) are taken on detached values and then held fixed, so
autograd returns the derivative of the piecewise-smooth function on the
current piece. A clamped alpha (sigma G > alpha_max) therefore passes no
gradient to G or sigma.

Formulas: Sec. 3.2 (Sigma = R S S^T R^T), Sec. 4.2 (view transform,
equirectangular map, Sigma' = J V Sigma V^T J^T), Eq. (3) (compositing).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import DEFAULT_VIEW, params as _params


def r32_keys(mean: np.ndarray, rx) -> np.ndarray:
    """The FP32 distance key, evaluated with numpy float32 (IEEE, one
    rounding per operation, no fusion)."""
    m = np.asarray(mean, dtype=np.float32)
    r = np.asarray(rx, dtype=np.float32).reshape(3, 1)
    d = (m - r).astype(np.float32)
    sq = (d * d).astype(np.float32)
    s = (sq[0] + sq[1]).astype(np.float32)
    s = (s + sq[2]).astype(np.float32)
    return np.sqrt(s).astype(np.float32)


def quat_to_rot(q: torch.Tensor) -> torch.Tensor:
    """q: [4, n] (w, x, y, z), any norm -> R: [n, 3, 3]."""
    q = q / torch.linalg.norm(q, dim=0, keepdim=True)
    w, x, y, z = q[0], q[1], q[2], q[3]
    R = torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], -2)
    return R


def project(mean, log_scale, quat, opacity_logit, rx, H, W, prm, tx=None, view=None):
    """Differentiable per-Gaussian quantities (all float64 tensors)."""
    dilation, r_near, apow, aref = prm[3], prm[4], prm[5], int(prm[6])
    V = torch.as_tensor(DEFAULT_VIEW if view is None else view, dtype=torch.float64)
    rx_t = torch.as_tensor(np.asarray(rx, dtype=np.float32), dtype=torch.float64)
    tx_t = rx_t if tx is None else torch.as_tensor(np.asarray(tx, dtype=np.float32), dtype=torch.float64)
    s2 = torch.exp(2.0 * log_scale)                       # [3, n]
    R = quat_to_rot(quat)                                 # [n, 3, 3]
    Sig = R @ torch.diag_embed(s2.T) @ R.transpose(1, 2)  # [n, 3, 3]
    t = (V @ (mean - rx_t[:, None])).T                    # [n, 3]
    Sv = V @ Sig @ V.T
    x, y, z = t[:, 0], t[:, 1], t[:, 2]
    r = torch.sqrt(x * x + y * y + z * z)
    az = torch.atan2(x, z)
    el = torch.asin(y / r)
    px = (az / math.pi + 1.0) * W / 2.0
    py = 2.0 * el * H / math.pi
    rho = torch.sqrt(x * x + z * z)
    rho = torch.maximum(rho, 1e-6 * r)
    kx, ky = W / (2.0 * math.pi), 2.0 * H / math.pi
    zero = torch.zeros_like(x)
    J = torch.stack([
        torch.stack([kx * z / rho ** 2, zero, -kx * x / rho ** 2], -1),
        torch.stack([-ky * x * y / (r * r * rho), ky * rho / (r * r), -ky * z * y / (r * r * rho)], -1),
    ], -2)                                                # [n, 2, 3]
    Sp = J @ Sv @ J.transpose(1, 2)
    a = Sp[:, 0, 0] + dilation
    b = Sp[:, 0, 1]
    c = Sp[:, 1, 1] + dilation
    det = a * c - b * b
    sigma = torch.sigmoid(opacity_logit)
    ref = tx_t if aref == 1 else rx_t
    dist = torch.linalg.norm(mean - ref[:, None], dim=0)
    att = 1.0 / torch.clamp(dist, min=r_near) ** apow
    return dict(px=px, py=py, ca=c / det, cb=-b / det, cc=a / det, sigma=sigma, att=att,
                s00=a, s01=b, s11=c)


def render(mean, log_scale, quat, opacity_logit, attr, rx, H, W, prm=None, tx=None, view=None,
           keys=None):
    """Dense forward. Tensors are float64 (requires_grad as wanted):
    mean/log_scale [3,n], quat [4,n], opacity_logit [n], attr [n,F] or
    [n,F,2]. Returns out [F,H,W] or [F,H,W,2], plus T_final and n_contrib."""
    prm = _params() if prm is None else np.asarray(prm)
    amin, amax, tmin, r_near = float(prm[0]), float(prm[1]), float(prm[2]), float(prm[4])
    n = opacity_logit.shape[0]
    if keys is None:
        keys = r32_keys(mean.detach().numpy(), rx)
    g = project(mean, log_scale, quat, opacity_logit, rx, H, W, prm, tx=tx, view=view)
    sig_d = g["sigma"].detach().numpy()
    keep = (keys >= np.float32(r_near)) & (sig_d >= amin)
    idx = np.array(sorted(np.nonzero(keep)[0], key=lambda i: (keys[i], i)), dtype=np.int64)
    cplx = attr.dim() == 3
    F = attr.shape[1]
    HW = H * W
    if idx.size == 0:
        shape = (F, H, W, 2) if cplx else (F, H, W)
        return dict(out=torch.zeros(shape, dtype=torch.float64), T_final=torch.ones(H, W, dtype=torch.float64),
                    n_contrib=np.zeros((H, W), np.int64), order=idx)
    it = torch.as_tensor(idx)
    rows = torch.arange(H, dtype=torch.float64).repeat_interleave(W) + 0.5
    cols = torch.arange(W, dtype=torch.float64).repeat(H) + 0.5
    dx = cols[:, None] - g["px"][it][None, :]
    dxd = dx.detach()
    shift = torch.where(dxd >= 0.5 * W, -float(W), torch.where(dxd < -0.5 * W, float(W), 0.0))
    dx = dx + shift
    dy = rows[:, None] - g["py"][it][None, :]
    q = g["ca"][it] * dx * dx + 2.0 * g["cb"][it] * dx * dy + g["cc"][it] * dy * dy
    sg = g["sigma"][it] * torch.exp(-0.5 * q)              # [HW, m]
    alpha = torch.where(sg.detach() < amax, sg, torch.full_like(sg, amax))
    ad = alpha.detach()
    contrib = ad >= amin
    # transmittance before each entry, non-contributors pass T unchanged
    one_minus = torch.where(contrib, 1.0 - ad, torch.ones_like(ad))
    Tb = torch.cumprod(torch.cat([torch.ones(HW, 1, dtype=torch.float64), one_minus[:, :-1]], 1), 1)
    stop = contrib & (Tb * (1.0 - ad) < tmin)
    m = idx.size
    first = torch.where(stop.any(1), stop.float().argmax(1), torch.full((HW,), m))
    active = contrib & (torch.arange(m)[None, :] < first[:, None])
    # differentiable transmittance with the decisions held fixed
    om = torch.where(active, 1.0 - alpha, torch.ones_like(alpha))
    T = torch.cumprod(torch.cat([torch.ones(HW, 1, dtype=torch.float64), om[:, :-1]], 1), 1)
    w = torch.where(active, T * alpha, torch.zeros_like(alpha)) * g["att"][it][None, :]
    if cplx:
        v = attr[it].reshape(m, F * 2)
        out = (w @ v).reshape(H, W, F, 2).permute(2, 0, 1, 3)
    else:
        out = (w @ attr[it]).reshape(H, W, F).permute(2, 0, 1)
    T_final = torch.prod(om, 1).reshape(H, W)
    return dict(out=out, T_final=T_final, n_contrib=active.sum(1).reshape(H, W).numpy(), order=idx)


def to_tensors(scene: dict, attr, requires_grad=False):
    t = {k: torch.tensor(np.asarray(scene[k], dtype=np.float64), requires_grad=requires_grad)
         for k in ("mean", "log_scale", "quat", "opacity_logit")}
    a = torch.tensor(np.asarray(attr, dtype=np.float64), requires_grad=requires_grad)
    return t, a
