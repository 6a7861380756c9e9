"""FP64 oracle of the training losses on rendered spectra.

TEST INFRASTRUCTURE ONLY (see the package docstring): the product path never
imports this module.

Spectra are stacked per set: zhat, z [S][F][H][W] (real) or [S][F][H][W][2]
(complex, interleaved re/im).

* Channel estimate (Eq. (2)): the coherent spatial mean of each channel,
  h_f = (1/(H W)) sum_p z_f(p), real and imaginary parts separately.
* Training loss for complex spectra (Eq. (4) read as the "phase-aware" term;
  the pixel term is a reading): per set
      L_b = (1/(F H W)) sum_{f,p} |zhat - z|^2 + lambda_ch sum_f |hhat_f - h_f|^2
  and the batch loss is the mean over sets.  Its gradient follows from the
  definition: dL/dzhat = (2 (zhat - z) / (F H W) + lambda_ch 2 (hhat - h) / (H W)) / S.
* Magnitude-spectrum loss (Eq. (5)): per set
      L_b = (1 - lambda_1) L1(zhat, z) + lambda_1 (1 - SSIM(zhat, z)),
  lambda_1 = 0.2 (hyper-parameter table), L1 = mean absolute error over
  channels and pixels.  SSIM reading (the paper names the index only): the
  standard structural similarity of Wang et al. (2004) as 3D Gaussian
  splatting computes it -- an 11 x 11 Gaussian window with sigma 1.5,
  normalised to sum 1, applied as a "same"-size filter with zero padding
  (no wrap at the azimuth seam), constants C1 = 0.01^2 and C2 = 0.03^2 (a
  dynamic range of 1), the SSIM map averaged over all pixels and channels.
  The gradient is that of the definition, taken by torch autograd in FP64;
  at |zhat - z| = 0 the L1 term contributes 0 (the sign's subgradient).
"""
from __future__ import annotations

import numpy as np
import torch

LAMBDA_1 = 0.2            # L1 / SSIM weight (hyper-parameter table)
SSIM_WIN = 11
SSIM_SIGMA = 1.5
SSIM_C1 = 0.01 ** 2
SSIM_C2 = 0.03 ** 2


def spatial_mean(z, is_complex):
    """Eq. (2): [S][F][H][W](2) -> [S][F](2)."""
    z = np.asarray(z, np.float64)
    return z.mean(axis=(2, 3))


def l2_channel_loss(zhat, z, is_complex, lambda_ch=1.0):
    """Per-set loss L_b [S], spatial means hhat [S][F](2), and dL/dzhat for
    L = mean_b L_b (same layout as zhat)."""
    zh = np.asarray(zhat, np.float64)
    zt = np.asarray(z, np.float64)
    S, F, H, W = zh.shape[:4]
    diff = zh - zt
    hh = spatial_mean(zh, is_complex)
    ht = spatial_mean(zt, is_complex)
    dm = hh - ht                                   # [S][F](2)
    pix = (diff ** 2).reshape(S, -1).sum(1) / (F * H * W)
    chan = (dm ** 2).reshape(S, -1).sum(1)
    L = pix + lambda_ch * chan
    dmb = dm[:, :, None, None] if not is_complex else dm[:, :, None, None, :]
    grad = (2.0 * diff / (F * H * W) + lambda_ch * 2.0 * dmb / (H * W)) / S
    return L, hh, grad


def _window(size=SSIM_WIN, sigma=SSIM_SIGMA):
    """1-D Gaussian weights, normalised to sum 1 (the 2-D window is their
    outer product)."""
    k = np.arange(size, dtype=np.float64) - (size - 1) / 2.0
    g = np.exp(-k * k / (2.0 * sigma * sigma))
    return g / g.sum()


def _filter(x, w):
    """'same' Gaussian filter with zero padding over the last two axes of a
    torch tensor [..., H, W], separable: rows, then columns."""
    r = (len(w) - 1) // 2
    wt = torch.as_tensor(w, dtype=torch.float64)
    lead = x.shape[:-2]
    H, W = x.shape[-2:]
    y = x.reshape(-1, 1, H, W)
    y = torch.nn.functional.conv2d(y, wt.view(1, 1, 1, -1), padding=(0, r))
    y = torch.nn.functional.conv2d(y, wt.view(1, 1, -1, 1), padding=(r, 0))
    return y.reshape(*lead, H, W)


def ssim_map(x, y, size=SSIM_WIN, sigma=SSIM_SIGMA, C1=SSIM_C1, C2=SSIM_C2):
    """Per-pixel SSIM of torch tensors x, y [..., H, W] (FP64)."""
    w = _window(size, sigma)
    mx, my = _filter(x, w), _filter(y, w)
    sxx = _filter(x * x, w) - mx * mx
    syy = _filter(y * y, w) - my * my
    sxy = _filter(x * y, w) - mx * my
    return ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))


def l1_ssim_loss(zhat, z, lambda_1=LAMBDA_1):
    """Eq. (5) per set for real spectra [S][F][H][W]: returns L_b [S],
    SSIM_b [S], L1_b [S] and dL/dzhat for L = mean_b L_b."""
    x = torch.tensor(np.asarray(zhat, np.float64), requires_grad=True)
    y = torch.tensor(np.asarray(z, np.float64))
    S = x.shape[0]
    l1 = (x - y).abs().reshape(S, -1).mean(1)
    ss = ssim_map(x, y).reshape(S, -1).mean(1)
    L = (1.0 - lambda_1) * l1 + lambda_1 * (1.0 - ss)
    L.mean().backward()
    return (L.detach().numpy(), ss.detach().numpy(), l1.detach().numpy(), x.grad.numpy())
