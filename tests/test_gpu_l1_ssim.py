"""The magnitude-spectrum loss, Eq. (5) (gs_loss_l1_ssim), against the FP64
loss oracle (L1 + SSIM with the 11 x 11, sigma 1.5 Gaussian window and zero
padding; gradient by FP64 autograd of the definition).

Cases: the training grid (ragged against the kernel's 32 x 16 tiles), the
0.5-degree grid, an image smaller than one tile, lambda_1 in {0, 0.2, 1},
identical spectra (loss 0, SSIM 1, zero gradient).

Tolerances: FP32 window sums against FP64: per-set loss, SSIM and L1 within
2e-6 absolute (they are means of O(1) values over 1e4..1e7 terms);
gradient as the other backward tests (2e-4 of the tensor's max, 2e-3
relative on entries above 1% of it).
"""
import numpy as np
import pytest
import torch

import paper_2511_22793_amd as gs
from oracle import loss_ref
from test_gpu_backward import compare

pytestmark = pytest.mark.gpu


def _magnitudes(shape, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    z = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    return (np.abs(z) * scale / 3.0).astype(np.float32)


@pytest.mark.parametrize("S,F,H,W,lam", [(2, 3, 90, 360, 0.2), (1, 2, 5, 7, 0.2), (2, 1, 180, 720, 0.2),
                                         (3, 2, 45, 90, 0.0), (2, 2, 33, 65, 1.0)])
def test_l1_ssim_matches_oracle(S, F, H, W, lam):
    zh = _magnitudes((S, F, H, W), 10 + H)
    # a target close to the prediction, as late in training
    z = np.clip(zh + _magnitudes((S, F, H, W), 20 + W, 0.3) - 0.1, 0, None).astype(np.float32)
    L, ss, l1, d = gs.loss_l1_ssim(torch.from_numpy(zh).cuda(), torch.from_numpy(z).cuda(), lam)
    torch.cuda.synchronize()
    Lr, ssr, l1r, dr = loss_ref.l1_ssim_loss(zh.astype(np.float64), z.astype(np.float64), lam)
    assert np.allclose(L.cpu().numpy(), Lr, rtol=0, atol=2e-6), (L, Lr)
    assert np.allclose(ss.cpu().numpy(), ssr, rtol=0, atol=2e-6), (ss, ssr)
    assert np.allclose(l1.cpu().numpy(), l1r, rtol=0, atol=2e-6), (l1, l1r)
    compare(d.cpu().numpy(), dr, "dL/dzhat")


def test_identical_spectra():
    zh = _magnitudes((2, 4, 90, 360), 3)
    t = torch.from_numpy(zh).cuda()
    L, ss, l1, d = gs.loss_l1_ssim(t, t.clone(), 0.2)
    torch.cuda.synchronize()
    assert np.allclose(ss.cpu().numpy(), 1.0, atol=2e-6)
    assert np.allclose(L.cpu().numpy(), 0.0, atol=1e-6)
    assert np.all(l1.cpu().numpy() == 0.0)
    # the L1 part is 0 at equality and the SSIM gradient vanishes at its maximum
    # (a gradient entry of a differing pair is of order lambda_1 / (F H W S))
    assert float(d.abs().max()) <= 1e-3 * 0.2 / (4 * 90 * 360 * 2)


def test_loss_only_call_writes_no_gradient():
    zh = _magnitudes((1, 1, 20, 40), 4)
    z = _magnitudes((1, 1, 20, 40), 5)
    L, ss, l1, d = gs.loss_l1_ssim(torch.from_numpy(zh).cuda(), torch.from_numpy(z).cuda(), 0.2, grad=False)
    torch.cuda.synchronize()
    Lr, _, _, _ = loss_ref.l1_ssim_loss(zh.astype(np.float64), z.astype(np.float64), 0.2)
    assert d is None and np.allclose(L.cpu().numpy(), Lr, atol=2e-6)
