"""Pins of the loss oracle (Eq. (2), Eq. (4), Eq. (5)) to closed forms, brute
force and finite differences, not to the oracle itself.

* Eq. (2): one nonzero pixel v gives the mean v / (H W).
* The L2 + channel loss: spectra that are constant per channel give
  L = (1/F) sum_f |a_f - b_f|^2 + lambda sum_f |a_f - b_f|^2 and the gradient
  2 (a - b) / (F H W S) + 2 lambda (a - b) / (H W S) by hand; a difference with
  zero spatial mean per channel leaves only the pixel term; finite
  differences.
* SSIM: SSIM(x, x) = 1; two constant images give (2ab + C1) / (a^2 + b^2 + C1)
  wherever the window lies inside the image (the variances vanish); a
  brute-force evaluation of the textbook definition, window pixel by window
  pixel with the 2-D window written out, on a small image; symmetry.
* Eq. (5): lambda_1 = 0 is the mean absolute error; zhat = z gives zero loss;
  finite differences of the loss.
"""
import numpy as np
import pytest

from oracle import loss_ref as lr


def test_spatial_mean_of_one_pixel():
    z = np.zeros((1, 2, 5, 7, 2))
    z[0, 1, 3, 4] = [2.0, -7.0]
    h = lr.spatial_mean(z, True)
    assert np.allclose(h[0, 1], [2.0 / 35, -7.0 / 35], rtol=0, atol=1e-17)
    assert np.all(h[0, 0] == 0)


@pytest.mark.parametrize("cplx", [True, False])
def test_constant_spectra_closed_form(cplx):
    S, F, H, W, lam = 2, 3, 4, 6, 0.7
    rng = np.random.default_rng(1)
    shp = (S, F, 2) if cplx else (S, F)
    a, b = rng.normal(size=shp), rng.normal(size=shp)
    expand = (lambda v: np.broadcast_to(v[:, :, None, None, :], (S, F, H, W, 2))) if cplx else \
        (lambda v: np.broadcast_to(v[:, :, None, None], (S, F, H, W)))
    L, hh, g = lr.l2_channel_loss(expand(a), expand(b), cplx, lam)
    d2 = ((a - b) ** 2).reshape(S, F, -1).sum(-1)             # |a_f - b_f|^2
    assert np.allclose(L, d2.mean(1) + lam * d2.sum(1), rtol=1e-14, atol=0)
    assert np.allclose(hh, a, rtol=1e-14, atol=1e-15)
    want = 2 * (a - b) / (F * H * W * S) + 2 * lam * (a - b) / (H * W * S)
    assert np.allclose(g, expand(want), rtol=1e-13, atol=0)


def test_zero_mean_difference_leaves_the_pixel_term():
    S, F, H, W = 2, 2, 4, 4
    rng = np.random.default_rng(2)
    zh = rng.normal(size=(S, F, H, W, 2))
    d = rng.normal(size=(S, F, H, W, 2))
    d -= d.mean(axis=(2, 3), keepdims=True)
    L, _, _ = lr.l2_channel_loss(zh, zh + d, True, 5.0)
    assert np.allclose(L, (d ** 2).reshape(S, -1).sum(1) / (F * H * W), rtol=1e-12, atol=1e-15)


def test_l2_channel_gradient_finite_differences():
    S, F, H, W = 2, 2, 3, 5
    rng = np.random.default_rng(3)
    zh = rng.normal(size=(S, F, H, W, 2))
    z = rng.normal(size=(S, F, H, W, 2))
    _, _, g = lr.l2_channel_loss(zh, z, True, 0.9)
    eps = 1e-6
    for idx in [(0, 0, 0, 0, 0), (1, 1, 2, 4, 1), (0, 1, 1, 3, 0), (1, 0, 2, 0, 1)]:
        a, b = zh.copy(), zh.copy()
        a[idx] += eps
        b[idx] -= eps
        num = (lr.l2_channel_loss(a, z, True, 0.9)[0].mean() - lr.l2_channel_loss(b, z, True, 0.9)[0].mean()) / (2 * eps)
        assert abs(g[idx] - num) <= 1e-8 * max(1.0, abs(num))


def _ssim_brute(x, y, C1=0.01 ** 2, C2=0.03 ** 2):
    """Textbook SSIM per pixel: an 11 x 11 window exp(-(i^2 + j^2) / (2 1.5^2))
    normalised over all its 121 taps, pixels outside the image read as 0."""
    H, W = x.shape
    w = np.array([[np.exp(-(i * i + j * j) / (2 * 1.5 ** 2)) for j in range(-5, 6)] for i in range(-5, 6)])
    w /= w.sum()
    out = np.zeros((H, W))
    for r in range(H):
        for c in range(W):
            mx = my = exx = eyy = exy = 0.0
            for i in range(-5, 6):
                for j in range(-5, 6):
                    rr, cc = r + i, c + j
                    if 0 <= rr < H and 0 <= cc < W:
                        a, b, k = x[rr, cc], y[rr, cc], w[i + 5, j + 5]
                        mx += k * a
                        my += k * b
                        exx += k * a * a
                        eyy += k * b * b
                        exy += k * a * b
            vx, vy, cxy = exx - mx * mx, eyy - my * my, exy - mx * my
            out[r, c] = (2 * mx * my + C1) * (2 * cxy + C2) / ((mx * mx + my * my + C1) * (vx + vy + C2))
    return out


def test_ssim_matches_brute_force_definition():
    rng = np.random.default_rng(4)
    x = rng.random((13, 17))
    y = 0.6 * x + 0.4 * rng.random((13, 17))
    import torch
    got = lr.ssim_map(torch.tensor(x), torch.tensor(y)).numpy()
    assert np.allclose(got, _ssim_brute(x, y), rtol=1e-12, atol=1e-14)
    sym = lr.ssim_map(torch.tensor(y), torch.tensor(x)).numpy()
    assert np.allclose(got, sym, rtol=1e-13, atol=0)
    assert got.max() <= 1.0


def test_ssim_of_identical_and_of_constant_images():
    import torch
    rng = np.random.default_rng(5)
    x = rng.random((2, 20, 24))
    s = lr.ssim_map(torch.tensor(x), torch.tensor(x)).numpy()
    assert np.allclose(s, 1.0, rtol=0, atol=1e-12)
    a, b = 0.3, 0.8
    s = lr.ssim_map(torch.full((20, 24), a, dtype=torch.float64), torch.full((20, 24), b, dtype=torch.float64)).numpy()
    want = (2 * a * b + lr.SSIM_C1) / (a * a + b * b + lr.SSIM_C1)
    assert np.allclose(s[5:-5, 5:-5], want, rtol=1e-12, atol=0)


def test_l1_ssim_special_cases():
    rng = np.random.default_rng(6)
    zh = rng.random((2, 3, 14, 16))
    z = rng.random((2, 3, 14, 16))
    L, ss, l1, g = lr.l1_ssim_loss(zh, z, lambda_1=0.0)
    assert np.allclose(L, np.abs(zh - z).reshape(2, -1).mean(1), rtol=1e-14, atol=0)
    assert np.allclose(g, np.sign(zh - z) / (3 * 14 * 16 * 2), rtol=1e-14, atol=0)
    L, ss, l1, g = lr.l1_ssim_loss(z, z)
    assert np.allclose(L, 0.0, atol=1e-13) and np.allclose(ss, 1.0, atol=1e-13)
    L, ss, _, _ = lr.l1_ssim_loss(zh, z, lambda_1=1.0)
    assert np.allclose(L, 1.0 - ss, rtol=1e-14, atol=0)


def test_l1_ssim_gradient_finite_differences():
    rng = np.random.default_rng(7)
    zh = rng.random((2, 2, 12, 13))
    z = np.clip(zh + rng.choice([-1, 1], size=zh.shape) * rng.uniform(0.05, 0.3, size=zh.shape), 0, None)
    _, _, _, g = lr.l1_ssim_loss(zh, z)
    eps = 1e-6
    for idx in [(0, 0, 0, 0), (1, 1, 11, 12), (0, 1, 6, 6), (1, 0, 3, 9), (0, 0, 11, 0)]:
        a, b = zh.copy(), zh.copy()
        a[idx] += eps
        b[idx] -= eps
        num = (lr.l1_ssim_loss(a, z)[0].mean() - lr.l1_ssim_loss(b, z)[0].mean()) / (2 * eps)
        assert abs(g[idx] - num) <= 1e-7 * max(1e-3, abs(num)), idx
