"""Compositing of attribute sets over one shared geometry (k_blend_sg: the
walk once per pixel, out = W^T V on the matrix cores) against the per-set,
per-channel-group kernel (GS_OPT_BLEND_PER_GROUP) and the oracle.

The walk takes the same decisions in the same order, so the per-pixel
state (final transmittance, stop position, contribution count) must be
bit-identical; the spectra differ only in FP32 summation order (the products
run over buffered entries instead of runs of 16), checked at 2e-6 of the
spectrum's magnitude; the oracle gate of the other forward tests applies
through test_gpu_forward.py (single-query forwards with F*c a multiple of 16
take this kernel)."""
import numpy as np
import pytest
import torch

import paper_2511_22793_amd as gs
import synth
from gpu_util import to_dev

pytestmark = pytest.mark.gpu


def render_both(sc, attrs, rx, S, cplx, tile, H=90, W=360):
    dev = to_dev(sc)
    rx_t = torch.tensor([rx], dtype=torch.float32).cuda()
    a = torch.from_numpy(np.ascontiguousarray(attrs, np.float32)).cuda()
    res = []
    for per_group in (False, True):
        prm = gs.Params(blend_per_group=per_group)
        ws = gs.prepare(dev, rx_t, grid=gs.Grid(H, W, tile[0], tile[1]), params=prm)
        out = gs.blend(ws, a, n_sets=S, is_complex=cplx)
        torch.cuda.synchronize()
        state = [ws.view(k, 0, H * W, dtype=torch.float32 if k == "T_final" else torch.int32).clone()
                 for k in ("T_final", "n_last", "n_contrib")]
        res.append((out.clone(), state))
    return res


# (sets, channels, complex, tile (h, w), Gaussians, seed)
CASES = [
    (16, 64, True, (16, 16), 3000, 1),   # the training shape
    (3, 8, True, (8, 32), 400, 2),       # 48 columns: waves without columns
    (1, 16, False, (8, 8), 300, 3),
    (2, 48, False, (32, 8), 500, 4),
    (5, 8, True, (16, 8), 400, 5),
]


@pytest.mark.parametrize("S,F,cplx,tile,n,seed", CASES)
def test_shared_blend_matches_per_group_blend(S, F, cplx, tile, n, seed):
    sc = synth.scene(n, seed=seed, lo=[-3, -3, 0.1], hi=[3, 3, 2.5], log_scale_mean=-1.3)
    attrs = np.stack([synth.channel_attrs(n, F, cplx, seed=10 * seed + s) for s in range(S)])
    (a, sa), (b, sb) = render_both(sc, attrs, [0.1, -0.2, 0.3], S, cplx, tile)
    for x, y in zip(sa, sb):
        assert torch.equal(x, y)
    scale = float(b.abs().max())
    assert float((a - b).abs().max()) <= 2e-6 * scale + 1e-30


def test_shared_blend_long_walks_flush_the_weight_buffer():
    # faint Gaussians around the receiver: pixels walk far past the 128
    # buffered entries, so the products are added to the stored spectrum
    n, S, F = 1500, 2, 8
    sc = synth.scene(n, seed=11, lo=[-3, -3, 0.1], hi=[3, 3, 2.0], log_scale_mean=-0.8)
    sc["opacity_logit"] = np.full(n, -4.0, np.float32)
    attrs = np.stack([synth.channel_attrs(n, F, True, seed=12 + s) for s in range(S)])
    (a, sa), (b, sb) = render_both(sc, attrs, [0.0, 0.0, 0.0], S, True, (16, 16))
    for x, y in zip(sa, sb):
        assert torch.equal(x, y)
    assert int(sa[1].max()) > 2 * 128
    scale = float(b.abs().max())
    assert float((a - b).abs().max()) <= 2e-6 * scale + 1e-30


def test_shared_blend_empty_and_outside_pixels_are_zero():
    # a handful of Gaussians: most tiles have no entries, edge groups are
    # partly outside the image; the spectrum there must be exactly zero
    n, S, F = 5, 3, 8
    sc = synth.scene(n, seed=13, lo=[1.0, 1.0, 0.5], hi=[1.5, 1.5, 1.0], log_scale_mean=-2.5)
    attrs = np.stack([synth.channel_attrs(n, F, True, seed=14 + s) for s in range(S)])
    (a, sa), (b, sb) = render_both(sc, attrs, [0.0, 0.0, 0.0], S, True, (16, 16))
    zero = sb[2].reshape(90, 360) == 0
    assert bool(zero.any())
    assert float(a[:, :, zero].abs().max()) == 0.0
    assert torch.equal(sa[2], sb[2])
