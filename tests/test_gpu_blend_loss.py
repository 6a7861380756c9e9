"""The compositing kernel with the training loss fused into its output stage
(gs_render_blend_loss) against gs_render_blend + gs_loss_spectrum_stats: the
spectrum and the elementwise gradient part bit-identical to the per-group
compositing kernel's (GS_OPT_BLEND_PER_GROUP: the fused stage lives in that
kernel, so the arithmetic is the same), the loss, spatial means and
channel-mean term equal up to FP32 summation order (the fused sums add
per-wave partials, the loss pass per-workgroup strided partials)."""
import numpy as np
import pytest
import torch

import paper_2511_22793_amd as gs
import synth
from gpu_util import to_dev

pytestmark = pytest.mark.gpu


# (sets, channels, complex, tile (h, w), Gaussians, seed): matrix-core
# output stages with 64 and 16 channels per group, the VALU stage with 1, 2
# and 3 channels per group, edge tiles of every shape
CASES = [
    (4, 64, True, (16, 16), 2000, 1),
    (3, 8, True, (8, 32), 500, 2),
    (2, 3, False, (16, 16), 400, 3),
    (1, 1, False, (32, 8), 300, 4),
    (5, 1, True, (8, 8), 300, 5),
]


@pytest.mark.parametrize("S,F,cplx,tile,n,seed", CASES)
def test_fused_loss_matches_blend_then_loss_pass(S, F, cplx, tile, n, seed):
    sc = synth.scene(n, seed=seed, lo=[-3, -3, 0.1], hi=[3, 3, 2.5], log_scale_mean=-1.3)
    dev = to_dev(sc)
    attrs = torch.from_numpy(np.stack([synth.channel_attrs(n, F, cplx, seed=10 * seed + s)
                                       for s in range(S)])).cuda()
    rx = torch.tensor([[0.1, -0.2, 0.3]]).cuda()
    grid = gs.Grid(90, 360, tile[0], tile[1])
    ws = gs.prepare(dev, rx, grid=grid, params=gs.Params(blend_per_group=True))
    ref = gs.blend(ws, attrs, n_sets=S, is_complex=cplx)
    target = torch.from_numpy(np.random.default_rng(seed + 99).normal(size=tuple(ref.shape)).astype(np.float32)).cuda()
    lam = 0.7
    part_ref = torch.empty_like(ref)
    loss_ref, hh_ref, mg_ref, scale_ref = gs.loss_stats(ref, target, cplx, lam, partial=part_ref)
    part = torch.full_like(ref, float("nan"))
    spec, loss, hh, mg, scale = gs.blend_loss(ws, attrs, target, lam, n_sets=S, is_complex=cplx, partial=part)
    torch.cuda.synchronize()
    assert scale == scale_ref
    assert torch.equal(spec, ref)
    assert torch.equal(part, part_ref)
    assert torch.allclose(loss, loss_ref, rtol=2e-5, atol=0)
    assert torch.allclose(hh, hh_ref, rtol=2e-5, atol=1e-7 * float(hh_ref.abs().max()))
    assert torch.allclose(mg, mg_ref, rtol=2e-5, atol=1e-7 * float(mg_ref.abs().max()))


def test_fused_loss_without_partial_and_repeated_calls():
    # d_partial NULL; the accumulators are cleared on every call
    n, S, F = 600, 2, 16
    sc = synth.scene(n, seed=7)
    dev = to_dev(sc)
    attrs = torch.from_numpy(np.stack([synth.channel_attrs(n, F, True, seed=70 + s) for s in range(S)])).cuda()
    rx = torch.zeros(1, 3).cuda()
    ws = gs.prepare(dev, rx, params=gs.Params(blend_per_group=True))
    ref = gs.blend(ws, attrs, n_sets=S, is_complex=True)
    target = torch.from_numpy(np.random.default_rng(8).normal(size=tuple(ref.shape)).astype(np.float32)).cuda()
    loss_ref, hh_ref, mg_ref, _ = gs.loss_stats(ref, target, True, 1.0)
    for _ in range(3):
        spec, loss, hh, mg, _ = gs.blend_loss(ws, attrs, target, 1.0, n_sets=S, is_complex=True)
        torch.cuda.synchronize()
        assert torch.equal(spec, ref)
        assert torch.allclose(loss, loss_ref, rtol=2e-5, atol=0)
        assert torch.allclose(mg, mg_ref, rtol=2e-5, atol=1e-7 * float(mg_ref.abs().max()))
