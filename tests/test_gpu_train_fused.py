"""The fused training pass (gs_render_train): compositing, the training loss
and the backward over S complex attribute sets sharing one receiver, in two
kernels, without the spectra or their gradient in memory.

* Against the unfused path on the same inputs (gs_render_blend, then
  gs_loss_spectrum_stats and gs_render_backward_l2): the spectrum it stores
  on request is bit-identical to gs_render_blend's; loss, h_hat and every
  gradient agree to FP32 summation order (h_hat is formed from the live
  pass's per-Gaussian weight sums instead of the image, the rest through
  float atomics in another order).  Cases: tile shapes, set and channel
  counts, groups whose walks fall in each band of the fused kernels'
  variants (up to 64, 128 and 256 entries) and beyond (those take the
  unfused kernels inside the call), a mix, the 100k-Gaussian training
  shape and the 300k-Gaussian 180x720 one (attribute gradients sampled).
* Against the oracles: the FP64 dense autograd renderer with the loss
  oracle (Eq. (2) means, Eq. (4) channel term, pixel term) for loss, h_hat
  and every gradient.

Tolerances: gradients as in test_gpu_backward (2e-4 of the tensor's max,
2e-3 relative on entries above 1% of it); loss and h_hat 1e-5 relative to
the largest entry (1e-4 for the loss against FP64: it sums ~1e7 FP32
squares).
"""
import numpy as np
import pytest
import torch

import paper_2511_22793_amd as gs
import synth
from gpu_util import oracle_params, to_dev
from oracle import loss_ref, torch_ref
from test_gpu_backward import NAMES, close_scene, compare

pytestmark = pytest.mark.gpu


def _close_rel(got, ref, label, rtol):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = max(float(np.abs(ref).max()), 1e-30)
    err = float(np.abs(got - ref).max())
    assert err <= rtol * scale, "%s: max err %.3g vs scale %.3g" % (label, err, scale)


def _targets(S, F, H, W, seed, scale=0.02):
    rng = np.random.default_rng(seed)
    return (rng.normal(size=(S, F, H, W, 2)) * scale).astype(np.float32)


def _run_both(sc, attrs, rx, tgt, grid, prm, lam=1.0):
    """(fused results, unfused results) on one prepared workspace."""
    S, n, F = attrs.shape[:3]
    dev = to_dev(sc)
    rx_t = torch.tensor(np.asarray(rx, np.float32).reshape(1, 3)).cuda()
    ws = gs.prepare(dev, rx_t, grid=grid, params=prm)
    lst, cnt = gs.live(ws)
    a = torch.from_numpy(np.ascontiguousarray(attrs, np.float32)).cuda()
    z = torch.from_numpy(tgt).cuda()
    h = gs.spatial_mean(z, True)
    loss_f, hh_f, g_f, spec_f = gs.train_pass(ws, dev, a, rx_t, lst, cnt, z, h, lam, write_spectrum=True)
    torch.cuda.synchronize()
    fused = {k: v.cpu().double().numpy() for k, v in g_f.items()}
    fused["loss"] = loss_f.cpu().double().numpy()
    fused["h_hat"] = hh_f.cpu().double().numpy()
    fused["spec"] = spec_f.cpu().numpy()
    # unfused: compositing, loss pass, backward
    spec = gs.blend(ws, a, n_sets=S, is_complex=True)
    part = torch.empty_like(spec)
    loss, hhat, mgrad, scale = gs.loss_stats(spec, z, True, lam, partial=part)
    g = gs.backward_l2(ws, dev, a, rx_t, spec, None, mgrad, scale, partial=part, is_complex=True, n_sets=S)
    torch.cuda.synchronize()
    ref = {k: v.cpu().double().numpy() for k, v in g.items()}
    ref["loss"] = loss.cpu().double().numpy()
    ref["h_hat"] = hhat.cpu().double().numpy()
    ref["spec"] = spec.cpu().numpy()
    return fused, ref, ws


def _check_against_unfused(fused, ref, S):
    assert np.array_equal(fused["spec"], ref["spec"]), "stored spectrum differs from gs_render_blend's"
    _close_rel(fused["loss"], ref["loss"], "loss", 1e-5)
    _close_rel(fused["h_hat"], ref["h_hat"], "h_hat", 1e-5)
    for s in range(S):
        compare(fused["d_attr"][s], ref["d_attr"][s], "d_attr set %d" % s)
    for k in NAMES:
        compare(fused["d_" + k], ref["d_" + k], k)


# (sets, channels, tile (h, w), Gaussians, seed)
CASES = [
    (4, 8, (16, 16), 120, 1),    # 64 columns: one column range, one round
    (3, 16, (8, 32), 90, 2),     # wide tiles, 96 columns
    (2, 24, (32, 8), 80, 3),     # narrow tiles
    (16, 8, (16, 8), 70, 4),     # 128-pixel tiles, 256 columns (two column ranges)
    (8, 64, (16, 16), 150, 5),   # 1024 columns (four column ranges); the bottom tiles' 32-pixel groups
    (5, 8, (8, 8), 60, 6),       # one group per tile, 80 columns (rounds with idle waves)
]


@pytest.mark.parametrize("S,F,tile,n,seed", CASES)
def test_fused_pass_matches_unfused_path(S, F, tile, n, seed):
    sc = close_scene(n, seed)
    attrs = np.stack([synth.channel_attrs(n, F, True, seed=100 * seed + s) for s in range(S)])
    tgt = _targets(S, F, 90, 360, seed + 50)
    fused, ref, _ = _run_both(sc, attrs, [0.1, -0.2, 0.05], tgt, gs.Grid(90, 360, tile[0], tile[1]), gs.Params())
    _check_against_unfused(fused, ref, S)


def _group_walks(ws, grid):
    """Walk length of every 64-pixel group (the in-image pixels of a tile,
    row-major, packed in 64s): the largest stop position among its pixels."""
    H, W, th, tw = grid.H, grid.W, grid.tile_h, grid.tile_w
    nl = ws.view("n_last", 0, H * W).cpu().numpy().reshape(H, W)
    out = []
    for ty in range(-(-H // th)):
        for tx in range(-(-W // tw)):
            blk = nl[ty * th:(ty + 1) * th, tx * tw:(tx + 1) * tw].reshape(-1)
            out += [blk[g:g + 64].max() for g in range(0, len(blk), 64)]
    return np.array(out)


def test_long_walks_take_the_wider_variants_and_the_unfused_kernels():
    # faint Gaussians in front of the receiver: groups walk 65-128 and
    # 129-256 entries (the wider fused variants); T_min = 0 makes every walk
    # run to the end of its list, past 256 entries (the unfused kernels
    # inside the call)
    S, F = 3, 8
    tgt = _targets(S, F, 90, 360, 23)
    bands = np.zeros(4, int)
    rng = np.random.default_rng(24)
    for n, logit, prm in ((300, -3.0, gs.Params()), (1500, None, gs.Params()), (1500, None, gs.Params(T_min=0.0))):
        sc = synth.scene(n, seed=21, lo=[-3, -3, 0.1], hi=[3, 3, 2.0], log_scale_mean=-0.8)
        # faint Gaussians; the larger scene mixes opacities so that its walks
        # spread over the bands
        sc["opacity_logit"] = (np.full(n, logit) if logit is not None else rng.uniform(-5.0, -2.0, n)).astype(
            np.float32)
        attrs = np.stack([synth.channel_attrs(n, F, True, seed=22 + s) for s in range(S)])
        fused, ref, ws = _run_both(sc, attrs, [0.0, 0.0, 0.0], tgt, gs.Grid(), prm)
        walks = _group_walks(ws, gs.Grid())
        bands += np.histogram(walks, bins=[0, 64.5, 128.5, 256.5, 1e9])[0]
        _check_against_unfused(fused, ref, S)
    assert np.all(bands > 0), "walk bands covered: %s" % bands


def test_mixed_short_and_long_groups():
    # a faint cluster on one side, an opaque sparse scene elsewhere
    n1, n2, S, F = 200, 400, 4, 16
    a = synth.scene(n1, seed=31, lo=[0.5, -1.0, 0.2], hi=[2.5, 1.0, 1.5], log_scale_mean=-1.0)
    a["opacity_logit"] = np.full(n1, -3.5, np.float32)
    b = synth.scene(n2, seed=32)
    sc = {k: np.ascontiguousarray(np.concatenate([a[k], b[k]], axis=-1)) for k in a}
    n = n1 + n2
    attrs = np.stack([synth.channel_attrs(n, F, True, seed=33 + s) for s in range(S)])
    tgt = _targets(S, F, 90, 360, 34)
    fused, ref, ws = _run_both(sc, attrs, [0.0, 0.0, 0.0], tgt, gs.Grid(), gs.Params())
    stops = ws.view("n_last", 0, 90 * 360).cpu().numpy()
    assert stops.max() > 64 and np.median(stops) <= 64
    _check_against_unfused(fused, ref, S)


def test_training_shape_100k_matches_unfused_path():
    n, S, F = 100_000, 16, 64
    sc = synth.scene(n, seed=0)
    attrs = np.stack([synth.channel_attrs(n, F, True, seed=40 + s) for s in range(S)])
    tgt = _targets(S, F, 90, 360, 41)
    fused, ref, _ = _run_both(sc, attrs, [0.0, 0.0, 0.0], tgt, gs.Grid(), gs.Params())
    _check_against_unfused(fused, ref, S)


def test_training_at_scale_shape_matches_unfused_path():
    # the at-scale training configuration: 300k Gaussians, 180x720, 32
    # complex subcarriers, 64 transmitter sets (the bench's train_300k
    # launch configuration); attributes and targets drawn on the device.
    # Loss, means and scene gradients in full; the attribute gradients of
    # sampled Gaussians in every seventh set.
    n, S, F, H, W = 300_000, 64, 32, 180, 720
    sc = synth.scene(n, seed=90)
    dev = to_dev(sc)
    gen = torch.Generator(device="cuda").manual_seed(91)
    a = torch.randn(S, n, F, 2, device="cuda", generator=gen) * 0.5
    z = torch.randn(S, F, H, W, 2, device="cuda", generator=gen) * 0.02
    grid = gs.Grid(H, W)
    rx_t = torch.zeros(1, 3, device="cuda")
    ws = gs.prepare(dev, rx_t, grid=grid)
    assert ws.flags()[0]["overflow"] == 0
    lst, cnt = gs.live(ws)
    h = gs.spatial_mean(z, True)
    loss_f, hh_f, g_f, _ = gs.train_pass(ws, dev, a, rx_t, lst, cnt, z, h, 1.0)
    torch.cuda.synchronize()
    spec = gs.blend(ws, a, n_sets=S, is_complex=True)
    part = torch.empty_like(spec)
    loss, hhat, mgrad, scale = gs.loss_stats(spec, z, True, 1.0, partial=part)
    g = gs.backward_l2(ws, dev, a, rx_t, spec, None, mgrad, scale, partial=part, is_complex=True, n_sets=S)
    torch.cuda.synchronize()
    _close_rel(loss_f.cpu().numpy(), loss.cpu().numpy(), "loss", 1e-5)
    _close_rel(hh_f.cpu().numpy(), hhat.cpu().numpy(), "h_hat", 1e-5)
    for k in NAMES:
        compare(g_f["d_" + k].cpu().numpy(), g["d_" + k].cpu().numpy(), k)
    # rows from the live list (the Gaussians with a nonzero attribute
    # gradient: about a hundred here, the scene being dense around the
    # receiver) and 2048 sampled from all Gaussians
    rng = np.random.default_rng(92)
    n_live = int(cnt[0])
    assert n_live > 0
    live_rows = lst[0, torch.from_numpy(rng.choice(n_live, min(n_live, 2048), replace=False)).cuda()].long()
    rows = torch.unique(torch.cat([live_rows, torch.from_numpy(rng.choice(n, 2048, replace=False)).cuda()]))
    sets = torch.arange(0, S, 7, device="cuda")
    got = g_f["d_attr"][sets][:, rows].cpu().numpy()
    want = g["d_attr"][sets][:, rows].cpu().numpy()
    for i, s_ in enumerate(sets.tolist()):
        compare(got[i], want[i], "d_attr set %d" % s_)


def test_fused_pass_matches_oracle_loss_and_gradients():
    n, S, F = 60, 4, 8
    sc = close_scene(n, 7)
    attrs = np.stack([synth.channel_attrs(n, F, True, seed=70 + s) for s in range(S)])
    tgt = _targets(S, F, 90, 360, 71, scale=0.05)
    rx = [0.1, -0.2, 0.05]
    lam = 0.7
    fused, _, _ = _run_both(sc, attrs, rx, tgt, gs.Grid(), gs.Params(), lam=lam)
    # FP64: the dense autograd renderer per set, the loss oracle on its spectra
    prm = oracle_params(gs.Params())
    t, at = torch_ref.to_tensors(sc, np.ascontiguousarray(attrs.transpose(1, 0, 2, 3).reshape(n, S * F, 2)),
                                 requires_grad=True)
    out = torch_ref.render(t["mean"], t["log_scale"], t["quat"], t["opacity_logit"], at, rx, 90, 360, prm=prm)["out"]
    zhat = out.reshape(S, F, 90, 360, 2)
    L, hh, dz = loss_ref.l2_channel_loss(zhat.detach().numpy(), tgt.astype(np.float64), True, lam)
    (zhat * torch.as_tensor(dz)).sum().backward()
    _close_rel(fused["loss"], L, "loss", 1e-4)
    _close_rel(fused["h_hat"], hh, "h_hat", 1e-5)
    d_attr = at.grad.numpy().reshape(n, S, F, 2).transpose(1, 0, 2, 3)
    for s in range(S):
        compare(fused["d_attr"][s], d_attr[s], "attr set %d" % s)
    for k in NAMES:
        compare(fused["d_" + k], t[k].grad.numpy(), k)


def test_deferred_geometry_on_a_second_stream_matches_the_one_call():
    # GS_TRAIN_DEFER_GEOMETRY + gs_render_train_geometry on another stream
    # (the training step's split): the same loss, attribute and scene
    # gradients as one gs_render_train call (float atomics: to rounding)
    n, S, F = 3000, 4, 16
    sc = synth.scene(n, seed=81)
    attrs = np.stack([synth.channel_attrs(n, F, True, seed=82 + s) for s in range(S)])
    tgt = _targets(S, F, 90, 360, 83)
    dev = to_dev(sc)
    rx_t = torch.zeros(1, 3, device="cuda")
    ws = gs.prepare(dev, rx_t)
    lst, cnt = gs.live(ws)
    a = torch.from_numpy(np.ascontiguousarray(attrs, np.float32)).cuda()
    z = torch.from_numpy(tgt).cuda()
    h = gs.spatial_mean(z, True)
    loss1, _, g1, _ = gs.train_pass(ws, dev, a, rx_t, lst, cnt, z, h, 1.0)
    torch.cuda.synchronize()
    one = {k: v.cpu().double().numpy() for k, v in g1.items()}
    one["loss"] = loss1.cpu().double().numpy()
    side = torch.cuda.Stream()
    main = torch.cuda.current_stream()
    loss2, _, g2, _ = gs.train_pass(ws, dev, a, rx_t, lst, cnt, z, h, 1.0, defer_geometry=True)
    side.wait_stream(main)
    with torch.cuda.stream(side):
        gs.train_geometry(ws, dev, rx_t, g2)
    main.wait_stream(side)
    torch.cuda.synchronize()
    two = {k: v.cpu().double().numpy() for k, v in g2.items()}
    _close_rel(loss2.cpu().double().numpy(), one["loss"], "loss", 1e-6)
    for s in range(S):
        compare(two["d_attr"][s], one["d_attr"][s], "d_attr set %d" % s)
    for k in NAMES:
        compare(two["d_" + k], one["d_" + k], k)
    # argument checks of the tail: wrong shapes are rejected on the host
    bad = dict(g2)
    bad["d_mean"] = torch.empty(3, n - 1, device="cuda")
    with pytest.raises(ValueError):
        gs.train_geometry(ws, dev, rx_t, bad)


def test_spatial_mean_matches_definition():
    rng = np.random.default_rng(3)
    for shape, cplx in (((3, 5, 17, 33, 2), True), ((2, 4, 90, 360), False)):
        z = rng.normal(size=shape).astype(np.float32)
        got = gs.spatial_mean(torch.from_numpy(z).cuda(), cplx).cpu().double().numpy()
        want = loss_ref.spatial_mean(z, cplx)
        _close_rel(got, want, "spatial mean %s" % (shape,), 1e-5)
