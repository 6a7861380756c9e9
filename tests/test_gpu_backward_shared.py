"""Backward over attribute sets that share one geometry.

Where the sets share the prepared geometry and F*c is a multiple of 16 the
library takes the factorised backward (the geometry walked once for every
set and channel, the set sums formed on the matrix cores).  Checked against
the autograd oracle per set (attribute gradients per set, scene gradients
summed over sets) across tile shapes, set counts that leave some of the
kernel's column slices empty, real and complex channels and tiles with more
than one batch of entries; and against the per-set, per-channel-group
kernel (GS_OPT_BWD_PER_GROUP) at the training shape.

Tolerance as in the other backward tests: FP32 with float atomics against
FP64, max|g - r| <= 2e-4 max|r| + 1e-7 and 2e-3 relative on entries above
1e-2 max|r|.
"""
import numpy as np
import pytest
import torch

import paper_2511_22793_amd as gs
import synth
from gpu_util import oracle_params, to_dev
from test_gpu_backward import NAMES, close_scene, compare, torch_grads

pytestmark = pytest.mark.gpu


def shared_grads(sc, attrs, rx, G, S, cplx, tile, prm):
    dev = to_dev(sc)
    rx_t = torch.tensor([rx], dtype=torch.float32).cuda()
    ws = gs.prepare(dev, rx_t, grid=gs.Grid(90, 360, tile[0], tile[1]), params=prm)
    a = torch.from_numpy(np.ascontiguousarray(attrs, np.float32)).cuda()
    out = gs.blend(ws, a, n_sets=S, is_complex=cplx)
    d = torch.from_numpy(np.ascontiguousarray(G, np.float32)).cuda()
    g = gs.backward(ws, dev, a, rx_t, out, d, is_complex=cplx, n_sets=S)
    torch.cuda.synchronize()
    return {k: v.cpu().double().numpy() for k, v in g.items()}


# (sets, channels, complex, tile (h, w), Gaussians, seed)
CASES = [
    (3, 8, True, (16, 16), 120, 1),   # 3 x 16 columns: five of the eight column slices empty
    (1, 16, False, (8, 8), 60, 2),    # one set, real, one 64-pixel group per tile
    (2, 24, True, (8, 32), 90, 3),    # 48 columns per set, wide tiles
    (4, 16, True, (32, 8), 80, 4),    # narrow tiles
    (2, 32, False, (16, 8), 70, 5),   # two pixel groups per tile
    (4, 32, True, (16, 16), 100, 6),  # 16 column blocks: two per wave; the bottom tiles' 32-pixel groups
]


@pytest.mark.parametrize("S,F,cplx,tile,n,seed", CASES)
def test_shared_backward_matches_oracle(S, F, cplx, tile, n, seed):
    sc = close_scene(n, seed)
    attrs = np.stack([synth.channel_attrs(n, F, cplx, seed=100 * seed + s) for s in range(S)])
    rng = np.random.default_rng(seed + 7)
    G = rng.normal(size=(S, F, 90, 360, 2) if cplx else (S, F, 90, 360))
    rx = [0.1, -0.2, 0.05]
    prm = gs.Params()
    got = shared_grads(sc, attrs, rx, G, S, cplx, tile, prm)
    want = None
    for s in range(S):
        r = torch_grads(sc, attrs[s], rx, G[s], oracle_params(prm), cplx=cplx)
        compare(got["d_attr"][s], r["attr"], "attr set %d" % s)
        want = r if want is None else {k: want[k] + r[k] for k in want}
    for k in NAMES:
        compare(got["d_" + k], want[k], k)


def test_more_than_one_batch_of_entries_per_tile():
    # a dense cluster in front of the receiver: every tile of the cluster
    # walks well past 64 entries before its pixels saturate
    n, S, F = 300, 2, 8
    sc = synth.scene(n, seed=21, lo=[-3, -3, 0.1], hi=[3, 3, 2.0], log_scale_mean=-0.8)
    sc["opacity_logit"] = np.full(n, -3.0, np.float32)  # faint: long walks
    attrs = np.stack([synth.channel_attrs(n, F, True, seed=22 + s) for s in range(S)])
    G = np.random.default_rng(23).normal(size=(S, F, 90, 360, 2))
    rx = [0.0, 0.0, 0.0]
    prm = gs.Params()
    dev = to_dev(sc)
    rx_t = torch.tensor([rx], dtype=torch.float32).cuda()
    ws = gs.prepare(dev, rx_t, params=prm)
    a = torch.from_numpy(attrs).cuda()
    gs.blend(ws, a, n_sets=S, is_complex=True)
    n_last = ws.view("n_last", 0, 90 * 360).cpu().numpy()
    got = shared_grads(sc, attrs, rx, G, S, True, (16, 16), prm)
    want = None
    for s in range(S):
        r = torch_grads(sc, attrs[s], rx, G[s], oracle_params(prm), cplx=True)
        compare(got["d_attr"][s], r["attr"], "attr set %d" % s)
        want = r if want is None else {k: want[k] + r[k] for k in want}
    for k in NAMES:
        compare(got["d_" + k], want[k], k)
    assert int(n_last.max()) > 64  # list positions walked by the deepest pixel


def test_shared_and_per_group_kernels_agree_at_training_shape():
    # 16 transmitter sets x 64 complex channels (2048 columns), 16x16 tiles
    n, S, F = 3000, 16, 64
    sc = synth.scene(n, seed=31)
    attrs = np.stack([synth.channel_attrs(n, F, True, seed=32 + s) for s in range(S)])
    G = np.random.default_rng(33).normal(size=(S, F, 90, 360, 2))
    rx = [0.3, -0.1, 0.2]
    a = shared_grads(sc, attrs, rx, G, S, True, (16, 16), gs.Params())
    b = shared_grads(sc, attrs, rx, G, S, True, (16, 16), gs.Params(bwd_per_group=True))
    for k in NAMES + ("attr",):
        compare(a["d_" + k], b["d_" + k], k)
