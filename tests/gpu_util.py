"""Helpers shared by the GPU tests: run the HIP path from numpy inputs and
compare with the oracle under the parity metric and guard band.

Parity metric (per pixel p, channel f): e = |x - ref| / max(A, 1e-30), A the
oracle's absolute-sum magnitude sum_i T_i alpha_i |u_i,f|.  Gate: e <= 1e-5
on every pixel whose decisions all clear their thresholds by more than 1e-5
relative (the oracle marks the others ambiguous).  Ambiguous pixels: at most
1e-3 of the image, each within the coarse flip bound e <= 0.05.  Pixels with
no contributor must be exactly 0 on both sides.
"""
import numpy as np
import torch

import oracle
import paper_2511_22793_amd as gs

GATE = 1e-5
AMBIG_FRACTION = 1e-3
FLIP_BOUND = 0.05


def to_dev(scene):
    return {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in scene.items()}


def gpu_forward(scene, attr, rx, tx=None, H=90, W=360, tile=(16, 16), prm=None, is_complex=False, per_query=False):
    """rx: [B,3]. attr: [n,F(,2)] shared, or [B,n,F(,2)] if per_query."""
    prm = prm or gs.Params()
    rx_t = torch.from_numpy(np.asarray(rx, np.float32).reshape(-1, 3).copy()).cuda()
    tx_t = None if tx is None else torch.from_numpy(np.asarray(tx, np.float32).reshape(-1, 3).copy()).cuda()
    out, ws = gs.forward(to_dev(scene), torch.from_numpy(np.ascontiguousarray(attr, np.float32)).cuda(), rx_t, tx_t,
                         grid=gs.Grid(H, W, tile[0], tile[1]), params=prm, is_complex=is_complex)
    torch.cuda.synchronize()
    o = out.cpu().double().numpy()
    if is_complex:
        o = o[..., 0] + 1j * o[..., 1]
    return o, ws


def oracle_params(p: gs.Params):
    return oracle.params(alpha_min=p.alpha_min, alpha_max=p.alpha_max, T_min=p.T_min, dilation=p.dilation,
                         r_near=p.r_near, atten_power=p.atten_power, atten_ref=p.atten_ref, margin=p.margin)


def check_parity(got, ref, label=""):
    """got: [F,H,W]; ref: oracle result dict. Returns the max gated error."""
    err = oracle.parity_error(got, ref["out"], ref["absacc"])
    amb = ref["ambig"][None].repeat(err.shape[0], 0)
    empty = ref["absacc"] == 0
    assert np.all(got[empty] == 0), "%s: pixels with no contributor are not exactly zero" % label
    gated = err[~amb]
    worst = float(gated.max()) if gated.size else 0.0
    assert worst <= GATE, "%s: max parity error %.3g > %g (pixel %s)" % (
        label, worst, GATE, np.unravel_index(np.argmax(np.where(amb, 0, err)), err.shape))
    frac = float(ref["ambig"].mean())
    assert frac <= AMBIG_FRACTION, "%s: ambiguous fraction %.3g" % (label, frac)
    if amb.any():
        assert float(err[amb].max()) <= FLIP_BOUND, "%s: ambiguous pixel beyond the flip bound" % label
    return worst


def pixel_state(ws, q, H, W):
    HW = H * W
    T = ws.view("T_final", q, HW, torch.float32).cpu().double().numpy().reshape(H, W)
    nc = ws.view("n_contrib", q, HW, torch.int32).cpu().numpy().reshape(H, W)
    nl = ws.view("n_last", q, HW, torch.int32).cpu().numpy().reshape(H, W)
    return T, nc, nl
