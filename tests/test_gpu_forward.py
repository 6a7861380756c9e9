"""GPU parity of the forward render against the CPU oracle, called through
the C ABI.  Stages: projection records, depth order and tile lists
(bit-exact), pixels (parity metric of tests/gpu_util.py)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2511_22793_amd as gs
import synth
from gpu_util import check_parity, check_parity_at, gpu_forward, oracle_params, pixel_state

pytestmark = pytest.mark.gpu


def _proj_from_ws(ws, q, n):
    rec = ws.view("rec", q, n * 12, torch.float32).cpu()
    rec_d = rec.view(torch.float64).reshape(n, 6).numpy()  # px py ca cb cc (+ packed floats)
    f32 = rec.reshape(n, 12).numpy()
    out = dict(px=rec_d[:, 0], py=rec_d[:, 1], ca=rec_d[:, 2], cb=rec_d[:, 3], cc=rec_d[:, 4],
               sigma=f32[:, 10].astype(np.float64), att=f32[:, 11].astype(np.float64))
    out["rect"] = ws.view("rect", q, 4 * n, torch.int32).cpu().numpy().reshape(n, 4)
    out["status"] = ws.view("status", q, n, torch.int32).cpu().numpy()
    out["keys"] = ws.view("keys", q, n, torch.int32).cpu().numpy().view(np.uint32)
    out["order"] = ws.view("order", q, n, torch.int32).cpu().numpy()
    return out


def test_projection_records_match_oracle():
    n = 3000
    sc = synth.scene(n, seed=0)
    rx = np.array([[0.0, 0.0, 0.0], [1.3, -2.2, 0.7]], np.float32)
    _, ws = gpu_forward(sc, synth.rss_attrs(n), rx)
    for q in range(2):
        g = _proj_from_ws(ws, q, n)
        p = oracle.project(sc, rx[q], 90, 360)
        assert np.array_equal(g["status"], p["status"])
        vis = p["status"] == oracle.ST_VISIBLE
        # after the depth sort the key buffer holds the keys in depth order
        order = oracle.depth_order(p)
        assert np.array_equal(g["keys"][:len(order)], p["r32"][order].view(np.uint32))
        assert np.all(g["keys"][len(order):] == 0xFFFFFFFF)
        assert np.abs(g["px"][vis] - p["px"][vis]).max() < 1e-9
        assert np.abs(g["py"][vis] - p["py"][vis]).max() < 1e-9
        for k in ("ca", "cb", "cc"):
            scale = np.sqrt(np.abs(p["ca"][vis] * p["cc"][vis]))
            assert (np.abs(g[k][vis] - p[k][vis]) / scale).max() < 1e-9, k
        assert np.allclose(g["sigma"][vis], p["sigma"][vis], rtol=1e-7)
        assert np.allclose(g["att"][vis], p["att"][vis], rtol=1e-7)
        assert np.array_equal(g["rect"][vis], p["rect"][vis])


def _check_order_and_lists(sc, rx, ws, n, H, W, tile, queries):
    flags = ws.flags()
    th, tw = tile
    TX, TY = oracle.tile_grid(H, W, tw, th)
    for q in queries:
        g = _proj_from_ws(ws, q, n)
        p = oracle.project(sc, rx[q], H, W)
        order = oracle.depth_order(p)
        nvis = len(order)
        assert flags[q]["n_visible"] == nvis and flags[q]["overflow"] == 0
        assert np.array_equal(g["order"][:nvis], order)
        # (i) the oracle's binning of the GPU's own rectangles
        off_i, lst_i = oracle.bin_tiles(p, g["order"][:nvis], H, W, tw, th, rect=g["rect"])
        # (ii) the oracle's binning of its own rectangles
        off_o, lst_o = oracle.bin_tiles(p, order, H, W, tw, th)
        assert flags[q]["n_pairs"] == len(lst_i)
        rng = ws.view("ranges", q, 2 * TX * TY, torch.int32).cpu().numpy().reshape(-1, 2)
        plist = ws.view("pair_list", q, len(lst_i), torch.int32).cpu().numpy()
        for t in range(TX * TY):
            got = plist[rng[t, 0]:rng[t, 1]] if rng[t, 1] > rng[t, 0] else plist[:0]
            assert np.array_equal(got, lst_i[off_i[t]:off_i[t + 1]]), (q, t)
        assert np.array_equal(off_i, off_o) and np.array_equal(lst_i, lst_o)


# Tile counts 138 (one 8-bit pass), 540 and 276 (one 10-bit pass) and 2070
# (12 bits: two 8-bit passes, then the range/list pass).  The pair sorts run
# in 16-wave workgroups when ceil(capacity / 8192) x queries >= 256 (here
# 512 pairs per Gaussian), else in 4-wave ones (the cases with fewer pairs
# per Gaussian).
@pytest.mark.parametrize("n,H,W,tile,per", [(2048, 90, 360, (16, 16), 512), (5000, 90, 360, (8, 8), 512),
                                            (4097, 180, 720, (16, 16), 512), (3000, 90, 360, (8, 16), 512),
                                            (3000, 180, 720, (8, 8), 512), (2048, 90, 360, (16, 16), 64),
                                            (4097, 180, 720, (16, 16), 200), (3000, 180, 720, (8, 8), 200)])
def test_depth_order_and_tile_lists_bit_exact(n, H, W, tile, per):
    sc = synth.scene(n, seed=1)
    rx = np.array([[0.0, 0.0, 0.0], [-2.0, 1.5, 0.3]], np.float32)
    wide = -(-(n * per + 4096) // 8192) * 2 >= 256
    assert wide == (per == 512)
    prm = gs.Params(pair_capacity=n * per + 4096)
    _, ws = gpu_forward(sc, synth.rss_attrs(n), rx, H=H, W=W, tile=tile, prm=prm)
    _check_order_and_lists(sc, rx, ws, n, H, W, tile, range(2))


def test_wide_depth_sort_bit_exact():
    # 40000 Gaussians x 52 receivers: ceil(40000 / 8192) x 52 = 260 >= 256
    # blocks, so the depth sort runs in 16-wave workgroups of 8192 keys (a
    # ragged last block of 7232); checked on the first, a middle and the last
    # receiver
    n, nq = 40_000, 52
    sc = synth.scene(n, seed=4)
    rx = synth.points(nq, seed=12)
    _, ws = gpu_forward(sc, synth.rss_attrs(n), rx)
    _check_order_and_lists(sc, rx, ws, n, 90, 360, (16, 16), (0, 25, nq - 1))


def test_depth_sort_with_a_separate_scan_bit_exact():
    # 140000 Gaussians, one receiver: ceil(140000 / 2048) = 69 blocks > 64,
    # so the depth sort's passes take the count / scan / scatter launches
    # (at most 64 blocks the scatter scans the counts itself: the tests above)
    n = 140_000
    sc = synth.scene(n, seed=5)
    rx = np.zeros((1, 3), np.float32)
    _, ws = gpu_forward(sc, synth.rss_attrs(n), rx)
    _check_order_and_lists(sc, rx, ws, n, 90, 360, (16, 16), (0,))


@pytest.mark.parametrize("n,seed,rx", [(2048, 0, (0.0, 0.0, 0.0)), (777, 5, (0.5, -0.5, 1.0)),
                                       (1, 3, (0.0, 0.0, 0.0)), (10_001, 7, (2.0, 2.0, 0.2))])
def test_pixels_match_oracle_real_f1(n, seed, rx):
    sc = synth.scene(n, seed=seed)
    attr = synth.rss_attrs(n, seed=seed + 100)
    got, ws = gpu_forward(sc, attr, np.array([rx], np.float32))
    ref = oracle.render(sc, attr, rx, 90, 360)
    check_parity(got[0], ref, "n=%d" % n)
    T, nc, _ = pixel_state(ws, 0, 90, 360)
    ok = ~ref["ambig"]
    assert np.array_equal(nc[ok], ref["n_contrib"][ok])
    assert np.allclose(T[ok], ref["T_final"][ok], rtol=1e-5, atol=1e-9)


@pytest.mark.parametrize("F,cplx,tile", [(4, True, (16, 16)), (3, False, (16, 16)), (16, True, (8, 8)),
                                         (64, True, (16, 16))])
def test_pixels_match_oracle_multichannel(F, cplx, tile):
    n = 1500
    sc = synth.scene(n, seed=11)
    attr = synth.channel_attrs(n, F, cplx, seed=12)
    got, _ = gpu_forward(sc, attr, np.zeros((1, 3), np.float32), tile=tile, is_complex=cplx)
    ref = oracle.render(sc, attr, [0, 0, 0], 90, 360)
    check_parity(got[0], ref, "F=%d" % F)


def test_batch_of_receivers_matches_single_queries():
    n = 2500
    sc = synth.scene(n, seed=21)
    attr = synth.rss_attrs(n, seed=22)
    rx = synth.points(5, seed=23)
    got, _ = gpu_forward(sc, attr, rx)
    for q in range(5):
        single, _ = gpu_forward(sc, attr, rx[q:q + 1])
        assert np.array_equal(got[q], single[0])
        ref = oracle.render(sc, attr, rx[q], 90, 360)
        check_parity(got[q], ref, "q=%d" % q)


def test_per_query_attributes_and_transmitter_attenuation():
    n = 1200
    sc = synth.scene(n, seed=31)
    B, F = 3, 2
    attr = np.stack([synth.channel_attrs(n, F, True, seed=40 + b) for b in range(B)])
    rx = np.zeros((B, 3), np.float32)
    tx = synth.points(B, seed=33)
    prm = gs.Params(atten_power=1.0, atten_ref=1)
    got, _ = gpu_forward(sc, attr, rx, tx=tx, prm=prm, is_complex=True)
    for b in range(B):
        ref = oracle.render(sc, attr[b], rx[b], 90, 360, prm=oracle_params(prm), tx=tx[b])
        check_parity(got[b], ref, "b=%d" % b)


@pytest.mark.parametrize("T_min", [0.0, 1e-2])
def test_termination_settings(T_min):
    n = 2048
    sc = synth.scene(n, seed=41)
    attr = synth.rss_attrs(n, seed=42)
    prm = gs.Params(T_min=T_min)
    got, ws = gpu_forward(sc, attr, np.zeros((1, 3), np.float32), prm=prm)
    ref = oracle.render(sc, attr, [0, 0, 0], 90, 360, prm=oracle_params(prm))
    check_parity(got[0], ref, "T_min=%g" % T_min)


def test_half_degree_grid():
    n = 4000
    sc = synth.scene(n, seed=51)
    attr = synth.rss_attrs(n, seed=52)
    got, _ = gpu_forward(sc, attr, np.zeros((1, 3), np.float32), H=180, W=720)
    ref = oracle.render(sc, attr, [0, 0, 0], 180, 720)
    check_parity(got[0], ref, "180x720")


def test_empty_scene_and_invalid_inputs_render_zero():
    n = 700
    sc = synth.scene(n, seed=61)
    sc["opacity_logit"][:] = -30.0
    got, ws = gpu_forward(sc, synth.rss_attrs(n), np.zeros((1, 3), np.float32))
    assert np.all(got == 0) and ws.flags()[0]["n_visible"] == 0
    assert ws.check() == gs._lib.GS_OK
    sc = synth.scene(n, seed=62)
    sc["mean"][0, :50] = np.nan
    sc["quat"][:, 50:60] = 0.0
    sc["log_scale"][1, 60:70] = np.inf
    attr = synth.rss_attrs(n, seed=63)
    got, ws = gpu_forward(sc, attr, np.zeros((1, 3), np.float32))
    assert ws.flags()[0]["n_invalid"] == 70
    assert ws.check() == gs._lib.GS_ERR_NONFINITE
    assert np.all(np.isfinite(got))
    ref = oracle.render(sc, attr, [0, 0, 0], 90, 360)
    check_parity(got[0], ref, "invalid")


def test_pair_capacity_overflow_is_flagged_not_faulted():
    n = 2048
    sc = synth.scene(n, seed=71)
    prm = gs.Params(pair_capacity=1000)
    got, ws = gpu_forward(sc, synth.rss_attrs(n), np.zeros((1, 3), np.float32), prm=prm)
    f = ws.flags()[0]
    assert f["overflow"] == 1 and f["n_pairs"] > 1000
    assert ws.check() == gs._lib.GS_ERR_CAPACITY
    assert np.all(np.isfinite(got))


def test_full_size_sampled_pixels_100k_64_complex():
    # the 100k-Gaussian, 64-subcarrier complex workload at full size; the
    # oracle computes a seeded sample of pixels one by one
    n, F = 100_000, 64
    sc = synth.scene(n, seed=0)
    attr = synth.channel_attrs(n, F, True, seed=81)
    got, ws = gpu_forward(sc, attr, np.zeros((1, 3), np.float32), is_complex=True)
    pix = np.sort(np.random.default_rng(82).choice(90 * 360, size=600, replace=False)).astype(np.int32)
    ref = oracle.render(sc, attr, [0, 0, 0], 90, 360, pixels=pix)
    r, c = pix // 360, pix % 360
    check_parity_at(got[0][:, r, c], ref, r, c, "100k x 64c sampled")
    assert ws.flags()[0]["overflow"] == 0
