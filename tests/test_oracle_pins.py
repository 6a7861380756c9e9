"""Pins for the CPU oracle: closed forms, invariants, special cases and brute
force, each independent of the oracle's own code path.

Paper passages: Sec. 3.2 (covariance, EWA footprint, compositing),
Sec. 4.2 (view transform, equirectangular map, projected covariance, Eq. (3)).
"""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import torch_ref

H, W = 90, 360
PI = math.pi


def one_gaussian(pos, log_s=(-2.0, -2.0, -2.0), quat=(1.0, 0.0, 0.0, 0.0), logit=0.0):
    return {"mean": np.array(pos, np.float32).reshape(3, 1),
            "log_scale": np.array(log_s, np.float32).reshape(3, 1),
            "quat": np.array(quat, np.float32).reshape(4, 1),
            "opacity_logit": np.array([logit], np.float32)}


def concat(*scenes):
    return {k: np.concatenate([s[k] for s in scenes], axis=-1) for k in scenes[0]}


def direction(az, el, r):
    """World point at azimuth az (from +x towards +y) and elevation el (from
    the horizon towards +z), distance r: the receiver frame of the default
    view, written from spherical coordinates."""
    return [r * math.cos(el) * math.cos(az), r * math.cos(el) * math.sin(az), r * math.sin(el)]


def quat_mul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def rotate_by_quat(q, v):
    """v rotated by unit quaternion q, as q v q* (Hamilton product)."""
    qc = np.array([q[0], -q[1], -q[2], -q[3]])
    return quat_mul(quat_mul(q, np.array([0.0, *v])), qc)[1:]


# ---------------------------------------------------------------- projection

@pytest.mark.parametrize("az_deg,el_deg", [(0, 0), (90, 0), (-90, 10), (45.5, 30.5), (179.5, 60.5),
                                           (-179.5, 5.5), (0.5, 89.5), (120.25, 44.75)])
def test_known_directions_land_on_known_pixels(az_deg, el_deg):
    # W/360 px per degree of azimuth starting at -180 deg; H/90 px per degree of elevation
    az, el = math.radians(az_deg), math.radians(el_deg)
    sc = one_gaussian(direction(az, el, 3.0))
    p = oracle.project(sc, [0, 0, 0], H, W)
    assert abs(p["px"][0] - (az_deg + 180.0) * W / 360.0) < 1e-4
    assert abs(p["py"][0] - el_deg * H / 90.0) < 1e-4


def test_projection_axes_follow_receiver_frame():
    # +x -> centre column, +y -> 3/4 across, -x -> seam (W == 0), zenith -> row H
    p = oracle.project(concat(one_gaussian([2, 0, 0]), one_gaussian([0, 2, 0]), one_gaussian([-2, 0, 0]),
                              one_gaussian([0, 0, 2])), [0, 0, 0], H, W)
    assert abs(p["px"][0] - W / 2) < 1e-9 and abs(p["px"][1] - 3 * W / 4) < 1e-9
    assert abs(p["px"][2] % W) < 1e-9
    assert abs(p["py"][3] - H) < 1e-9


def test_isotropic_footprint_closed_form():
    # Sigma = s^2 I  ->  Sigma' = s^2 diag((W/2pi)^2/(r cos el)^2, (2H/pi)^2/r^2) + eps I
    eps = 0.3
    for az_deg, el_deg, r, ls in [(10, 20, 3.0, -2.0), (-100, 60, 1.5, -1.0), (170, 5, 6.0, -1.5)]:
        az, el = math.radians(az_deg), math.radians(el_deg)
        p = oracle.project(one_gaussian(direction(az, el, r), log_s=(ls,) * 3), [0, 0, 0], H, W)
        s2 = math.exp(2 * ls)
        sx2 = s2 * (W / (2 * PI)) ** 2 / (r * math.cos(el)) ** 2
        sy2 = s2 * (2 * H / PI) ** 2 / r ** 2
        assert p["s00"][0] == pytest.approx(sx2 + eps, rel=1e-5)
        assert p["s11"][0] == pytest.approx(sy2 + eps, rel=1e-5)
        assert abs(p["s01"][0]) < 1e-6 * math.sqrt(sx2 * sy2)


def _world_cov(quat, log_s):
    q = np.asarray(quat, np.float64)
    q = q / np.linalg.norm(q)
    S = np.zeros((3, 3))
    for k in range(3):
        e = np.zeros(3)
        e[k] = 1.0
        a = rotate_by_quat(q, e)
        S += math.exp(2 * log_s[k]) * np.outer(a, a)
    return S


@pytest.mark.parametrize("pos,rx", [([2.0, 1.0, 1.2], [0, 0, 0]), ([-1.5, -2.5, 2.5], [0.5, 0.2, 0.3]),
                                    ([-3.0, 0.05, 0.6], [0, 0, 0])])
def test_projected_covariance_matches_numerical_linearisation(pos, rx):
    # J V Sigma V^T J^T against a central-difference Jacobian of the oracle's
    # own pixel map and a covariance built from q v q* (not from R(q)).
    quat = np.array([0.8, 0.3, -0.4, 0.35])
    log_s = (-1.2, -2.0, -1.6)
    base = one_gaussian(pos, log_s=log_s, quat=quat)
    p0 = oracle.project(base, rx, H, W)
    h = 1e-4
    Jn = np.zeros((2, 3))
    for k in range(3):
        pp, pm = [list(map(float, pos)) for _ in range(2)]
        pp[k] += h
        pm[k] -= h
        a = oracle.project({**base, "mean": np.array(pp, np.float64).reshape(3, 1)}, rx, H, W)
        b = oracle.project({**base, "mean": np.array(pm, np.float64).reshape(3, 1)}, rx, H, W)
        dpx = (a["px"][0] - b["px"][0] + W / 2) % W - W / 2
        Jn[0, k] = dpx / (2 * h)
        Jn[1, k] = (a["py"][0] - b["py"][0]) / (2 * h)
    # means are float32 inside the oracle: use the realised step
    S = _world_cov(quat, log_s)
    Sp = Jn @ S @ Jn.T + 0.3 * np.eye(2)
    assert p0["s00"][0] == pytest.approx(Sp[0, 0], rel=2e-3)
    assert p0["s11"][0] == pytest.approx(Sp[1, 1], rel=2e-3)
    assert p0["s01"][0] == pytest.approx(Sp[0, 1], rel=2e-3, abs=2e-3 * math.sqrt(Sp[0, 0] * Sp[1, 1]))


def test_projected_covariance_monte_carlo():
    # Sample a small anisotropic Gaussian, map every sample through the exact
    # equirectangular pixel map, compare the sample covariance (+ dilation).
    rng = np.random.default_rng(7)
    quat = np.array([0.6, -0.2, 0.5, 0.59])
    log_s = (-4.0, -5.0, -4.5)
    pos = np.array([1.0, 2.0, 1.5])
    S = _world_cov(quat, log_s)
    pts = rng.multivariate_normal(pos, S, size=400_000)
    az = np.arctan2(pts[:, 1], pts[:, 0])
    el = np.arcsin(pts[:, 2] / np.linalg.norm(pts, axis=1))
    px = (az / PI + 1) * W / 2
    py = 2 * el * H / PI
    C = np.cov(np.stack([px, py]))
    p = oracle.project(one_gaussian(pos, log_s=log_s, quat=quat), [0, 0, 0], H, W)
    assert p["s00"][0] - 0.3 == pytest.approx(C[0, 0], rel=1e-2)
    assert p["s11"][0] - 0.3 == pytest.approx(C[1, 1], rel=1e-2)
    assert p["s01"][0] == pytest.approx(C[0, 1], rel=3e-2)


def test_r32_key_contract_is_ieee_single():
    sc = synth.scene(5000, seed=11)
    rx = np.array([0.37, -1.21, 0.5], np.float32)
    p = oracle.project(sc, rx, H, W)
    ref = torch_ref.r32_keys(sc["mean"], rx)
    assert np.array_equal(p["r32"].view(np.uint32), ref.view(np.uint32))


# ---------------------------------------------------------------- compositing

def _centre_direction(col, row):
    """Direction of pixel centre (col + 1/2, row + 1/2)."""
    az = (col + 0.5) / W * 2 * PI - PI
    el = (row + 0.5) * PI / (2 * H)
    return az, el


@pytest.mark.parametrize("logit", [0.0, 2.5, 6.0])
def test_single_isotropic_gaussian_peak_and_profile(logit):
    col, row, r, ls = 100, 40, 2.5, -2.2
    az, el = _centre_direction(col, row)
    sc = one_gaussian(direction(az, el, r), log_s=(ls,) * 3, logit=logit)
    v = np.array([[0.7]], np.float32)
    res = oracle.render(sc, v, [0, 0, 0], H, W, prm=oracle.params(T_min=0.0))
    sigma = 1 / (1 + math.exp(-logit))
    rr = float(np.linalg.norm(sc["mean"][:, 0].astype(np.float64)))
    att = 1 / rr ** 2
    peak = min(0.99, sigma) * att * 0.7
    assert res["out"][0, row, col] == pytest.approx(peak, rel=1e-6)
    # off-peak pixels follow the closed-form footprint
    s2 = math.exp(2 * ls)
    sx2 = s2 * (W / (2 * PI)) ** 2 / (r * math.cos(el)) ** 2 + 0.3
    sy2 = s2 * (2 * H / PI) ** 2 / r ** 2 + 0.3
    for dc, dr in [(1, 0), (0, 1), (-2, 1), (3, -2)]:
        G = math.exp(-0.5 * (dc * dc / sx2 + dr * dr / sy2))
        a = min(0.99, sigma * G)
        expect = a * att * 0.7 if a >= 1 / 255 else 0.0
        assert res["out"][0, row + dr, col + dc] == pytest.approx(expect, rel=1e-4, abs=1e-12)


def test_zero_opacity_renders_nothing():
    sc = synth.scene(300, seed=3)
    sc["opacity_logit"][:] = -40.0
    res = oracle.render(sc, synth.rss_attrs(300), [0, 0, 0], H, W)
    assert res["proj"]["nvis"] == 0
    assert np.all(res["out"] == 0.0) and np.all(res["T_final"] == 1.0)


def test_telescoping_unit_values():
    # u == 1 (no attenuation, unit attribute): sum_k T_k alpha_k = 1 - prod(1 - alpha)
    sc = synth.scene(400, seed=4)
    prm = oracle.params(atten_power=0.0, T_min=0.0)
    res = oracle.render(sc, np.ones((400, 1), np.float32), [0, 0, 0], H, W, prm=prm)
    assert np.allclose(res["out"][0], 1.0 - res["T_final"], atol=1e-12)


def test_transmittance_monotone_along_list():
    # brute force per pixel: T after each accepted Gaussian never increases
    sc = synth.scene(120, seed=8)
    prm = oracle.params(T_min=0.0)
    t, a = torch_ref.to_tensors(sc, np.ones((120, 1)))
    ref = torch_ref.render(t["mean"], t["log_scale"], t["quat"], t["opacity_logit"], a, [0, 0, 0], H, W, prm)
    res = oracle.render(sc, np.ones((120, 1), np.float32), [0, 0, 0], H, W, prm=oracle.params(atten_power=0.0, T_min=0.0))
    assert np.all(res["T_final"] <= 1.0) and np.all(res["T_final"] > 0.0)
    assert np.allclose(ref["T_final"].numpy(), res["T_final"], atol=1e-14)


def test_three_gaussians_by_hand():
    # out = a1 u1 + (1-a1) a2 u2 + (1-a1)(1-a2) a3 u3 at the common pixel centre
    col, row = 200, 30
    az, el = _centre_direction(col, row)
    logits = [0.5, -0.3, 1.2]
    vals = [0.3, 0.9, 0.5]
    rs = [1.5, 2.5, 4.0]
    sc = concat(*[one_gaussian(direction(az, el, r), log_s=(-1.8,) * 3, logit=lg) for r, lg in zip(rs, logits)])
    res = oracle.render(sc, np.array(vals, np.float32)[:, None], [0, 0, 0], H, W, prm=oracle.params(T_min=0.0))
    T, out = 1.0, 0.0
    for r, lg, v in zip(rs, logits, vals):
        rr = float(np.linalg.norm(np.array(direction(az, el, r), np.float32).astype(np.float64)))
        a = min(0.99, 1 / (1 + math.exp(-lg)))
        out += T * a * v / rr ** 2
        T *= 1 - a
    assert res["out"][0, row, col] == pytest.approx(out, rel=1e-6)
    assert res["n_contrib"][row, col] == 3


def test_stop_rule_excludes_the_crossing_gaussian():
    # opaque stack: alpha = 0.99 each; T: 1 -> 0.01 -> ~1e-4 -> ~1e-6; the Gaussian that
    # would take T below T_min is not added
    col, row = 50, 10
    az, el = _centre_direction(col, row)
    sc = concat(*[one_gaussian(direction(az, el, r), log_s=(-1.0,) * 3, logit=9.0) for r in (1.0, 2.0, 3.0, 4.0)])
    prm = oracle.params(atten_power=0.0, T_min=0.9e-4)
    res = oracle.render(sc, np.ones((4, 1), np.float32), [0, 0, 0], H, W, prm=prm)
    assert res["n_contrib"][row, col] == 2
    prm = oracle.params(atten_power=0.0, T_min=1.1e-4)
    res = oracle.render(sc, np.ones((4, 1), np.float32), [0, 0, 0], H, W, prm=prm)
    assert res["n_contrib"][row, col] == 1


def test_channel_linearity_and_complex_split():
    n = 500
    sc = synth.scene(n, seed=9)
    A = synth.channel_attrs(n, 3, True, seed=10)
    full = oracle.render(sc, A, [0.1, 0.2, 0.3], H, W)
    for f in range(3):
        re = oracle.render(sc, A[:, f:f + 1, 0], [0.1, 0.2, 0.3], H, W)["out"][0]
        im = oracle.render(sc, A[:, f:f + 1, 1], [0.1, 0.2, 0.3], H, W)["out"][0]
        assert np.allclose(full["out"][f].real, re, rtol=0, atol=1e-14)
        assert np.allclose(full["out"][f].imag, im, rtol=0, atol=1e-14)


def test_over_operator_near_far_split():
    # every Gaussian of A nearer than every one of B:
    # render(A u B) = render(A) + T_A * render(B), T = T_A * T_B  (T_min = 0)
    prm = oracle.params(T_min=0.0)
    near = synth.scene(300, seed=12, lo=[-1.2, -1.2, 0.0], hi=[1.2, 1.2, 1.0])
    far = synth.scene(300, seed=13, lo=[-5, -5, 2.0], hi=[5, 5, 3.0])
    assert torch_ref.r32_keys(near["mean"], [0, 0, 0]).max() < torch_ref.r32_keys(far["mean"], [0, 0, 0]).min()
    va, vb = synth.rss_attrs(300, seed=1), synth.rss_attrs(300, seed=2)
    ra = oracle.render(near, va, [0, 0, 0], H, W, prm=prm)
    rb = oracle.render(far, vb, [0, 0, 0], H, W, prm=prm)
    rab = oracle.render(concat(near, far), np.concatenate([va, vb]), [0, 0, 0], H, W, prm=prm)
    assert np.allclose(rab["out"], ra["out"] + ra["T_final"] * rb["out"], rtol=1e-12, atol=1e-15)
    assert np.allclose(rab["T_final"], ra["T_final"] * rb["T_final"], rtol=1e-12)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_azimuth_rotation_rolls_the_image(k):
    # rotating the scene by k * 90 degrees about the up axis through the
    # receiver rolls the image by k * W/4 columns (exact in float32 for means)
    n = 800
    sc = synth.scene(n, seed=14)
    v = synth.rss_attrs(n, seed=15)
    prm = oracle.params()
    base = oracle.render(sc, v, [0, 0, 0], H, W, prm=prm)
    m = sc["mean"].copy()
    for _ in range(k):
        m = np.stack([-m[1], m[0], m[2]])
    ang = k * PI / 2
    qr = np.array([math.cos(ang / 2), 0.0, 0.0, math.sin(ang / 2)])
    q = np.stack([quat_mul(qr, sc["quat"][:, i].astype(np.float64)) for i in range(n)], 1).astype(np.float32)
    rot = oracle.render({**sc, "mean": m.astype(np.float32), "quat": q}, v, [0, 0, 0], H, W, prm=prm)
    rolled = np.roll(base["out"][0], k * W // 4, axis=1)
    ok = ~(base["ambig"] | np.roll(rot["ambig"], -k * W // 4, axis=1))
    ok = np.roll(ok, k * W // 4, axis=1)
    err = np.abs(rot["out"][0] - rolled) / np.maximum(np.roll(base["absacc"][0], k * W // 4, axis=1), 1e-30)
    assert err[ok].max() < 1e-6


def test_seam_straddler_equals_rotated_copy():
    # a Gaussian centred on the seam (azimuth 180 deg) renders the same as its
    # copy rotated to azimuth 0, rolled by W/2
    g = one_gaussian([-2.0, 0.0, 0.8], log_s=(-1.0, -1.6, -1.3), quat=(0.9, 0.1, 0.3, 0.2), logit=1.0)
    r1 = oracle.render(g, np.array([[1.0]], np.float32), [0, 0, 0], H, W)
    q = quat_mul(np.array([0.0, 0.0, 0.0, 1.0]), g["quat"][:, 0].astype(np.float64)).astype(np.float32)
    g2 = {**g, "mean": np.array([[2.0], [0.0], [0.8]], np.float32), "quat": q.reshape(4, 1)}
    r2 = oracle.render(g2, np.array([[1.0]], np.float32), [0, 0, 0], H, W)
    assert (r1["out"][0][:, :5] > 0).any() and (r1["out"][0][:, -5:] > 0).any()
    assert np.allclose(r1["out"][0], np.roll(r2["out"][0], W // 2, axis=1), rtol=1e-6, atol=1e-15)


def test_input_permutation_does_not_change_output():
    n = 600
    sc = synth.scene(n, seed=16)
    v = synth.rss_attrs(n, seed=17)
    perm = np.random.default_rng(3).permutation(n)
    keys = torch_ref.r32_keys(sc["mean"], [0, 0, 0])
    assert len(np.unique(keys)) == n
    a = oracle.render(sc, v, [0, 0, 0], H, W)
    b = oracle.render({k: x[..., perm] for k, x in sc.items()}, v[perm], [0, 0, 0], H, W)
    assert np.array_equal(a["out"], b["out"])


# ---------------------------------------------------------------- tiling

def _brute_tiles(rect, tw, th):
    c0, c1, r0, r1 = (int(x) for x in rect)
    cols = {c % W for c in range(c0, c1 + 1)} if c1 - c0 + 1 < W else set(range(W))
    TX = (W + tw - 1) // tw
    return sorted({(r // th) * TX + (c // tw) for r in range(r0, r1 + 1) for c in cols})


@pytest.mark.parametrize("tw,th", [(16, 16), (8, 8), (32, 8)])
def test_binning_matches_brute_force_and_tiling_changes_nothing(tw, th):
    n = 1500
    sc = synth.scene(n, seed=18)
    v = synth.rss_attrs(n, seed=19)
    res = oracle.render(sc, v, [0, 0, 0], H, W)
    p = res["proj"]
    off, lst = oracle.bin_tiles(p, res["order"], H, W, tw, th)
    TX, TY = oracle.tile_grid(H, W, tw, th)
    want = [[] for _ in range(TX * TY)]
    for g in res["order"]:
        for t in _brute_tiles(p["rect"][g], tw, th):
            want[t].append(int(g))
    got = [list(lst[off[t]:off[t + 1]]) for t in range(TX * TY)]
    assert got == want
    tiled = oracle.composite_tiled(p, off, lst, v, H, W, tw, th)
    assert np.array_equal(tiled["out"], res["out"])
    assert np.array_equal(tiled["T_final"], res["T_final"])
    assert np.array_equal(tiled["n_contrib"], res["n_contrib"])


def test_support_rectangle_is_conservative():
    # every pixel where alpha >= alpha_min lies inside the rectangle
    n = 400
    sc = synth.scene(n, seed=20)
    p = oracle.project(sc, [0, 0, 0], H, W)
    rows = np.arange(H)[:, None] + 0.5
    cols = np.arange(W)[None, :] + 0.5
    for g in np.nonzero(p["status"] == oracle.ST_VISIBLE)[0][:200]:
        dx = cols - p["px"][g]
        dx = np.where(dx >= W / 2, dx - W, np.where(dx < -W / 2, dx + W, dx))
        dy = rows - p["py"][g]
        q = p["ca"][g] * dx * dx + 2 * p["cb"][g] * dx * dy + p["cc"][g] * dy * dy
        inside = p["sigma"][g] * np.exp(-0.5 * q) >= 1 / 255
        c0, c1, r0, r1 = p["rect"][g]
        cols_in = np.zeros(W, bool)
        cols_in[np.arange(c0, c1 + 1) % W] = True
        rows_in = np.zeros(H, bool)
        rows_in[r0:r1 + 1] = True
        assert not np.any(inside & ~(rows_in[:, None] & cols_in[None, :]))


def test_offgrid_and_near_culls():
    below = one_gaussian([2.0, 0.0, -2.0], log_s=(-3,) * 3)
    near = one_gaussian([0.05, 0.05, 0.05])
    ok = one_gaussian([2.0, 0.0, 1.0])
    p = oracle.project(concat(below, near, ok), [0, 0, 0], H, W)
    assert list(p["status"]) == [oracle.ST_OFFGRID, oracle.ST_NEAR, oracle.ST_VISIBLE]


# ---------------------------------------------------------------- two implementations, gradients

@pytest.mark.parametrize("cplx", [False, True])
def test_c_oracle_matches_dense_torch_oracle(cplx):
    n = 150
    sc = synth.scene(n, seed=21)
    A = synth.channel_attrs(n, 2, cplx, seed=22)
    rx = [0.4, -0.3, 0.2]
    res = oracle.render(sc, A, rx, H, W)
    t, a = torch_ref.to_tensors(sc, A)
    tr = torch_ref.render(t["mean"], t["log_scale"], t["quat"], t["opacity_logit"], a, rx, H, W)
    o = tr["out"].numpy()
    if cplx:
        o = o[..., 0] + 1j * o[..., 1]
    assert np.abs(o - res["out"]).max() < 1e-13
    assert np.array_equal(tr["n_contrib"], res["n_contrib"])


def _loss_c(sc, A, G, rx, prm):
    r = oracle.render(sc, A, rx, H, W, prm=prm)
    o = r["out"]
    if np.iscomplexobj(o):
        o = np.stack([o.real, o.imag], -1)
    return float((o * G).sum()), r["n_contrib"]


@pytest.mark.slow
def test_autograd_gradients_match_central_differences():
    # FD on the C oracle, analytic via autograd on the torch oracle
    n = 24
    sc = synth.scene(n, seed=23, lo=[-2, -2, 0.2], hi=[2, 2, 2.0])
    sc64 = {k: v.astype(np.float64) for k, v in sc.items()}
    A = synth.channel_attrs(n, 2, True, seed=24)
    rx = [0.1, 0.05, 0.0]
    prm = oracle.params(T_min=0.0)
    G = np.random.default_rng(25).normal(size=(2, H, W, 2))
    t, a = torch_ref.to_tensors(sc, A, requires_grad=True)
    out = torch_ref.render(t["mean"], t["log_scale"], t["quat"], t["opacity_logit"], a, rx, H, W, prm)["out"]
    (out * torch.as_tensor(G)).sum().backward()
    rng = np.random.default_rng(26)
    checked = 0
    for name in ("mean", "log_scale", "quat", "opacity_logit"):
        grad = t[name].grad.numpy()
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in sc64[name].shape)
            th = sc64[name][idx]
            h = 1e-6 * max(1.0, abs(th))
            # the oracle reads float32 inputs: FD must move by representable steps
            vals = []
            for sgn in (+1, -1):
                s2 = {k: v.copy() for k, v in sc64.items()}
                s2[name][idx] = th + sgn * h
                vals.append(_loss_c({k: v.astype(np.float32) for k, v in s2.items()}, A, G, rx, prm))
            hp = float(np.float32(th + h)) - float(np.float32(th))
            hm = float(np.float32(th)) - float(np.float32(th - h))
            if vals[0][1].tolist() != vals[1][1].tolist() or hp == 0 or hm == 0:
                continue
            fd = (vals[0][0] - vals[1][0]) / (hp + hm)
            assert fd == pytest.approx(grad[idx], rel=2e-3, abs=2e-6 * (1 + abs(grad).max())), (name, idx)
            checked += 1
    # attributes enter linearly: FD is exact
    ga = a.grad.numpy()
    base = _loss_c(sc, A, G, rx, prm)[0]
    A2 = A.copy()
    A2[3, 1, 0] += 0.25
    assert (_loss_c(sc, A2, G, rx, prm)[0] - base) / np.float64(np.float32(A2[3, 1, 0]) - np.float32(A[3, 1, 0])) == \
        pytest.approx(ga[3, 1, 0], rel=1e-5, abs=1e-9)
    assert checked >= 12


@pytest.mark.parametrize("n,seed,rx,T_min", [(2048, 0, (0.0, 0.0, 0.0), 1e-4), (10_001, 7, (2.0, 2.0, 0.2), 1e-4),
                                             (2048, 41, (0.0, 0.0, 0.0), 1e-2)])
def test_flip_bound_covers_flipped_decisions(n, seed, rx, T_min):
    # Moving alpha_min and T_min by 1e-5 relative takes exactly the
    # decisions within the ambiguity margin the other way (the oracle's
    # model of an evaluation that decides them differently): every changed
    # pixel must be marked ambiguous and stay within its flip bound.
    sc = synth.scene(n, seed=seed)
    attr = synth.channel_attrs(n, 3, True, seed=seed + 1)
    base = oracle.render(sc, attr, rx, 90, 360, prm=oracle.params(T_min=T_min))
    amb = base["ambig"]
    assert amb.any()
    changed_any = np.zeros_like(amb)
    for sa, st in ((1, 1), (-1, -1), (1, -1), (-1, 1)):
        prm = oracle.params(T_min=T_min)
        prm[0] *= 1.0 + sa * 1e-5
        prm[2] *= 1.0 + st * 1e-5
        r = oracle.render(sc, attr, rx, 90, 360, prm=prm)
        d = np.abs(r["out"] - base["out"])
        changed = (d > 1e-12 * np.maximum(base["absacc"], 1e-30)).any(axis=0)
        assert not (changed & ~amb).any()
        assert np.all(d[:, amb] <= base["flip_bound"][:, amb])
        changed_any |= changed
    assert changed_any.any()
    assert np.all(base["flip_bound"][:, ~amb] == 0)


def test_live_set_is_whose_attributes_reach_the_image():
    # a Gaussian outside the live set is never added at any pixel (it is
    # skipped, or lies past the stop; the Gaussian that stops a pixel is not
    # added either): any attributes for all of them leave the image
    # bit-identical, while changing a live Gaussian's attributes changes it
    n = 2000
    sc = synth.scene(n, seed=91, lo=[-3, -3, 0.1], hi=[3, 3, 2.0], log_scale_mean=-1.0)
    attr = synth.channel_attrs(n, 2, True, seed=92)
    rx = [0.1, 0.2, 0.0]
    base = oracle.render(sc, attr, rx, 90, 360)
    live = base["live"]
    L = np.nonzero(live & 1)[0]
    dead = np.nonzero(live == 0)[0]
    assert 20 < len(L) < n and len(dead) > n // 2
    a2 = attr.copy()
    a2[dead] = synth.channel_attrs(len(dead), 2, True, seed=94) * 1e3
    r = oracle.render(sc, a2, rx, 90, 360)
    assert np.array_equal(r["out"], base["out"]) and np.array_equal(r["live"], live)
    for g in L[synth.subset(len(L), 24, seed=93)]:
        a3 = attr.copy()
        a3[g] += 1.0
        assert not np.array_equal(oracle.render(sc, a3, rx, 90, 360)["out"], base["out"]), g
