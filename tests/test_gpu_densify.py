"""Densification, pruning and opacity reset (Algorithm 1's densify branch)
against the oracle (oracle/densify_ref.py).

* statistics: the live Gaussians' |dL/dmu| sums (1e-6 relative) and counts
  (exact);
* the plan: the new set's slots (parent, kind) and count bit for bit, on
  inputs whose statistics, scales, opacities and radii keep 1% or more
  from each threshold (the decisions are FP32 comparisons on both sides);
  sizes of one Gaussian, across two scan blocks (1025) and 20000;
* the new scene: copies exact, split children within 2e-6 of the FP64
  oracle (relative to the scale of the numbers);
* gathers exact (FP32 rows, SoA components, 16-bit rows), new rows zeroed
  when asked; the opacity reset; the screen radius from a prepared
  workspace against the oracle projection's rectangles;
* in training: a LearnedScene densifies mid-run and keeps training.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2511_22793_amd as gs
import synth
from oracle import densify_ref as dr
from paper_2511_22793_amd import densify as gd
from paper_2511_22793_amd import train

pytestmark = pytest.mark.gpu

P = gd.DensifyParams(grad_threshold=0.1, clone_extent=0.05, split_n=2, opacity_min=0.005, radius_max=20.0)


def _inputs(n, seed, split_n=2):
    rng = np.random.default_rng(seed)
    sc = synth.scene(n, seed=seed)
    # scales away from clone_extent by >= 10%, opacities from sigma_min
    s = np.exp(rng.uniform(np.log(0.005), np.log(0.5), size=(3, n)))
    smax = s.max(0)
    s[:, np.abs(smax / P.clone_extent - 1.0) < 0.1] *= 0.5
    sc["log_scale"] = np.log(s).astype(np.float32)
    op = rng.uniform(-9.0, 3.0, n)
    sig = 1.0 / (1.0 + np.exp(-op))
    op[np.abs(sig / P.opacity_min - 1.0) < 0.05] += 1.0
    sc["opacity_logit"] = op.astype(np.float32)
    cnt = rng.integers(0, 4, n).astype(np.int32)
    g = np.where(rng.random(n) < 0.3, rng.uniform(2.0, 5.0, n), rng.uniform(0.0, 0.5, n)) * P.grad_threshold
    acc = (g * cnt).astype(np.float32)
    radius = np.where(rng.random(n) < 0.1, rng.uniform(25.0, 60.0, n), rng.uniform(0.0, 15.0, n)).astype(np.float32)
    xi = rng.normal(size=(n, split_n, 3)).astype(np.float32)
    return sc, acc, cnt, radius, xi


def d(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("n,seed", [(1, 1), (1025, 2), (20_000, 3)])
def test_plan_apply_gather_match_oracle(n, seed):
    sc, acc, cnt, radius, xi = _inputs(n, seed)
    dsc = {k: d(v) for k, v in sc.items()}
    src, kind, n_out = gd.plan(dsc, d(acc), d(cnt), d(radius), P)
    rs, rk = dr.plan(sc["log_scale"], sc["opacity_logit"], acc, cnt, radius, P.grad_threshold, P.clone_extent,
                     P.split_n, P.opacity_min, P.radius_max)
    assert n_out == len(rs)
    assert np.array_equal(src[:n_out].cpu().numpy(), rs) and np.array_equal(kind[:n_out].cpu().numpy(), rk)
    if n_out == 0:
        return
    out = gd.apply(dsc, src, kind, n_out, d(xi), P.split_n)
    ref = dr.apply(sc, rs, rk, xi, P.split_n)
    for k in ("mean", "log_scale", "quat", "opacity_logit"):
        got = out[k].cpu().double().numpy()
        want = ref[k]
        assert np.abs(got - want).max() <= 2e-6 * max(1.0, np.abs(want).max()), k
    keep = rk < 0
    assert np.array_equal(out["mean"].cpu().numpy()[:, keep], sc["mean"][:, rs[keep]])
    # gathers: [3][n] floats, [n][8] floats, [n][32] 16-bit words
    rng = np.random.default_rng(seed + 1)
    a3 = rng.normal(size=(3, n)).astype(np.float32)
    a8 = rng.normal(size=(n, 8)).astype(np.float32)
    ah = rng.integers(-30000, 30000, size=(n, 32)).astype(np.int16)
    for arr, comps, z in ((a3, 3, True), (a8, 1, False), (ah, 1, True)):
        got = gd.gather(d(arr), src, kind, n, n_out, comps, z).cpu().numpy()
        view = arr.reshape(comps, n, -1)
        want = dr.gather(view, rs, rk, z).reshape(got.shape)
        assert np.array_equal(got, want)


def test_stats_reset_and_radius():
    n = 3000
    rng = np.random.default_rng(5)
    dm = rng.normal(size=(3, n)).astype(np.float32)
    live = np.sort(rng.choice(n, 700, replace=False)).astype(np.int32)
    acc = torch.zeros(n, device="cuda")
    cnt = torch.zeros(n, dtype=torch.int32, device="cuda")
    for _ in range(2):
        gd.stats(d(dm), d(live), d(np.array([len(live)], np.int32)), acc, cnt)
    ra, rc = dr.stats(dm, live, np.zeros(n), np.zeros(n, np.int64))
    ra, rc = dr.stats(dm, live, ra, rc)
    assert np.allclose(acc.cpu().numpy(), ra, rtol=1e-6, atol=0) and np.array_equal(cnt.cpu().numpy(), rc)
    ol = rng.uniform(-8, 4, n).astype(np.float32)
    t = d(ol)
    gd.opacity_reset(t)
    assert np.allclose(t.cpu().numpy(), dr.opacity_reset(ol), rtol=0, atol=1e-6)
    # screen radius of a prepared receiver against the oracle's rectangles
    sc = synth.scene(n, seed=6)
    ws = gs.prepare({k: d(v) for k, v in sc.items()}, torch.zeros(1, 3, device="cuda"))
    r = gd.screen_radius(ws).cpu().numpy()
    proj = oracle.project(sc, [0, 0, 0], 90, 360)
    rect, vis = proj["rect"], proj["status"] == 0
    want = np.where(vis, 0.5 * np.maximum(rect[:, 1] - rect[:, 0] + 1, rect[:, 3] - rect[:, 2] + 1), 0.0)
    assert np.array_equal(r, want.astype(np.float32))


def test_training_densifies_and_continues():
    n, B = 3000, 2
    sc = synth.scene(n, seed=81, lo=[-3, -3, 0.1], hi=[3, 3, 2.5])
    model = train.LearnedScene(sc, synth.embeddings(n, seed=82), train.init_weights(83), [0, 0, 0], B,
                               [-5.0, -5.0, 0.0], [5.0, 5.0, 3.0], densify_stats=True)
    tx = torch.from_numpy(synth.points(B, seed=84)).cuda()
    target = torch.from_numpy(synth.normal((B, train.F, 90, 360, 2), 0.05, seed=85)).cuda()
    for _ in range(3):
        model.train_step(tx, target)
    torch.cuda.synchronize()
    cnt = model.grad_cnt.cpu().numpy()
    assert cnt.max() == 3 and (cnt > 0).sum() >= int(model.live_count.item())
    # a threshold that densifies a share of the live set
    g = (model.grad_acc.cpu().numpy() / np.maximum(cnt, 1))[cnt > 0]
    prm = gd.DensifyParams(grad_threshold=float(np.quantile(g, 0.5)), clone_extent=0.05, split_n=2,
                           opacity_min=0.005, radius_max=1e4)
    n_new = model.densify(prm, seed=86)
    assert n_new > n * 0.5 and model.n == n_new and model.g["mean"].shape == (3, n_new)
    model.opacity_reset()
    for _ in range(2):
        loss = model.train_step(tx, target)
    torch.cuda.synchronize()
    assert np.all(np.isfinite(loss.cpu().numpy())) and int(model.skipped.item()) == 0
    assert torch.all(torch.sigmoid(model.g["opacity_logit"]) <= 0.0101 + 1e-3)
