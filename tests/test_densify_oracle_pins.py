"""Pins of the densification oracle (oracle/densify_ref.py) against values
worked out by hand from Algorithm 1's densify branch (Sec. 4.2) and the
readings in the oracle's header."""
import numpy as np

from oracle import densify_ref as dr


def _scene5():
    # five Gaussians, one per outcome: kept, faint (pruned), large (pruned),
    # small with a high gradient (cloned), large-scale with a high gradient
    # (split in two)
    mean = np.array([[0.0, 1.0, 2.0, 3.0, 4.0], [0.0, 0.0, 0.0, 0.0, 0.0], [1.0, 1.0, 1.0, 1.0, 1.0]])
    ls = np.log(np.array([[0.05, 0.05, 0.05, 0.01, 0.2], [0.05, 0.05, 0.05, 0.01, 0.1],
                          [0.05, 0.05, 0.05, 0.01, 0.1]]))
    quat = np.array([[1.0] * 5, [0.0] * 5, [0.0] * 5, [0.0] * 5])
    op = np.array([2.0, -8.0, 2.0, 2.0, 2.0])  # sigmoid(-8) = 3.4e-4 < 0.005
    acc = np.array([0.0, 0.0, 0.0, 0.5, 0.6])  # cnt 2: means 0.25, 0.3 >= 0.1
    cnt = np.array([3, 3, 3, 2, 2])
    radius = np.array([4.0, 4.0, 50.0, 3.0, 6.0])
    return {"mean": mean, "log_scale": ls, "quat": quat, "opacity_logit": op}, acc, cnt, radius


P = dict(grad_threshold=0.1, clone_extent=0.02, opacity_min=0.005, radius_max=20.0)


def test_plan_by_hand():
    sc, acc, cnt, radius = _scene5()
    src, kind = dr.plan(sc["log_scale"], sc["opacity_logit"], acc, cnt, radius, split_n=2, **P)
    assert src.tolist() == [0, 3, 3, 4, 4]
    assert kind.tolist() == [dr.KEEP, dr.KEEP, dr.CLONE, 0, 1]


def test_prune_rules_of_new_gaussians():
    sc, acc, cnt, radius = _scene5()
    # the small Gaussian also large on screen: the parent leaves, its clone stays
    radius = radius.copy()
    radius[3] = 30.0
    src, kind = dr.plan(sc["log_scale"], sc["opacity_logit"], acc, cnt, radius, split_n=2, **P)
    assert src.tolist() == [0, 3, 4, 4] and kind.tolist() == [dr.KEEP, dr.CLONE, 0, 1]
    # a faint split candidate leaves with all its children
    op = sc["opacity_logit"].copy()
    op[4] = -9.0
    src, kind = dr.plan(sc["log_scale"], op, acc, cnt, None, split_n=3, **P)
    assert src.tolist() == [0, 2, 3, 3] and kind.tolist() == [dr.KEEP, dr.KEEP, dr.KEEP, dr.CLONE]
    # no live steps: never densified whatever the sums
    cnt0 = np.zeros(5, np.int64)
    src, kind = dr.plan(sc["log_scale"], sc["opacity_logit"], acc + 1.0, cnt0, None, split_n=2, **P)
    assert src.tolist() == [0, 2, 3, 4] and all(k == dr.KEEP for k in kind)


def test_children_by_hand():
    sc, acc, cnt, radius = _scene5()
    src, kind = np.array([4, 4]), np.array([0, 1])
    xi = np.zeros((5, 2, 3))
    xi[4, 0] = [1.0, 0.0, 0.0]
    xi[4, 1] = [0.0, -2.0, 0.5]
    out = dr.apply(sc, src, kind, xi, 2)
    # identity rotation: mu + s * xi with s = (0.2, 0.1, 0.1)
    assert np.allclose(out["mean"][:, 0], [4.2, 0.0, 1.0])
    assert np.allclose(out["mean"][:, 1], [4.0, -0.2, 1.05])
    assert np.allclose(np.exp(out["log_scale"][:, 0]), np.array([0.2, 0.1, 0.1]) / 1.6)
    assert np.allclose(out["opacity_logit"], [2.0, 2.0]) and np.allclose(out["quat"][0], 1.0)
    # a quarter turn about z: the x axis goes to y
    sc2 = {k: v.copy() for k, v in sc.items()}
    sc2["quat"][:, 4] = [np.cos(np.pi / 4), 0.0, 0.0, np.sin(np.pi / 4)]
    out = dr.apply(sc2, np.array([4]), np.array([0]), xi, 2)
    assert np.allclose(out["mean"][:, 0], [4.0, 0.2, 1.0])


def test_gather_and_clone_copies():
    sc, acc, cnt, radius = _scene5()
    src, kind = np.array([0, 3, 3, 4, 4]), np.array([dr.KEEP, dr.KEEP, dr.CLONE, 0, 1])
    arr = np.arange(2 * 5 * 3, dtype=np.float64).reshape(2, 5, 3)
    g = dr.gather(arr, src, kind, zero_new=False)
    assert g.shape == (2, 5, 3) and np.array_equal(g[:, 2], arr[:, 3]) and np.array_equal(g[:, 4], arr[:, 4])
    z = dr.gather(arr, src, kind, zero_new=True)
    assert np.array_equal(z[:, :2], arr[:, [0, 3]]) and not z[:, 2:].any()
    out = dr.apply(sc, src, kind, np.zeros((5, 2, 3)), 2)
    assert np.array_equal(out["mean"][:, 1], out["mean"][:, 2])  # a clone sits on its parent


def test_stats_and_reset():
    d = np.array([[3.0, 0.0, 1.0], [4.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    acc, cnt = dr.stats(d, [0, 2], np.zeros(3), np.zeros(3, np.int64))
    acc, cnt = dr.stats(d, [0], acc, cnt)
    assert np.allclose(acc, [10.0, 0.0, 1.0]) and cnt.tolist() == [2, 0, 1]
    r = dr.opacity_reset(np.array([3.0, -6.0, np.log(0.01 / 0.99)]))
    assert np.allclose(1.0 / (1.0 + np.exp(-r)), [0.01, 1.0 / (1.0 + np.exp(6.0)), 0.01])
