"""Pins of the per-Gaussian emission oracle (Sec. 4.1, Eq. (1)) to facts
fixed by the formula and by calculus, not by the oracle itself:

* with every network weight zero, s_i = sigmoid(-log d_i) = 1 / (1 + d_i) on
  both parts (closed form), and the floor d_i >= r_near holds;
* the 3 -> 16 -> 2 shape has 98 parameters (the paper's count);
* Gaussian i's emission depends on its own parameters only;
* the gradients match central finite differences of sum(ds * s).
"""
import numpy as np

from oracle import emission_ref as er


def scene(n, seed):
    r = np.random.default_rng(seed)
    P = r.normal(0, 0.6, (n, er.NPARAM))
    mean = r.uniform(-3, 3, (n, 3))
    rx = r.uniform(-2, 2, (3, 3))
    tx = r.uniform(-4, 4, (3, 3))
    return P, mean, rx, tx


def test_parameter_count():
    assert er.NPARAM == 98 == er.nparam(16)
    assert er.nparam(8) == 50 and er.nparam(64) == 386


def test_other_widths_zero_network_and_finite_differences():
    for H in (8, 64):
        P, mean, rx, tx = scene(3, 20 + H)
        P = np.random.default_rng(H).normal(0, 0.4, (3, er.nparam(H)))
        s = er.forward(np.zeros_like(P), mean, rx, tx)
        d = np.maximum(np.linalg.norm(tx[0] - mean, axis=1), er.R_NEAR)
        assert np.allclose(s[0, :, 0], 1.0 / (1.0 + d), rtol=0, atol=1e-15)
        ds = np.random.default_rng(H + 1).normal(size=(3, 3, 2))
        dP, _ = er.backward(P, mean, rx, tx, ds)
        f = lambda P_: float((ds * er.forward(P_, mean, rx, tx)).sum())  # noqa: E731
        for k in range(0, er.nparam(H), 7):
            a = P.copy(); a[1, k] += 1e-6
            b = P.copy(); b[1, k] -= 1e-6
            num = (f(a) - f(b)) / 2e-6
            assert abs(dP[1, k] - num) <= 1e-6 * max(1.0, abs(num)), (H, k)


def test_zero_network_is_inverse_one_plus_distance():
    P, mean, rx, tx = scene(50, 1)
    tx[0] = mean[7]          # distance 0: the floor applies
    s = er.forward(np.zeros_like(P), mean, rx, tx)
    for q in range(3):
        d = np.maximum(np.linalg.norm(tx[q] - mean, axis=1), er.R_NEAR)
        assert np.allclose(s[q, :, 0], 1.0 / (1.0 + d), rtol=0, atol=1e-15)
        assert np.allclose(s[q, :, 1], 1.0 / (1.0 + d), rtol=0, atol=1e-15)
    assert abs(s[0, 7, 0] - 1.0 / (1.0 + er.R_NEAR)) < 1e-15


def test_each_gaussian_uses_its_own_parameters():
    P, mean, rx, tx = scene(20, 2)
    s0 = er.forward(P, mean, rx, tx)
    P2 = P.copy()
    P2[5] += 1.0
    s1 = er.forward(P2, mean, rx, tx)
    changed = np.abs(s1 - s0).max(axis=(0, 2)) > 0
    assert changed[5] and changed.sum() == 1


def test_gradients_match_finite_differences():
    P, mean, rx, tx = scene(4, 3)
    ds = np.random.default_rng(4).normal(size=(3, 4, 2))
    dP, dmean = er.backward(P, mean, rx, tx, ds)
    f = lambda P_, m_: float((ds * er.forward(P_, m_, rx, tx)).sum())  # noqa: E731
    eps = 1e-6
    for i in range(4):
        for k in range(er.NPARAM):
            a = P.copy(); a[i, k] += eps
            b = P.copy(); b[i, k] -= eps
            num = (f(a, mean) - f(b, mean)) / (2 * eps)
            assert abs(dP[i, k] - num) <= 1e-6 * max(1.0, abs(num)), (i, k)
        for k in range(3):
            a = mean.copy(); a[i, k] += eps
            b = mean.copy(); b[i, k] -= eps
            num = (f(P, a) - f(P, b)) / (2 * eps)
            assert abs(dmean[i, k] - num) <= 1e-6 * max(1.0, abs(num)), (i, k)
