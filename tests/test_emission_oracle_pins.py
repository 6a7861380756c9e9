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


def _hand_network(H):
    """A network whose outputs are worked out by hand (receiver x = (0.5, -1, 2)).

    Unit j < 8 reads input j mod 3 with weight 1 and bias b[j]:
      j  input  z = x + b           h = relu(z)
      0  0.5    0.5 + 0.25 = 0.75   0.75
      1  -1     -1 + 0.5 = -0.5     0
      2  2      2 - 3 = -1          0
      3  0.5    0.5 + 1 = 1.5       1.5
      4  -1     -1 + 0 = -1         0
      5  2      2 - 1 = 1           1
      6  0.5    0.5 - 1 = -0.5      0
      7  -1     -1 + 2 = 1          1
    Units j >= 8 read (1, 1, 1) with bias -10 (z = 1.5 - 10 < 0: dead) and
    carry output weight 5, which only a missing ReLU would let through.
    Output row 0 weighs every live unit by 1: 0.75 + 1.5 + 1 + 1 = 4.25;
    row 1 weighs unit j by j: 3 * 1.5 + 5 * 1 + 7 * 1 = 16.5.
    With b2 = (-3, -15): f = (1.25, 1.5)."""
    W1 = np.zeros((H, 3))
    b1 = np.zeros(H)
    W2 = np.zeros((2, H))
    for j in range(8):
        W1[j, j % 3] = 1.0
        W2[0, j] = 1.0
        W2[1, j] = float(j)
    b1[:8] = [0.25, 0.5, -3.0, 1.0, 0.0, -1.0, -1.0, 2.0]
    W1[8:] = 1.0
    b1[8:] = -10.0
    W2[:, 8:] = 5.0
    b2 = np.array([-3.0, -15.0])
    # the documented flat order: W1 [H][3] row-major, b1 [H], W2 [2][H] row-major, b2 [2]
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2])


def test_hand_computed_network_at_each_width():
    # pins the parameter order, the ReLU, which layer the output weights act
    # on, and the sign of the log-distance bias: f = (1.25, 1.5) by hand
    for H in (8, 16, 64):
        p = _hand_network(H)
        assert p.size == er.nparam(H)
        P = np.stack([p, p, p])
        mean = np.array([[1.0, 1.0, 1.0], [0.0, 0.0, 0.0], [3.0, 4.0, 0.0]])
        rx = np.array([[0.5, -1.0, 2.0]])
        # transmitter at distance 1 from Gaussian 0 (log d = 0), e from
        # Gaussian 1 (log d = 1) and 0.05 from Gaussian 2 (floored at 0.2)
        e = np.e
        tx = np.array([[1.0, 1.0, 2.0]])
        s = er.forward(P, mean, rx, tx)[0]
        assert abs(np.linalg.norm(tx[0] - mean[0]) - 1.0) < 1e-15
        sig = lambda u: 1.0 / (1.0 + np.exp(-u))  # noqa: E731
        assert np.allclose(s[0], [sig(1.25), sig(1.5)], rtol=0, atol=1e-15)
        tx1 = np.array([[e, 0.0, 0.0]])
        s1 = er.forward(P, mean, rx, tx1)[0]
        assert np.allclose(s1[1], [sig(1.25 - 1.0), sig(1.5 - 1.0)], rtol=0, atol=1e-15)
        tx2 = np.array([[3.0, 4.0, 0.05]])
        s2 = er.forward(P, mean, rx, tx2)[0]
        # sigmoid(f - log 0.2) = 1 / (1 + 0.2 exp(-f))
        assert np.allclose(s2[2], [1.0 / (1.0 + 0.2 * np.exp(-1.25)), 1.0 / (1.0 + 0.2 * np.exp(-1.5))],
                           rtol=0, atol=1e-15)
