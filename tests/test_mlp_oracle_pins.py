"""Pins for the attribute-network and Adam oracle (library routines and
autograd on an independent torch formulation)."""
import numpy as np
import pytest
import torch

from oracle import mlp_ref


def test_bf16_rounding_matches_torch_conversion():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=20000) * 10.0 ** rng.integers(-8, 8, size=20000),
                        [0.0, -0.0, 1.0, 3.0 / 256, 1.00390625, 1.01171875, -2.5, 65504.0]])
    want = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp_ref.bf16(x), want)


def test_fourier_encoding_values():
    lo, hi = [-5, -5, 0], [5, 5, 3]
    g = mlp_ref.fourier(np.array([[0.0, 5.0, 0.0]]), lo, hi)[0]
    assert g.shape == (51,)
    assert np.allclose(g[:3], [0.0, 1.0, -1.0])
    # band k: sin then cos of 2^k pi u
    for k in range(8):
        s = g[3 + 6 * k:6 + 6 * k]
        c = g[6 + 6 * k:9 + 6 * k]
        assert np.allclose(s, np.sin(2 ** k * np.pi * np.array([0.0, 1.0, -1.0])), atol=1e-12)
        assert np.allclose(c, np.cos(2 ** k * np.pi * np.array([0.0, 1.0, -1.0])), atol=1e-12)


def _torch_net(w, E, tx, mean, r_near, lo, hi):
    # an independent formulation: one dense layer stack in torch FP64
    t = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in w.items()}
    Et = torch.tensor(E, dtype=torch.float64, requires_grad=True)
    g = torch.tensor(mlp_ref.fourier(tx, lo, hi))
    S, n = g.shape[0], E.shape[0]
    x = torch.cat([Et[None].expand(S, n, 32), g[:, None, :].expand(S, n, 51), torch.zeros(S, n, 13,
                                                                                             dtype=torch.float64)], -1)
    h1 = torch.relu(x @ t["W1"].T + t["b1"])
    h2 = torch.relu(h1 @ t["W2"].T + t["b2"])
    o = h2 @ t["W3"].T + t["b3"]
    d = torch.clamp(torch.linalg.norm(torch.tensor(mean.T)[None] - torch.tensor(tx)[:, None], dim=-1), min=r_near)
    amp = torch.sigmoid(o[..., :64] - torch.log(d)[..., None])
    ph = o[..., 64:]
    attr = torch.stack([amp * torch.cos(ph), amp * torch.sin(ph)], -1)
    return attr, t, Et


def test_forward_and_backward_match_torch_autograd_without_rounding():
    rng = np.random.default_rng(1)
    w = mlp_ref.init(2)
    w["b1"] = rng.normal(0, 0.1, 64)
    w["b3"] = rng.normal(0, 0.1, 128)
    n, S = 40, 3
    E = rng.normal(0, 0.1, size=(n, 32))
    tx = rng.uniform([-5, -5, 0], [5, 5, 3], size=(S, 3))
    mean = rng.uniform([-5, -5, 0], [5, 5, 3], size=(n, 3)).T
    lo, hi = [-5, -5, 0], [5, 5, 3]
    fw = mlp_ref.forward(w["W1"], w["b1"], w["W2"], w["b2"], w["W3"], w["b3"], E, tx, mean, 0.2, lo, hi,
                         round_bf16=False)
    attr, t, Et = _torch_net(w, E, tx, mean, 0.2, lo, hi)
    assert np.allclose(fw["attr"], attr.detach().numpy(), rtol=1e-12, atol=1e-14)
    G = rng.normal(size=attr.shape)
    (attr * torch.tensor(G)).sum().backward()
    gr = mlp_ref.backward(fw, G, round_bf16=False)
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        ref = t[k].grad.numpy()
        if k == "W1":
            ref = ref.copy()
            ref[:, 83:] = 0.0  # padding columns carry no input
        assert np.allclose(gr[k], ref, rtol=1e-10, atol=1e-12), k
    assert np.allclose(gr["E"], Et.grad.numpy(), rtol=1e-10, atol=1e-12)


def test_rounding_points_change_the_result_only_at_bf16_scale():
    rng = np.random.default_rng(3)
    w = mlp_ref.init(4)
    E = rng.normal(0, 0.1, size=(30, 32))
    tx = rng.uniform([-5, -5, 0], [5, 5, 3], size=(2, 3))
    mean = rng.uniform([-5, -5, 0], [5, 5, 3], size=(30, 3)).T
    a = mlp_ref.forward(w["W1"], w["b1"], w["W2"], w["b2"], w["W3"], w["b3"], E, tx, mean, 0.2,
                        [-5, -5, 0], [5, 5, 3])["attr"]
    b = mlp_ref.forward(w["W1"], w["b1"], w["W2"], w["b2"], w["W3"], w["b3"], E, tx, mean, 0.2,
                        [-5, -5, 0], [5, 5, 3], round_bf16=False)["attr"]
    rel = np.abs(a - b).max() / np.abs(b).max()
    assert 1e-5 < rel < 5e-2


def test_adam_matches_torch_optim():
    rng = np.random.default_rng(5)
    p0 = rng.normal(size=100)
    p = torch.tensor(p0.copy(), requires_grad=True)
    opt = torch.optim.Adam([p], lr=3e-3, betas=(0.9, 0.999), eps=1e-15)
    q, m, v = p0.copy(), np.zeros(100), np.zeros(100)
    for t in range(1, 8):
        g = rng.normal(size=100)
        opt.zero_grad()
        p.grad = torch.tensor(g)
        opt.step()
        q, m, v = mlp_ref.adam(q, g, m, v, t, 3e-3)
    assert np.allclose(q, p.detach().numpy(), rtol=0, atol=1e-14)


LO, HI = [-5.0, -5.0, 0.0], [5.0, 5.0, 3.0]


def _zeros():
    return dict(W1=np.zeros((64, 96)), b1=np.zeros(64), W2=np.zeros((64, 64)), b2=np.zeros(64),
                W3=np.zeros((128, 64)), b3=np.zeros(128))


@pytest.mark.parametrize("rounding", [True, False])
def test_zero_network_closed_form(rounding):
    # every weight zero: o = b3, amplitude sigmoid(b3_f - ln d) = 1 / (1 + d exp(-b3_f)),
    # phase b3_{64+f}; with b3 = 0, amplitude 1 / (1 + d) and phase 0
    w = _zeros()
    w["b3"][:64] = np.linspace(-2.0, 2.0, 64)
    w["b3"][64:] = np.linspace(-3.0, 3.0, 64)
    rng = np.random.default_rng(7)
    n = 6
    E = rng.normal(0, 0.1, size=(n, 32))
    tx = np.array([[1.0, -2.0, 0.5], [0.0, 0.0, 3.0]])
    mean = rng.uniform(LO, HI, size=(n, 3))
    mean[2] = tx[0] + [0.0, 0.05, 0.0]          # within r_near of transmitter 0: d floored at 0.2
    fw = mlp_ref.forward(w["W1"], w["b1"], w["W2"], w["b2"], w["W3"], w["b3"], E, tx, mean.T, 0.2, LO, HI,
                         round_bf16=rounding)
    for s in range(2):
        d = np.maximum(np.linalg.norm(mean - tx[s], axis=1), 0.2)
        amp = 1.0 / (1.0 + d[:, None] * np.exp(-w["b3"][None, :64]))
        ph = w["b3"][None, 64:]
        assert np.allclose(fw["attr"][s, ..., 0], amp * np.cos(ph), rtol=0, atol=1e-15)
        assert np.allclose(fw["attr"][s, ..., 1], amp * np.sin(ph), rtol=0, atol=1e-15)
    assert abs(np.hypot(*fw["attr"][0, 2, 32]) - 1.0 / (1.0 + 0.2 * np.exp(-w["b3"][32]))) < 1e-15


@pytest.mark.parametrize("rounding", [True, False])
def test_one_hot_network_by_hand(rounding):
    """Three Gaussians with one-hot embeddings 0.5 e_i, a transmitter at
    (2.5, 0, 1.5) (encoded u = (0.5, 0, 0)); every value is exact in BF16, so
    the rounding points change nothing.
      layer 1: unit j < 3 reads embedding dim j (weight 1), unit 3 reads u_x
               (weight 2); b1[1] = -0.75, b1[3] = 0.25
               z1 for Gaussian 0 = (0.5, -0.75, 0, 1.25)  h1 = (0.5, 0, 0, 1.25)
                          1      (0, -0.25, 0, 1.25)             (0, 0, 0, 1.25)
                          2      (0, -0.75, 0.5, 1.25)           (0, 0, 0.5, 1.25)
      layer 2: identity on units 0..3: h2 = h1
      layer 3: o_0 = 2 h2_0 + h2_3, o_1 = -4 h2_2, o_2 = b3[2] = 0.5,
               o_64 = h2_3, o_65 = -2 h2_0, o_66 = b3[66] = 0.25
               Gaussian 0: o_0 = 2.25, o_1 = 0,  phases (1.25, -1, 0.25)
                        1: o_0 = 1.25, o_1 = 0,  phases (1.25, 0, 0.25)
                        2: o_0 = 1.25, o_1 = -2, phases (1.25, 0, 0.25)
    Distances to the transmitter: 1, 2 and 0.1 (floored at r_near = 0.2);
    amplitude 1 / (1 + d exp(-o)), all other subcarriers amplitude 1/(1+d),
    phase 0."""
    w = _zeros()
    for j in range(3):
        w["W1"][j, j] = 1.0
    w["W1"][3, 32] = 2.0
    w["b1"][1], w["b1"][3] = -0.75, 0.25
    for j in range(4):
        w["W2"][j, j] = 1.0
    w["W3"][0, 0], w["W3"][0, 3] = 2.0, 1.0
    w["W3"][1, 2] = -4.0
    w["W3"][64, 3] = 1.0
    w["W3"][65, 0] = -2.0
    w["b3"][2], w["b3"][66] = 0.5, 0.25
    E = np.zeros((3, 32))
    for i in range(3):
        E[i, i] = 0.5
    tx = np.array([[2.5, 0.0, 1.5]])
    mean = np.array([[3.5, 0.0, 1.5], [2.5, 2.0, 1.5], [2.5, 0.0, 1.4]], np.float32)
    fw = mlp_ref.forward(w["W1"], w["b1"], w["W2"], w["b2"], w["W3"], w["b3"], E, tx, mean.T, 0.2, LO, HI,
                         round_bf16=rounding)
    assert np.allclose(fw["g"][0, :3], [0.5, 0.0, 0.0], rtol=0, atol=1e-15)
    d = [1.0, 2.0, 0.2]
    o = [(2.25, 0.0), (1.25, 0.0), (1.25, -2.0)]
    ph = [(1.25, -1.0), (1.25, 0.0), (1.25, 0.0)]
    for i in range(3):
        amp = np.full(64, 1.0 / (1.0 + d[i]))
        amp[0] = 1.0 / (1.0 + d[i] * np.exp(-o[i][0]))
        amp[1] = 1.0 / (1.0 + d[i] * np.exp(-o[i][1]))
        amp[2] = 1.0 / (1.0 + d[i] * np.exp(-0.5))
        phase = np.zeros(64)
        phase[0], phase[1], phase[2] = ph[i][0], ph[i][1], 0.25
        a = fw["attr"][0, i]
        assert np.allclose(a[:, 0], amp * np.cos(phase), rtol=0, atol=1e-12), i
        assert np.allclose(a[:, 1], amp * np.sin(phase), rtol=0, atol=1e-12), i
