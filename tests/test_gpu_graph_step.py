"""The training step and the serving render captured as HIP graphs
(torch.cuda.CUDAGraph around the library's launches) replay what the eager
calls compute.

Training cases: 4000 Gaussians with 4 transmitters at 90x360, and the
at-scale shape (300k Gaussians, 180x720, 32 complex subcarriers, 64
transmitters) that the benchmark replays.  Every replay is checked against
an eager call from the same state: the model
state is snapshotted, one eager step runs, the state is restored, unrelated
eager work and a synchronisation follow, then the graph replays.  Losses and
every gradient agree to FP32 summation order (float atomics), the updated
parameters to the same order through Adam; the serving spectra of every
replay equal the eager ones bit for bit (no atomics on that path).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import mlp_ref
from paper_2511_22793_amd import train
from test_gpu_backward import compare

pytestmark = pytest.mark.gpu

LO, HI = [-5.0, -5.0, 0.0], [5.0, 5.0, 3.0]


def capture(fn, warm=2):
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(warm):
            fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    torch.cuda.synchronize()
    return g


def _state(m):
    ts = [m.g[k] for k in sorted(m.g)] + [m.E, m.E_bf, m.step_dev, m.skipped]
    ts += [m.net.w[k] for k in sorted(m.net.w)] + [m.net.bf[k] for k in sorted(m.net.bf)]
    for k in sorted(m.moments):
        ts += list(m.moments[k])
    return ts


def _grads(m):
    # (d_attr is cleared by the network backward once consumed: not an output)
    out = {"loss": m.loss.clone()}
    out.update({"g_" + k: v.clone() for k, v in m.ggrads.items() if k != "d_attr"})
    out.update({"m_" + k: v.clone() for k, v in m.mgrads.items()})
    return out


def _groups(m):
    """(parameter, gradient, first moment, second moment, lr at step u) per
    Adam segment of the training step."""
    r = m.rates
    gr = [(m.net.w[k], m.mgrads[k], m.moments[k], lambda u: r.mlp) for k in ("W1", "b1", "W2", "b2", "W3", "b3")]
    gr.append((m.E, m.mgrads["E"], m.moments["E"], lambda u: r.embedding))
    gr.append((m.g["mean"], m.ggrads["d_mean"], m.moments["mean"],
               lambda u: r.position * (r.position_final / r.position) ** u))
    for k, lr in (("log_scale", r.scaling), ("quat", r.rotation), ("opacity_logit", r.opacity)):
        gr.append((m.g[k], m.ggrads["d_" + k], m.moments[k], lambda u, lr=lr: lr))
    return gr


def test_training_step_graph_replays_match_eager_steps():
    n, B, F = 4000, 4, 64
    total = 50
    sc = synth.scene(n, seed=51, lo=[-3, -3, 0.1], hi=[3, 3, 2.5])
    model = train.LearnedScene(sc, synth.embeddings(n, seed=52), train.init_weights(53), [0, 0, 0], B, LO, HI,
                               total_steps=total)
    tx = torch.from_numpy(synth.points(B, seed=54)).cuda()
    target = torch.from_numpy(synth.normal((B, F, 90, 360, 2), 0.05, seed=55)).cuda()
    _replays_match_eager(model, tx, target, total)


def test_training_step_graph_replays_match_eager_steps_at_scale():
    # the at-scale training shape: 300k Gaussians, 180x720, 32 complex
    # subcarriers, 64 transmitters (targets drawn on the device)
    n, B, F = 300_000, 64, 32
    total = 1000
    sc = synth.scene(n, seed=56)
    model = train.LearnedScene(sc, synth.embeddings(n, seed=57), train.init_weights(58, n_chan=F), [0, 0, 0], B,
                               list(synth.BOX_LO), list(synth.BOX_HI), grid=train.Grid(180, 720),
                               total_steps=total)
    tx = torch.from_numpy(synth.points(B, seed=59)).cuda()
    gen = torch.Generator(device="cuda").manual_seed(60)
    target = torch.randn(B, F, 180, 720, 2, device="cuda", generator=gen) * 0.05
    _replays_match_eager(model, tx, target, total)


def _replays_match_eager(model, tx, target, total):
    tmean = train.spatial_mean(target, True)

    def step():
        model.train_step(tx, target, target_mean=tmean)

    g = capture(step)
    for rep in range(3):
        before = [t.clone() for t in _state(model)]
        t_done = int(model.step_dev.item())
        step()
        torch.cuda.synchronize()
        eager = _grads(model)
        for t, b in zip(_state(model), before):
            t.copy_(b)
        old = [(p.double().cpu().numpy(), mm.double().cpu().numpy(), vv.double().cpu().numpy())
               for p, _, (mm, vv), _ in _groups(model)]
        # unrelated eager work between the eager step and the replay
        x = torch.randn(512, 512, device="cuda")
        (x @ x).sum().item()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert int(model.skipped.item()) == 0
        assert int(model.step_dev.item()) == t_done + 1, "the replay advances the device step counter"
        got = _grads(model)
        for k, v in eager.items():
            a, b = got[k].double().cpu().numpy(), v.double().cpu().numpy()
            if k.startswith("m_"):
                # network gradients pass through BF16-rounded intermediates:
                # a last-bit difference upstream (float atomics) can flip a
                # rounding, so they agree to the BF16 flip bound
                assert np.abs(a - b).max() <= 2e-2 * np.abs(b).max(), "replay %d %s" % (rep, k)
            else:
                compare(a, b, "replay %d %s" % (rep, k))
        # the replay's update is Adam at the device step number and schedule,
        # applied to the replay's own gradients
        u = min((t_done + 1) / (total - 1), 1.0)
        # (FP32 against FP64 arithmetic: 1e-3 of each update; a wrong step
        # number or rate moves the updates by 10% or more)
        for gi, ((p, grad, _, lr), (p0, m0, v0)) in enumerate(zip(_groups(model), old)):
            want, _, _ = mlp_ref.adam(p0, grad.double().cpu().numpy(), m0, v0, t_done + 1, lr(u))
            got_p = p.double().cpu().numpy()
            allow = 1e-3 * np.abs(want - p0) + 1e-6 * lr(u) + 2.4e-7 * np.abs(want)
            excess = np.abs(got_p - want) - allow
            assert np.all(excess <= 0), "replay %d group %d: max excess %.3g (lr %.3g, step %d)" % (
                rep, gi, excess.max(), lr(u), t_done + 1)


def test_serving_render_graph_replays_match_eager():
    n, B = 20_000, 8
    sc = synth.scene(n, seed=61)
    model = train.LearnedScene(sc, synth.embeddings(n, seed=62), train.init_weights(63), [0, 0, 0], B, LO, HI)
    tx = torch.from_numpy(synth.points(B, seed=64)).cuda()
    ref = model.render(tx).clone()
    torch.cuda.synchronize()
    g = capture(lambda: model.render(tx))
    for rep in range(3):
        model.spec.fill_(float("nan"))
        y = torch.randn(256, 256, device="cuda")
        (y @ y).sum().item()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(model.spec, ref), "replay %d" % rep
