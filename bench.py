"""Benchmark of the hemispherical RF splatting hot path on one MI355X.

Workload: 100,000 Gaussians (means U([-5,5]x[-5,5]x[0,3]) m, log-scales
N(-1.5,0.5), uniform unit quaternions, opacity logits N(0,1)), a 32-d
embedding per Gaussian N(0, 0.1^2), the attribute network (Fourier-encoded
transmitter, 2 hidden layers of 64, BF16 weights, FP32 accumulation) giving
64 complex subcarriers, a receiver at the floor centre, 90 x 360 grid.
Targets: spectra of an independent ground-truth scene whose Gaussians emit
reflectivity x transmitter-leg delay phase / distance, rendered by the plain
renderer.  All data synthetic and seeded.

A step is one pass of the whole hot path over a batch of B = 16 transmitter
queries: network forward, projection + depth sort + tile binning, live
pass, blend, loss (spectrum L2 + channel loss on the spatial mean), blend
and projection backward, network backward and fused Adam.  `value` counts
the spectra that go through that step per second.  Also reported:
batched serving (network + render for 64 transmitters per launch sequence)
and the "plain" comparisons (one query at a time with fixed attributes for
serving, one query per step for training).
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402  (seeded synthetic inputs)

# FP32 vector peak without packed-FP32 instructions (the HIP sources are
# compiled with them disabled): 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
PEAK_VALU_F32_TFLOPS = 78.6
PEAK_MFMA_F32_TFLOPS = 157.3  # dense FP32 matrix cores
PEAK_HBM_GBS = 8000.0
# Algorithmic work of the compositing kernels for B attribute sets over one
# shared geometry (the training step):
#  forward  : per set, n_contrib accepted pairs x 2 Fc (out += w v, on the
#             matrix cores); once for all sets, n_eval (pixel, entry)
#             evaluations x FLOPS_PER_EVAL + n_contrib x FLOPS_PER_CONTRIB
#  backward : per set, n_contrib x 4 Fc: gv = v . g (2 Fc) and dL/dv += w g
#             (2 Fc), the two products on the matrix cores; once for all sets
#             (the geometry is shared), the re-walk n_eval x FLOPS_PER_EVAL
#             and n_contrib x FLOPS_BWD_CONTRIB for dalpha, the
#             transmittance/prefix updates and the geometric terms
FLOPS_PER_EVAL = 12.0       # offsets, quadratic form, exp, clamp and tests of one (pixel, entry)
FLOPS_PER_CONTRIB = 4.0     # weight and transmittance update of one accepted pair
FLOPS_BWD_CONTRIB = 22.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=100_000)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--serve-batch", type=int, default=64)
    ap.add_argument("--channels", type=int, default=64)
    ap.add_argument("--H", type=int, default=90)
    ap.add_argument("--W", type=int, default=360)
    ap.add_argument("--tile", type=int, nargs=2, default=(16, 16), metavar=("TH", "TW"),
                    help="tile rows and columns of the training and serving renders")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-mix", action="store_true")
    ap.add_argument("--loss-mode", default="train_pass",
                    choices=("train_pass", "partial", "fused", "target", "two_pass"),
                    help="compositing, loss and backward in one fused pass (train_pass), or as separate passes: "
                         "a one-pass loss writing the elementwise gradient (partial), the same folded into the "
                         "compositing kernel (fused), a loss pass without the gradient, formed in the backward "
                         "from the target (target), or loss + stored gradient (two_pass)")
    ap.add_argument("--mix-only", action="store_true", help="run only the uneven serving mix (for profiling)")
    ap.add_argument("--pmc-run", action="store_true",
                    help="short run for hardware-counter passes: 2 training steps, one serving render, one "
                         "network forward over all n Gaussians, then a 256 MiB copy that calibrates the byte "
                         "counters")
    ap.add_argument("--tune-cache", default=None, help="autotuner cache file (JSON) for the serving mix")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other workloads (plain 2k render, 50k fwd+bwd, 300k training step, N sweep)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path, run it with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2511_22793_amd as gs
    from paper_2511_22793_amd import train

    dev = torch.device("cuda:0")
    if args.mix_only:
        print(json.dumps({"serving_mix": serving_mix(args, gs, dev)}), flush=True)
        return
    n, B, SB, F, H, W = args.n, args.batch, args.serve_batch, args.channels, args.H, args.W
    assert F == train.F, "the attribute network has 64 complex outputs"
    grid = gs.Grid(H, W, args.tile[0], args.tile[1])
    scene = synth.scene(n, seed=synth.SEED_SCENE)
    emb = synth.embeddings(n)
    box_lo, box_hi = list(synth.BOX_LO), list(synth.BOX_HI)
    # ground truth and transmitters
    gt = synth.scene(n, seed=synth.SEED_GT_SCENE)
    rho = synth.uniform(n, 0.0, 1.0, seed=synth.SEED_GT_SCENE + 10)
    tx_all = synth.points(max(B, SB), seed=synth.SEED_QUERIES)
    gt_dev = {k: torch.from_numpy(v).to(dev) for k, v in gt.items()}
    rx1 = torch.zeros(1, 3, device=dev)
    targets = torch.empty(B, F, H, W, 2, device=dev)
    for b in range(B):
        a = torch.from_numpy(synth.ground_truth_attributes(gt, rho, tx_all[b:b + 1])[0]).to(dev)
        out, _ = gs.forward(gt_dev, a, rx1, grid=grid, is_complex=True)
        targets[b] = out[0]
    tx = torch.from_numpy(tx_all[:B]).to(dev)
    # each training sample's channel (Eq. (2) of its target spectrum), formed
    # once with the samples
    target_means = gs.spatial_mean(targets, True)

    if args.pmc_run:
        args.warmup, args.steps = 1, 2
    # ---------------------------------------------------------------- training
    model = train.LearnedScene(scene, emb, train.init_weights(0), [0, 0, 0], B, box_lo, box_hi, grid=grid,
                               total_steps=1000, loss_mode=args.loss_mode)
    for _ in range(args.warmup):
        model.train_step(tx, targets, target_mean=target_means)
    torch.cuda.synchronize()
    if args.loss_mode == "train_pass":
        names = ["start", "prepare", "live", "mlp_fwd", "train_pass", "mlp_bwd", "adam"]
    else:
        names = ["start", "prepare", "live", "mlp_fwd", "blend", "loss", "render_bwd", "mlp_bwd", "adam"]
    evs = [{k: torch.cuda.Event(enable_timing=True) for k in names} for _ in range(args.steps)]
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    L = gs._lib.lib()
    L.gs_timing_enable(1)
    t0.record()
    for k in range(args.steps):
        e = evs[k]
        model.train_step(tx, targets, marks=lambda name, e=e: e[name].record(), target_mean=target_means)
    t1.record()
    torch.cuda.synchronize()
    L.gs_timing_enable(0)
    kernel_ms = {}
    timers = (("train", 2),) if args.loss_mode == "train_pass" else (("blend", 0), ("blend_bwd", 1))
    for name, tid in timers:
        tot, cnt = ctypes.c_double(), ctypes.c_int64()
        assert L.gs_timing_read(tid, ctypes.byref(tot), ctypes.byref(cnt)) == 0 and cnt.value == args.steps
        kernel_ms[name] = tot.value / cnt.value
    ms_step_eager = t0.elapsed_time(t1) / args.steps
    stages = {}
    for a, b in zip(names[:-1], names[1:]):
        stages[b] = float(np.mean([e[a].elapsed_time(e[b]) for e in evs]))
    if args.pmc_run:
        # the counter runs also cover the serving render of the same batch
        # (the shared-geometry forward blend) and one network forward over
        # every Gaussian (all n rows listed), where the matrix cores bind
        from paper_2511_22793_amd import mlp as gmlp
        model.render(tx)
        all_rows = torch.arange(n, dtype=torch.int32, device=dev)
        n_all = torch.full((1,), n, dtype=torch.int32, device=dev)
        gmlp.forward(model.net, model.Z1, model.g["mean"], gmlp.Rows(tx, all_rows, n_all, row_cap=n), model.attr,
                     model.state)
        torch.cuda.synchronize()
        # calibration: a plain device copy of exactly 256 MiB (read 256, write 256)
        src = torch.ones(64 << 20, device=dev)
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"pmc_run": "done", "copy_bytes": src.numel() * 4}), flush=True)
        return
    live_count = int(model.live_count.item())
    HW = H * W
    n_contrib = model.ws.view("n_contrib", 0, HW, torch.int32).double().sum().item()
    n_eval = model.ws.view("n_last", 0, HW, torch.int32).double().sum().item()
    flags = model.ws.flags()[0]
    # the step captured once as a HIP graph: K replays timed as a block (the
    # headline), then REPLAYS replays timed one by one (median, p99); every
    # replay is a whole training step (parameters move each time)
    step_graph = capture(lambda: model.train_step(tx, targets, target_mean=target_means))
    for _ in range(args.warmup):
        step_graph.replay()
    torch.cuda.synchronize()
    t0.record()
    for _ in range(args.steps):
        step_graph.replay()
    t1.record()
    torch.cuda.synchronize()
    ms_step = t0.elapsed_time(t1) / args.steps
    step_each = replay_times(step_graph, REPLAYS)
    assert model.skipped_steps() == 0, "a step overflowed its pair buffer"

    # ---------------------------------------------------------------- serving
    serve = train.LearnedScene(scene, emb, train.init_weights(0), [0, 0, 0], SB, box_lo, box_hi, grid=grid)
    stx = torch.from_numpy(tx_all[:SB]).to(dev)
    for _ in range(args.warmup):
        serve.render(stx)
    torch.cuda.synchronize()
    s0 = torch.cuda.Event(enable_timing=True)
    s1 = torch.cuda.Event(enable_timing=True)
    s0.record()
    for _ in range(args.steps):
        serve.render(stx)
    s1.record()
    torch.cuda.synchronize()
    ms_serve_eager = s0.elapsed_time(s1) / args.steps
    serve_graph = capture(lambda: serve.render(stx))
    serve_each = replay_times(serve_graph, REPLAYS)
    ms_serve = float(np.median(serve_each))

    res = {
        "metric": "hemispherical spectra/s + fwd+bwd steps/s, 100k Gaussians 360x90, vs plain",
        "value": round(B / (ms_step / 1e3), 2),
        "unit": "spectra/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "fwd+bwd training step: %d Gaussians, %dx%d grid, %d complex subcarriers from the "
                               "BF16 attribute network, %d transmitter queries per step, fixed receiver"
                               % (n, H, W, F, B, ),
                   "n_gaussians": n, "grid": [H, W], "tile": list(args.tile), "channels": F, "complex": True,
                   "queries_per_step": B, "network": "32-d embedding + 51-d transmitter encoding -> 64 -> 64 -> 128, "
                                                     "bf16 weights, fp32 accumulation"},
        "fwd_bwd_steps_per_s": round(1e3 / ms_step, 3),
        "timing": {"headline": "the step captured as a HIP graph, %d replays timed as one block" % args.steps,
                   "graph_replays": REPLAYS, "step_median_ms": round(float(np.median(step_each)), 4),
                   "step_p99_ms": round(float(np.percentile(step_each, 99)), 4),
                   "steps_per_s_at_median": round(1e3 / float(np.median(step_each)), 3),
                   "eager_ms_per_step": round(ms_step_eager, 4),
                   "target_channels": "Eq. (2) of each target, formed once with the training samples"},
        "stages_ms": {k: round(v, 4) for k, v in stages.items()},
        "stages_note": "eager steps with events between stages (the graph has no stage marks)",
        "serving": {"spectra_per_s": round(SB / (ms_serve / 1e3), 2), "queries_per_launch_sequence": SB,
                    "ms_per_batch_median": round(ms_serve, 4),
                    "ms_per_batch_p99": round(float(np.percentile(serve_each, 99)), 4), "graph_replays": REPLAYS,
                    "eager_ms_per_batch": round(ms_serve_eager, 4),
                    "includes": "network + prepare + live pass + blend, captured as a HIP graph"},
        "stats": {"n_visible": flags["n_visible"], "n_pairs": flags["n_pairs"], "live_gaussians": live_count,
                  "mean_contrib_per_pixel": round(n_contrib / HW, 2), "entries_evaluated_per_pixel":
                  round(n_eval / HW, 2)},
    }
    # roofline of the dominant kernel, from the library's HIP-event timing of
    # every launch of the two compositing kernels during the timed steps
    Fc = 2 * F
    blend_flops = B * n_contrib * 2.0 * Fc + n_eval * FLOPS_PER_EVAL + n_contrib * FLOPS_PER_CONTRIB
    bwd_flops = B * n_contrib * 4.0 * Fc + n_eval * FLOPS_PER_EVAL + n_contrib * FLOPS_BWD_CONTRIB
    if args.loss_mode == "train_pass":
        # the fused pass: the forward product, GV and dL/dv (three products
        # of 2 Fc flops per set and accepted pair), the walk twice (alpha and
        # weights, then the backward recurrence and geometric terms)
        train_flops = B * n_contrib * 6.0 * Fc + n_eval * FLOPS_PER_EVAL + n_contrib * (FLOPS_PER_CONTRIB +
                                                                                         FLOPS_BWD_CONTRIB)
        kt = {"k_train_fb + k_train_walk": (kernel_ms["train"], train_flops, "mfma", PEAK_MFMA_F32_TFLOPS)}
    else:
        fwd_name = "k_blend<32, true>" if args.loss_mode == "fused" else "k_blend_sg<1>"
        bwd_name = "k_blend_bwd_sg<1, %s>" % ("true" if args.loss_mode == "target" else "false")
        kt = {fwd_name: (kernel_ms["blend"], blend_flops, "mfma", PEAK_MFMA_F32_TFLOPS),
              bwd_name: (kernel_ms["blend_bwd"], bwd_flops, "mfma", PEAK_MFMA_F32_TFLOPS)}
    kname = max(kt, key=lambda k: kt[k][0])
    ms, fl, bound, peak = kt[kname]
    ach = fl / (ms / 1e3) / 1e12
    res["roofline"] = {"kernel": kname, "bound": bound, "achieved": round(ach, 3), "peak": peak,
                       "unit": "TFLOP/s", "frac": round(ach / peak, 4), "traffic": measured_traffic(kname),
                       "launch_ms": round(ms, 4), "flops_per_launch": fl,
                       "work": {"pairs_evaluated_per_set": n_eval, "contributions_per_set": n_contrib, "sets": B,
                                "channel_floats": Fc},
                       "other": {k: {"launch_ms": round(v[0], 4),
                                     "achieved_tflops": round(v[1] / (v[0] / 1e3) / 1e12, 3),
                                     "bound": v[2], "frac": round(v[1] / (v[0] / 1e3) / 1e12 / v[3], 4)}
                                 for k, v in kt.items()}}
    res["confidence"] = confidence_head(gs, dev)
    res["emission"] = emission_nets(gs, dev, args.n, B)
    if not args.no_mix:
        res["serving_mix"] = serving_mix(args, gs, dev)
    if not args.no_plain:
        res["plain"] = plain(args, gs, train, scene, emb, gt, rho, tx_all, grid, targets, target_means, box_lo,
                             box_hi, dev)
        res["plain"]["speedup_training"] = round(res["value"] / res["plain"]["training_spectra_per_s"], 3)
        res["plain"]["speedup_serving"] = round(res["serving"]["spectra_per_s"] / res["plain"]["serving_spectra_per_s"], 3)
    if not args.no_configs:
        res["configs"] = other_configs(args, gs, train, dev)
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(gt, rho, tx_all, H, W, args.cpu_seconds,
                                           gpu_forward=res.get("serving", {}).get("spectra_per_s"))
    print(json.dumps(res), flush=True)


REPLAYS = 100


def capture(fn, warm=2):
    """fn captured into a HIP graph (torch.cuda.CUDAGraph) after `warm`
    eager calls on the capture stream."""
    import torch
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


def replay_times(g, reps):
    """Per-replay times (ms) of `reps` back-to-back replays, HIP events
    around each replay on the replay stream."""
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    torch.cuda.synchronize()
    for a, b in ev:
        a.record()
        g.replay()
        b.record()
    torch.cuda.synchronize()
    return np.array([a.elapsed_time(b) for a, b in ev])


TRAFFIC_PROFILES = [os.path.join(ROOT, "profiles", f) for f in ("fused_train_pass_traffic_100k_90x360_f64c_b16.md",
                                                                  "compositing_traffic_100k_90x360_f64c_b16.md")]


def kernel_source_hash(path):
    """sha256 of a kernel's source file and the shared header it includes."""
    import hashlib
    h = hashlib.sha256()
    for f in (path, os.path.join(ROOT, "paper_2511_22793_amd", "csrc", "common.h")):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, each scaled by a plain copy's reading), or None
    when there is none or the kernel's source changed since it was taken."""
    for path in TRAFFIC_PROFILES:
        if not os.path.exists(path):
            continue
        text = open(path).read()
        start = text.find("```json")
        if start < 0:
            continue
        data = json.loads(text[start + 7:text.index("```", start + 7)])
        k = data.get("kernels", {}).get(kernel)
        if not k:
            continue
        src = os.path.join(ROOT, "paper_2511_22793_amd", "csrc", k["source"])
        if kernel_source_hash(src) != k["source_sha256"]:
            return None
        return k["fetch_bytes_per_launch"] + k["write_bytes_per_launch"]
    return None


# confidence head + Eq. (6) per sample: layer 1 (3x32 FMA), layer 2 (32 FMA),
# the backward through both (32 + 3x32 + 32 + 32 FMA/adds): ~600 flops
CONF_FLOPS_PER_SAMPLE = 2 * (3 * 32 + 32) + 32 + 2 * 3 * 32 + 32 + 2 * 32


def _timed(g, reps):
    t = replay_times(g, reps)
    return {"ms_median": round(float(np.median(t)), 4), "ms_p99": round(float(np.percentile(t, 99)), 4),
            "replays": reps}


def other_configs(args, gs, train, dev):
    """The other workloads of the metric, each captured as a HIP graph and
    replayed (median and p99 per replay):
      plain_2k   2,048 Gaussians, one receiver at the origin, 1 real RSS
                 channel (1/d^2 to the receiver), 90x360: spectra/s;
      fwd_bwd_50k  50,000 Gaussians, 16 receivers uniform in the room, 1
                 real channel: forward, L2 loss to the render of a perturbed
                 scene, backward (scene and attribute gradients): steps/s;
      train_300k the whole training step at 300,000 Gaussians, 180x720, 32
                 complex subcarriers from the attribute network, 64
                 transmitters: steps/s and spectra/s;
      n_sweep    the plain single-query forward (1 real channel, 90x360) at
                 N in {2k, 10k, 30k, 62k, 100k, 200k, 300k}: ms per spectrum."""
    import torch
    out = {}
    reps = REPLAYS
    grid = gs.Grid(90, 360)
    rx0 = torch.zeros(1, 3, device=dev)

    def forward_graph(n, seed):
        sc = {k: torch.from_numpy(v).to(dev) for k, v in synth.scene(n, seed=seed).items()}
        a = torch.from_numpy(synth.rss_attrs(n)).to(dev)
        ws = gs.Workspace(n, 1, grid, gs.Params(forward_only=True), device=dev)
        o = torch.empty(1, 1, 90, 360, device=dev)
        g = capture(lambda: gs.forward(sc, a, rx0, grid=grid, workspace=ws, out=o))
        return g, ws

    g, ws = forward_graph(2048, synth.SEED_SCENE)
    t = _timed(g, reps)
    out["plain_2k"] = dict(workload="plain forward render, 2048 Gaussians, 1 real channel, 90x360, one receiver",
                           spectra_per_s=round(1e3 / t["ms_median"], 1), **t)
    # 50k forward + L2 loss + backward over 16 receivers
    n, B = 50_000, 16
    base = synth.scene(n, seed=synth.SEED_SCENE)
    attr = synth.rss_attrs(n)
    pert = synth.perturbation(n)
    tgt_scene = {k: (base[k] + pert[k]).astype(np.float32) if k in pert else base[k] for k in base}
    tgt_attr = (attr + pert["rng"].normal(0.0, pert["attr_sd"], size=attr.shape)).astype(np.float32)
    rx = torch.from_numpy(synth.points(B, seed=synth.SEED_QUERIES)).to(dev)
    scd = {k: torch.from_numpy(v).to(dev) for k, v in base.items()}
    tsd = {k: torch.from_numpy(v).to(dev) for k, v in tgt_scene.items()}
    a = torch.from_numpy(attr).to(dev)
    target, _ = gs.forward(tsd, torch.from_numpy(tgt_attr).to(dev), rx, grid=grid)
    ws = gs.Workspace(n, B, grid, gs.Params(), device=dev)
    spec = torch.empty(B, 1, 90, 360, device=dev)
    gout = {"d_mean": torch.empty(3, n, device=dev), "d_log_scale": torch.empty(3, n, device=dev),
            "d_quat": torch.empty(4, n, device=dev), "d_opacity_logit": torch.empty(n, device=dev)}
    d_attr = torch.empty_like(a)
    lbuf = {}

    def step50k():
        gs.forward(scd, a, rx, grid=grid, workspace=ws, out=spec)
        lbuf["l"] = gs.loss_spectrum(spec, target, False, 0.0)
        gs.backward(ws, scd, a, rx, spec, lbuf["l"][2], out=gout)
    g = capture(step50k)
    t = _timed(g, reps)
    out["fwd_bwd_50k"] = dict(workload="forward + L2 loss + backward, 50000 Gaussians, 16 receivers, 1 real "
                                       "channel, 90x360", steps_per_s=round(1e3 / t["ms_median"], 2),
                              spectra_per_s=round(B * 1e3 / t["ms_median"], 1), **t)
    del ws, spec, target, gout, d_attr, lbuf
    # the 300k training step at 180x720, 32 subcarriers, 64 transmitters
    n, B, F = 300_000, 64, 32
    grid4 = gs.Grid(180, 720)
    sc4 = synth.scene(n, seed=synth.SEED_SCENE)
    gt = synth.scene(n, seed=synth.SEED_GT_SCENE)
    rho = synth.uniform(n, 0.0, 1.0, seed=synth.SEED_GT_SCENE + 10)
    tx = synth.points(B, seed=synth.SEED_QUERIES)
    gtd = {k: torch.from_numpy(v).to(dev) for k, v in gt.items()}
    targets = torch.empty(B, F, 180, 720, 2, device=dev)
    wsg = gs.Workspace(n, 1, grid4, gs.Params(forward_only=True), device=dev)
    for b in range(B):
        ab = torch.from_numpy(synth.ground_truth_attributes(gt, rho, tx[b:b + 1], nf=F)[0]).to(dev)
        gs.forward(gtd, ab, rx0, grid=grid4, is_complex=True, workspace=wsg, out=targets[b:b + 1])
    del wsg, gtd
    tmeans = gs.spatial_mean(targets, True)
    model = train.LearnedScene(sc4, synth.embeddings(n), train.init_weights(0, n_chan=F), [0, 0, 0], B,
                               list(synth.BOX_LO), list(synth.BOX_HI), grid=grid4, total_steps=1000)
    txd = torch.from_numpy(tx).to(dev)
    g = capture(lambda: model.train_step(txd, targets, target_mean=tmeans))
    t = _timed(g, max(20, reps // 4))
    assert model.skipped_steps() == 0
    live4 = int(model.live_count.item())
    out["train_300k"] = dict(workload="whole training step, 300000 Gaussians, 180x720, 32 complex subcarriers "
                                      "from the attribute network, 64 transmitters, fixed receiver",
                             steps_per_s=round(1e3 / t["ms_median"], 3),
                             spectra_per_s=round(B * 1e3 / t["ms_median"], 1), live_gaussians=live4, **t)
    del model, targets, tmeans
    torch.cuda.empty_cache()
    sweep = {}
    for n in (2_000, 10_000, 30_000, 62_000, 100_000, 200_000, 300_000):
        g, _ = forward_graph(n, synth.SEED_SCENE)
        tt = _timed(g, 50)
        sweep[str(n)] = {"ms_median": tt["ms_median"], "ms_p99": tt["ms_p99"]}
    out["n_sweep"] = {"workload": "plain single-query forward (projection, sort, binning, blend), 1 real channel, "
                                  "90x360, receiver at the floor centre", "ms_per_spectrum": sweep}
    return out


def confidence_head(gs, dev):
    """Time of gs_confidence_loss for one sample per step (the training
    workload's single receiver: one workgroup) and for 65536 and 1M samples
    (the multi-workgroup path with its fixed-order sum), inputs resident on
    the device, HIP events on the launch stream."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(5)
    w = {"W1": torch.randn(32, 3, generator=g) * 0.5, "b1": torch.randn(32, generator=g) * 0.5,
         "w2": torch.randn(32, generator=g) * 0.3, "b2": torch.randn(1, generator=g) * 0.3}
    w = {k: v.to(dev) for k, v in w.items()}
    out = {}
    for n in (1, 65536, 1 << 20):
        x = (torch.randn(n, 3, generator=g) * 2).to(dev)
        L = (torch.rand(n, generator=g) * 0.5 + 0.01).to(dev)
        nb = int(gs._lib.lib().gs_confidence_scratch_bytes(n))
        sc = torch.empty(max(nb, 4) // 4, device=dev) if nb else None
        for _ in range(3):
            gs.confidence_loss(x, L, w, scratch=sc)
        reps = 50
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            gs.confidence_loss(x, L, w, scratch=sc)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        out["n%d_call_us" % n] = round(us, 2)  # per call, host marshalling included
        if n > 1:
            ach = CONF_FLOPS_PER_SAMPLE * n / (us * 1e-6) / 1e12
            out["n%d_samples_per_s" % n] = round(n / (us * 1e-6), 1)
            out["n%d_roofline" % n] = {"bound": "alu", "achieved": round(ach, 5), "peak": PEAK_VALU_F32_TFLOPS,
                                       "unit": "TFLOP/s", "frac": round(ach / PEAK_VALU_F32_TFLOPS, 6)}
    return out


def emission_nets(gs, dev, n, Q):
    """The paper's per-Gaussian 3 -> H -> 2 emission networks at the training
    workload's size (n Gaussians, Q queries) for the widths of the paper's
    ablation (8, 16, 64): forward and backward kernel times from HIP events,
    priced against HBM (parameter-major storage; algorithmic bytes:
    parameters and means read once, attributes written or read once,
    gradients written once)."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(9)
    mean = (torch.rand(3, n, generator=g) * 10 - 5).to(dev)   # the scene's [3][n]
    rx = (torch.rand(Q, 3, generator=g) * 4 - 2).to(dev)
    tx = (torch.rand(Q, 3, generator=g) * 10 - 5).to(dev)
    ds = torch.randn(Q, n, 2, generator=g).to(dev)
    out = {"gaussians": n, "queries": Q, "widths": {}}
    for H in (8, 16, 64):
        P = (torch.randn(6 * H + 2, n, generator=g) * 0.6 * (16 / H) ** 0.5).to(dev)
        per = (6 * H + 2 + 3) * 4
        nbytes = {"forward": n * per + Q * n * 2 * 4, "backward": 2 * n * per + Q * n * 2 * 4}
        row = {}
        for name, fn in (("forward", lambda: gs.emission_forward(P, mean, rx, tx)),
                         ("backward", lambda: gs.emission_backward(P, mean, rx, tx, ds))):
            for _ in range(3):
                fn()
            reps = 20
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / reps
            gbs = nbytes[name] / (us * 1e-6) / 1e9
            row[name] = {"us": round(us, 2), "bytes": nbytes[name],
                         "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS,
                                      "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4)}}
        out["widths"][str(H)] = row
    return out


def serving_mix(args, gs, dev):
    """256 receivers over 8 scenes of uneven size (10k-200k Gaussians), grid
    (90x360 / 180x720) and channel count (1 real, 16 or 64 complex), with
    fixed attributes: autotuned, captured once as a graph and replayed.
    Per-query latency = completion of its spectrum - batch start (device
    clock), over every timed replay; against one gs_render_forward per
    query, back to back."""
    import torch
    import synth
    from paper_2511_22793_amd import serve
    mix = synth.serving_mix()
    jobs = serve.make_jobs(synth.serving_arrays(mix), device=dev)
    t = time.perf_counter()
    tuner = serve.Autotuner(path=args.tune_cache)
    batch = tuner.tune(jobs)
    tune_s = time.perf_counter() - t
    batch.capture()
    for _ in range(args.warmup):
        batch.replay()
    torch.cuda.synchronize()
    lat, spans, preps = [], [], []
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = max(3, min(args.steps, 10))
    total_ms = 0.0
    for _ in range(reps):
        e0.record()
        batch.replay()
        e1.record()
        e1.synchronize()
        total_ms += e0.elapsed_time(e1)
        L = batch.latencies_ms()
        lat.append(L["per_query"])
        spans.append(L["makespan"])
        preps.append(L["prepare"])
    lat = np.concatenate(lat)
    ms_batch = total_ms / reps
    # plain: one forward per query, each on its own scene, back to back
    # (a workspace and an output per scene, reused by its queries in turn)
    singles = []
    for i, j in enumerate(batch.jobs):
        ws = gs.Workspace(j.n, 1, gs.Grid(j.grid.H, j.grid.W), gs.Params(forward_only=True), device=dev)
        o = torch.empty((1,) + tuple(batch.spectra[i].shape[1:]), device=dev)
        for q in range(j.B):
            singles.append((j, j.rx[q:q + 1].contiguous(), ws, o))

    def run_plain():
        for j, rx, ws, o in singles:
            gs.forward(j.scene, j.attr, rx, grid=ws.grid, params=ws.params, is_complex=j.is_complex, workspace=ws,
                       out=o)
    run_plain()
    torch.cuda.synchronize()
    e0.record()
    run_plain()
    e1.record()
    e1.synchronize()
    ms_plain = e0.elapsed_time(e1)
    nq = batch.n_queries
    ws_bytes = sum(w.nbytes for w in batch.workspaces)
    return {"queries": nq, "scenes": [j.signature() for j in batch.jobs],
            "workspace_bytes": ws_bytes, "pair_capacity": [int(j.params.pair_capacity) for j in batch.jobs],
            "tuned": {"block": tuner.choice["block"], "workgroups": tuner.choice.get("workgroups"),
                      "tiles_and_groups": [list(x[1:]) for x in tuner.choice["jobs"]], "tune_s": round(tune_s, 2)},
            "ms_per_batch": round(ms_batch, 4), "makespan_ms_device": round(float(np.mean(spans)), 4),
            "prepare_ms_device": round(float(np.mean(preps)), 4),
            "p50_ms": round(float(np.percentile(lat, 50)), 4), "p99_ms": round(float(np.percentile(lat, 99)), 4),
            "queries_per_s": round(nq / (ms_batch / 1e3), 2), "replays": reps,
            "plain_ms_per_batch": round(ms_plain, 4), "plain_queries_per_s": round(nq / (ms_plain / 1e3), 2),
            "speedup_vs_plain": round(ms_plain / ms_batch, 3)}


def plain(args, gs, train, scene, emb, gt, rho, tx_all, grid, targets, target_means, box_lo, box_hi, dev):
    """One query at a time: fixed-attribute forward per query (serving) and a
    one-query training step (training), same shapes."""
    import torch
    n, B, SB = args.n, args.batch, args.serve_batch
    sc = {k: torch.from_numpy(v).to(dev) for k, v in scene.items()}
    rx1 = torch.zeros(1, 3, device=dev)
    attrs = [torch.from_numpy(synth.ground_truth_attributes(gt, rho, tx_all[b:b + 1])[0]).to(dev) for b in range(4)]
    ws = gs.Workspace(n, 1, grid, gs.Params(), device=dev)
    out = torch.empty(1, train.F, grid.H, grid.W, 2, device=dev)
    for a in attrs:
        gs.forward(sc, a, rx1, grid=grid, is_complex=True, workspace=ws, out=out)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for q in range(SB):
        gs.forward(sc, attrs[q % 4], rx1, grid=grid, is_complex=True, workspace=ws, out=out)
    e1.record()
    torch.cuda.synchronize()
    serve_ms = e0.elapsed_time(e1) / SB
    one = train.LearnedScene(scene, emb, train.init_weights(0), [0, 0, 0], 1, box_lo, box_hi, grid=grid,
                             loss_mode=args.loss_mode)
    tx = torch.from_numpy(tx_all[:B]).to(dev)
    tgt1 = [targets[b:b + 1].contiguous() for b in range(B)]
    tm1 = [target_means[b:b + 1].contiguous() for b in range(B)]
    for b in range(2):
        one.train_step(tx[b:b + 1].contiguous(), tgt1[b], target_mean=tm1[b])
    torch.cuda.synchronize()
    e0.record()
    for b in range(B):
        one.train_step(tx[b:b + 1].contiguous(), tgt1[b], target_mean=tm1[b])
    e1.record()
    torch.cuda.synchronize()
    train_ms = e0.elapsed_time(e1) / B
    return {"serving_spectra_per_s": round(1e3 / serve_ms, 2), "training_spectra_per_s": round(1e3 / train_ms, 2),
            "serving": "one gs_render_forward per query, fixed attributes",
            "training": "one-query training steps, same stages"}


def cpu_baseline(gt, rho, tx_all, H, W, seconds, gpu_forward=None):
    """The FP64 oracle on the host cores: full spectra (64 complex
    subcarriers, fixed attributes) of the same scene size, as many queries
    as fit in `seconds`, with every host thread; then the same at one thread
    and at T_min = 0 (every walk to the end of its list), a third of the time
    each.  The oracle renders forward only (it has no batched backward), so
    the headline's training unit has no oracle counterpart: the forward-only
    GPU rate of the same workload (`gpu_forward`, spectra/s) stands beside
    it, with the ratio."""
    import oracle
    threads = min(os.cpu_count() or 1, 64)

    # the inputs (attributes for a few transmitters) are formed outside the
    # timed region
    attrs = [synth.ground_truth_attributes(gt, rho, tx_all[i:i + 1])[0] for i in range(min(4, len(tx_all)))]

    def run(nthreads, budget, prm=None, stride=1):
        # stride > 1: the per-pixel compositing over every stride-th pixel
        # only, its time scaled by stride (the work per pixel is the same);
        # projection and depth order run in full and count once
        pix = None if stride == 1 else np.arange(0, H * W, stride, dtype=np.int32)
        t_all = 0.0  # estimated time of k whole spectra
        k = 0
        start = time.perf_counter()
        while True:
            attr = attrs[k % len(attrs)]
            t0 = time.perf_counter()
            proj = oracle.project(gt, [0, 0, 0], H, W, prm)
            order = oracle.depth_order(proj)
            t1 = time.perf_counter()
            oracle.composite(proj, order, attr, H, W, prm, pixels=pix, nthreads=nthreads)
            t2 = time.perf_counter()
            t_all += (t1 - t0) + (t2 - t1) * stride
            k += 1
            if time.perf_counter() - start >= budget and k >= 2:
                break
        return k, t_all

    k, dt = run(threads, seconds)
    out = {"value": round(k / dt, 4), "unit": "spectra/s", "cores": threads, "kind": "oracle",
           "sample": "%d full %dx%d forward spectra (64 complex subcarriers, fixed attributes) of a %d-Gaussian "
                     "scene (projection, depth order, compositing; attributes formed beforehand); the oracle "
                     "has no batched backward" % (k, H, W, gt["opacity_logit"].shape[0])}
    k1, dt1 = run(1, seconds / 3.0, stride=16)
    out["one_thread"] = {"value": round(k1 / dt1, 4), "unit": "spectra/s", "cores": 1,
                         "sample": "%d spectra, compositing timed at every 16th pixel and scaled" % k1}
    k0, dt0 = run(threads, seconds / 3.0, prm=oracle.params(T_min=0.0), stride=64)
    out["t_min_0"] = {"value": round(k0 / dt0, 4), "unit": "spectra/s", "cores": threads,
                      "sample": "%d spectra with T_min = 0 (every walk to the end of its list), compositing "
                                "timed at every 64th pixel and scaled" % k0}
    if gpu_forward:
        out["gpu_forward_same_workload"] = {"value": gpu_forward, "unit": "spectra/s",
                                            "ratio_to_oracle": round(gpu_forward / out["value"], 1),
                                            "what": "the serving forward (network + prepare + live + blend) of "
                                                    "the same scene and grid, per spectrum"}
    return out


if __name__ == "__main__":
    main()
