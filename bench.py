"""Benchmark of the hemispherical splatting hot path on one MI355X.

Workload (default): 100,000 Gaussians (means U([-5,5]x[-5,5]x[0,3]) m,
log-scales N(-1.5,0.5), uniform unit quaternions, opacity logits N(0,1)),
receiver at the origin, 90 x 360 grid (1 degree), 16 x 16 tiles, 64
complex subcarriers per Gaussian, B = 64 transmitter queries per step.
The receiver is fixed, so one prepared geometry (projection, depth sort,
tile lists) serves every query; each query has its own attribute set
(random stand-ins for per-transmitter emissions).

A step renders B spectra: prepare once + blend B attribute sets.  The
"plain" comparison renders the same B spectra with one full forward call
per query (projection, sort, binning and blend each time).

Prints one JSON line; see the README section in the design doc for the fields.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# FP32 vector peak without packed-FP32 instructions (disabled in this build):
# 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
PEAK_VALU_F32_TFLOPS = 78.6
FLOPS_PER_EVAL = 12.0      # offsets, quadratic form, exp, clamp and tests per evaluated pair
FLOPS_PER_CONTRIB = 4.0    # weight and transmittance update per accepted pair


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=100_000)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--channels", type=int, default=64)
    ap.add_argument("--H", type=int, default=90)
    ap.add_argument("--W", type=int, default=360)
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-queries", type=int, default=2)
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (see DESIGN.md, sharding)",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2511_22793_amd as gs
    import synth

    dev = torch.device("cuda:0")
    n, B, F, H, W = args.n, args.batch, args.channels, args.H, args.W
    sc_np = synth.scene(n, seed=synth.SEED_SCENE)
    scene = {k: torch.from_numpy(v).to(dev) for k, v in sc_np.items()}
    rx = torch.zeros(B, 3, dtype=torch.float32, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(1234)
    attr = 0.5 * torch.randn(B, n, F, 2, generator=gen, device=dev, dtype=torch.float32)
    grid = gs.Grid(H, W)
    prm = gs.Params()
    out = torch.empty(B, F, H, W, 2, dtype=torch.float32, device=dev)
    ws = gs.prepare(scene, rx[:1], grid=grid, params=prm)

    def step(ev=None):
        gs.prepare(scene, rx[:1], grid=grid, params=prm, workspace=ws)
        if ev is not None:
            ev[0].record()
        gs.blend(ws, attr, n_sets=B, is_complex=True, out=out)
        if ev is not None:
            ev[1].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    flags = ws.flags()[0]
    assert flags["overflow"] == 0
    blend_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                for _ in range(args.steps)]
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record()
    for k in range(args.steps):
        step(blend_ev[k])
    t1.record()
    torch.cuda.synchronize()
    total_ms = t0.elapsed_time(t1)
    ms_per_step = total_ms / args.steps
    blend_ms = float(np.mean([a.elapsed_time(b) for a, b in blend_ev]))
    spectra_per_s = B / (ms_per_step / 1e3)

    # plain: one full forward per query
    plain_ws = gs.Workspace(n, 1, grid, prm)
    plain_out = torch.empty(1, F, H, W, 2, dtype=torch.float32, device=dev)

    def plain_step():
        for b in range(B):
            gs.forward(scene, attr[b], rx[b:b + 1], grid=grid, params=prm, is_complex=True, workspace=plain_ws,
                       out=plain_out)

    plain_step()
    torch.cuda.synchronize()
    p0 = torch.cuda.Event(enable_timing=True)
    p1 = torch.cuda.Event(enable_timing=True)
    p0.record()
    for _ in range(args.plain_steps):
        plain_step()
    p1.record()
    torch.cuda.synchronize()
    plain_ms = p0.elapsed_time(p1) / args.plain_steps
    plain_spectra_per_s = B / (plain_ms / 1e3)

    # algorithmic work of one blend launch (B attribute sets over one geometry)
    HW = H * W
    n_contrib = ws.view("n_contrib", 0, HW, torch.int32).double().sum().item()
    n_eval = ws.view("n_last", 0, HW, torch.int32).double().sum().item()
    Fc = 2 * F
    flops = B * (n_eval * FLOPS_PER_EVAL + n_contrib * (2.0 * Fc + FLOPS_PER_CONTRIB))
    achieved = flops / (blend_ms / 1e3) / 1e12

    res = {
        "metric": "hemispherical spectra/s + fwd+bwd steps/s, 100k Gaussians 360x90, vs plain",
        "value": round(spectra_per_s, 2),
        "unit": "spectra/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "render %d Gaussians, %dx%d grid, %d complex channels, %d transmitter queries per "
                               "step sharing one receiver" % (n, H, W, F, B),
                   "n_gaussians": n, "grid": [H, W], "tile": [16, 16], "channels": F, "complex": True,
                   "queries_per_step": B, "attributes": "fixed per query (random stand-ins)"},
        "plain": {"spectra_per_s": round(plain_spectra_per_s, 2), "ms_per_batch": round(plain_ms, 4),
                  "speedup_batched_vs_plain": round(spectra_per_s / plain_spectra_per_s, 3)},
        "roofline": {"kernel": "k_blend<32>", "bound": "alu", "achieved": round(achieved, 3),
                     "peak": PEAK_VALU_F32_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / PEAK_VALU_F32_TFLOPS, 4),
                     "traffic": None, "launch_ms": round(blend_ms, 4),
                     "work": {"pairs_evaluated": n_eval, "contributions": n_contrib, "sets": B}},
        "stats": {"n_visible": flags["n_visible"], "n_pairs": flags["n_pairs"],
                  "mean_contrib_per_pixel": round(n_contrib / HW, 2), "prepare_ms": round(ms_per_step - blend_ms, 4)},
    }
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(sc_np, F, H, W, args.cpu_queries)
    print(json.dumps(res), flush=True)


def cpu_baseline(sc_np, F, H, W, nq):
    """The FP64 oracle on the host cores: full spectra of `nq` queries of the
    same workload (one receiver, F complex channels)."""
    import oracle
    import synth
    rng = np.random.default_rng(99)
    n = sc_np["opacity_logit"].shape[0]
    threads = min(os.cpu_count() or 1, 64)
    t = time.perf_counter()
    for q in range(nq):
        attr = (0.5 * rng.standard_normal((n, F, 2))).astype(np.float32)
        oracle.render(sc_np, attr, [0, 0, 0], H, W, nthreads=threads)
    dt = time.perf_counter() - t
    return {"value": round(nq / dt, 4), "unit": "spectra/s", "cores": threads, "kind": "oracle",
            "sample": "%d full %dx%d spectra of the same workload (%d complex channels)" % (nq, H, W, F)}


if __name__ == "__main__":
    main()
