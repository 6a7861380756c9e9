"""Training step of the learned-attribute renderer (Algorithm 1's loop with a
shared attribute network, a fixed receiver and a batch of transmitters).

One step, all on the device with no host synchronisation:
  prepare (projection, depth sort, tile binning) for the receiver
  live pass: Gaussians that reach some pixel (and their weight sums)
  network forward for (transmitter, live Gaussian) rows -> attributes
  the fused training pass over the shared geometry: blend of the batch's
  attribute sets, loss (spectrum L2 + Eq. (4) on the Eq. (2) mean) and the
  blend + projection backward -> Gaussian-parameter and attribute gradients
  (other loss modes run blend, loss and backward as separate passes)
  network backward -> weight, bias and embedding gradients
  fused Adam over every parameter group (Table 2 learning rates; the
  position rate decays exponentially)
Optionally (confidence=True) the confidence-weighted objective of Eq. (6):
the head's C for the receiver scales every gradient of the pass, and the
head itself trains on the step's task losses.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import confidence as gc
from . import densify as gd
from . import mlp as gm
from .render import (Grid, Params, TrainScratch, Workspace, backward, backward_l2, blend, blend_loss, live,
                     loss_spectrum, loss_stats, prepare, spatial_mean, train_geometry, train_pass)

F = gm.F


@dataclass
class Rates:
    position: float = 1.6e-4
    position_final: float = 1.6e-7
    opacity: float = 0.0055
    scaling: float = 0.005
    rotation: float = 0.001
    mlp: float = 0.005
    embedding: float = 0.005


def init_weights(seed: int = 0, n_chan: int = F) -> dict:
    """He-normal initial weights in [out, in] layout (W1 [64, 96] with zero
    columns beyond the 83 inputs, W3 [2 n_chan, 64]), zero biases."""
    rng = np.random.default_rng(seed)
    fan1 = gm.EMB + gm.ENC
    W1 = np.zeros((gm.HID, gm.IN_PAD))
    W1[:, :fan1] = rng.normal(0, np.sqrt(2.0 / fan1), size=(gm.HID, fan1))
    return {"W1": W1, "b1": np.zeros(gm.HID),
            "W2": rng.normal(0, np.sqrt(2.0 / gm.HID), size=(gm.HID, gm.HID)), "b2": np.zeros(gm.HID),
            "W3": rng.normal(0, np.sqrt(2.0 / gm.HID), size=(2 * n_chan, gm.HID)), "b3": np.zeros(2 * n_chan)}


class LearnedScene:
    """Gaussian geometry, per-Gaussian embeddings and the attribute network,
    with Adam state, for batches of `batch` transmitters seen from `rx`."""

    def __init__(self, scene: dict, embeddings: np.ndarray, weights: dict, rx, batch: int, box_lo, box_hi,
                 grid: Grid = Grid(), params: Params = Params(), rates: Rates = Rates(), total_steps: int = 1000,
                 train_geometry: bool = True, lambda_ch: float = 1.0, loss_mode: str = "train_pass",
                 keep_spectra: bool = False, confidence: bool = False, conf_alpha: float = gc.ALPHA,
                 conf_weights: dict = None, densify_stats: bool = False, device="cuda"):
        dev = torch.device(device)
        self.dev, self.grid, self.params, self.rates = dev, grid, params, rates
        self._side = None  # second stream of the step (created on first use)
        self.B, self.total_steps, self.train_geometry, self.lambda_ch = batch, total_steps, train_geometry, lambda_ch
        if loss_mode not in ("train_pass", "fused", "partial", "target", "two_pass"):
            raise ValueError("loss_mode is 'train_pass', 'fused', 'partial', 'target' or 'two_pass'")
        self.loss_mode = loss_mode
        if confidence and loss_mode != "train_pass":
            raise ValueError("the confidence-weighted objective (Eq. (6)) runs with loss_mode 'train_pass'")
        # train_pass: also store the step's spectra in self.spec (the other
        # modes always do)
        self.keep_spectra = keep_spectra
        self.g = {k: torch.tensor(np.asarray(v, np.float32), device=dev) for k, v in scene.items()}
        self.E = torch.tensor(np.asarray(embeddings, np.float32), device=dev)
        self.E_bf = torch.from_numpy(gm.bf16_bits(embeddings).view(np.int16)).to(dev)
        self.net = gm.AttributeNet(weights, box_lo, box_hi, params.r_near, device=dev)
        self.F = F = self.net.F
        self.rx = torch.tensor(np.asarray(rx, np.float32).reshape(1, 3), device=dev)
        self.spec = torch.empty(batch, F, grid.H, grid.W, 2, device=dev)
        self.dpart = torch.empty_like(self.spec) if loss_mode in ("partial", "fused") else None
        self.loss = torch.empty(batch, device=dev)
        self.h_hat = torch.empty(batch, F, 2, device=dev)
        self.tscratch = TrainScratch(batch, F, grid, device=dev) if loss_mode == "train_pass" else None
        # Algorithm 1's per-Gaussian positional-gradient statistics (for densify())
        self.densify_stats = densify_stats
        self._size_buffers(scene["opacity_logit"].shape[0])
        self.mgrads = None
        self.moments = {}
        self.step_count = 0
        # steps whose pair buffer overflowed: their spectra and gradients are
        # undefined, so Adam skips them (guarded on the device) and counts them
        self.skipped = torch.zeros(1, dtype=torch.int32, device=dev)
        # completed steps, on the device: Adam reads its step number and the
        # position rate's schedule from it (so a captured step replays)
        self.step_dev = torch.zeros(1, dtype=torch.int32, device=dev)
        # Eq. (6): the confidence head C = 1 + exp(g(x_rx)) on the receiver;
        # every set of the batch is one sample with the shared receiver, so C
        # is one number per step and scales every task-loss gradient
        self.confidence, self.conf_alpha = confidence, conf_alpha
        if confidence:
            w = conf_weights if conf_weights is not None else gc.init_weights(0, device=dev)
            self.conf_w = {k: v.to(dev, torch.float32).contiguous().clone() for k, v in w.items()}
            self.conf_x = self.rx.expand(batch, 3).contiguous()
            self.conf_zero = torch.zeros(batch, device=dev)
            self.conf_c = torch.empty(batch, device=dev)
            self.conf_loss = torch.empty(batch, device=dev)
            self.conf_grads = {k: torch.empty_like(v) for k, v in self.conf_w.items()}

    def _size_buffers(self, n: int):
        """Every buffer whose size is the Gaussian count."""
        dev, B, F = self.dev, self.B, self.F
        self.n = n
        self.ws = Workspace(n, 1, self.grid, self.params, device=dev)
        # attribute rows never written stay zero (the blend multiplies them by 0)
        self.attr = torch.zeros(B, n, F, 2, device=dev)
        self.d_attr = torch.zeros(B, n, F, 2, device=dev)
        self.live_list = torch.empty(1, n, dtype=torch.int32, device=dev)
        self.live_count = torch.empty(1, dtype=torch.int32, device=dev)
        # 64 split-K workgroups for the weight gradients: the live rows are few
        # (a few hundred per set), so more workgroups shorten each one's chain
        self.state = gm.State(B, n, training=True, device=dev, n_chan=F, n_partial=64)
        self.Z1 = torch.empty(n, gm.HID, device=dev)
        self.ggrads = {"d_mean": torch.empty(3, n, device=dev), "d_log_scale": torch.empty(3, n, device=dev),
                       "d_quat": torch.empty(4, n, device=dev), "d_opacity_logit": torch.empty(n, device=dev)}
        self.grad_acc = torch.zeros(n, device=dev) if self.densify_stats else None
        self.grad_cnt = torch.zeros(n, dtype=torch.int32, device=dev) if self.densify_stats else None

    def densify(self, prm: "gd.DensifyParams" = None, seed: int = 0) -> int:
        """Algorithm 1's densify branch on the statistics gathered since the
        last call: clone / split / prune (gd.plan) into a new Gaussian set;
        the scene, the embeddings (and their BF16 copy) follow, Adam moments
        of kept Gaussians follow and those of new ones start at zero, every
        per-Gaussian buffer is rebuilt and the statistics restart.  Child
        positions draw standard normals from a seeded generator.  Returns the
        new count (one synchronisation; a captured step must be captured
        again afterwards)."""
        if not self.densify_stats:
            raise ValueError("densify() needs LearnedScene(densify_stats=True)")
        prm = prm or gd.DensifyParams()
        n = self.n
        # the screen radius from the last prepare of the receiver
        radius = gd.screen_radius(self.ws, 0)
        src, kind, n_out = gd.plan(self.g, self.grad_acc, self.grad_cnt, radius, prm)
        gen = torch.Generator(device="cpu").manual_seed(seed)
        xi = torch.randn(n, prm.split_n, 3, generator=gen).to(self.dev)
        self.g = gd.apply(self.g, src, kind, n_out, xi, prm.split_n)
        self.E = gd.gather(self.E, src, kind, n, n_out, 1, zero_new=False)
        self.E_bf = gd.gather(self.E_bf, src, kind, n, n_out, 1, zero_new=False)
        comps = {"mean": 3, "log_scale": 3, "quat": 4, "opacity_logit": 1, "E": 1}
        for k, c in comps.items():
            if k in self.moments:
                m, v = self.moments[k]
                self.moments[k] = (gd.gather(m, src, kind, n, n_out, c, zero_new=True),
                                   gd.gather(v, src, kind, n, n_out, c, zero_new=True))
        self._size_buffers(n_out)
        self.mgrads = None  # (the embedding gradient has a row per Gaussian)
        return n_out

    def opacity_reset(self, cap: float = 0.01):
        """sigma <- min(sigma, cap) for every Gaussian (Algorithm 1)."""
        gd.opacity_reset(self.g["opacity_logit"], cap)

    def _rows(self, tx):
        return gm.Rows(tx, self.live_list[0], self.live_count, row_cap=self.n)

    def render(self, tx: torch.Tensor, keep: bool = False) -> torch.Tensor:
        """Spectra [B, F, H, W, 2] for transmitters tx [B, 3] (B = batch)."""
        sc = self.g
        prepare(sc, self.rx, grid=self.grid, params=self.params, workspace=self.ws)
        live(self.ws, self.live_list, self.live_count)
        # (one stream here: the second stream of train_step measured slower
        # for this shorter sequence)
        gm.embed(self.net, self.E_bf, self.Z1)
        gm.forward(self.net, self.Z1, sc["mean"], self._rows(tx), self.attr, self.state)
        blend(self.ws, self.attr, n_sets=self.B, is_complex=True, out=self.spec)
        return self.spec

    def _embed_beside(self) -> torch.cuda.Stream:
        """Enqueues Z1 = E W1e^T (all rows; it depends on neither the
        geometry nor the transmitters) on a second stream, forked from the
        current one, so that it runs beside the prepare and live passes;
        returns the current stream, which must wait for the second before
        the network forward."""
        main = torch.cuda.current_stream(self.dev)
        if self._side is None:
            self._side = torch.cuda.Stream(self.dev)
        self._side.wait_stream(main)
        with torch.cuda.stream(self._side):
            gm.embed(self.net, self.E_bf, self.Z1)
        return main

    def _moment(self, key, like):
        if key not in self.moments:
            self.moments[key] = (torch.zeros_like(like), torch.zeros_like(like))
        return self.moments[key]

    def train_step(self, tx: torch.Tensor, target: torch.Tensor, marks=None,
                   target_mean: torch.Tensor = None) -> torch.Tensor:
        """One step on transmitters tx [B,3] with target spectra [B,F,H,W,2];
        returns the per-set losses (device tensor, before the update).
        marks: optional callable(name) invoked between stages (timing).
        target_mean: the targets' channels (Eq. (2) of each target, [B,F,2]),
        a property of the training samples; formed here when not given."""
        mark = marks or (lambda name: None)
        sc = self.g
        geo_side = False
        mark("start")
        main = self._embed_beside()
        prepare(sc, self.rx, grid=self.grid, params=self.params, workspace=self.ws)
        mark("prepare")
        live(self.ws, self.live_list, self.live_count)
        mark("live")
        main.wait_stream(self._side)
        gm.forward(self.net, self.Z1, sc["mean"], self._rows(tx), self.attr, self.state)
        mark("mlp_fwd")
        if self.loss_mode == "train_pass":
            # compositing, loss and backward in one fused pass (no spectra
            # or spectrum gradients in memory)
            if target_mean is None:
                target_mean = spatial_mean(target, True)
            scale = None
            if self.confidence:
                # C first (it does not depend on the task loss): it scales the
                # pass's gradients
                gc.confidence_loss(self.conf_x, self.conf_zero, self.conf_w, self.conf_alpha,
                                   out=(self.conf_c, self.conf_loss, self.conf_grads))
                scale = self.conf_c[:1]
            loss, _, _, _ = train_pass(self.ws, sc, self.attr, self.rx, self.live_list[0], self.live_count, target,
                                       target_mean, self.lambda_ch, spectrum=self.spec,
                                       write_spectrum=self.keep_spectra, d_attr=self.d_attr, out=self.ggrads,
                                       scratch=self.tscratch, loss=self.loss, h_hat=self.h_hat, grad_scale=scale,
                                       defer_geometry=True)
            # the scene gradients (per-pair fold, projection backward) on the
            # second stream, beside the network backward below
            self._side.wait_stream(main)
            with torch.cuda.stream(self._side):
                train_geometry(self.ws, sc, self.rx, self.ggrads)
            geo_side = True
            if self.confidence:
                # Eq. (6) per sample with the step's task losses: the
                # confidence-weighted loss and the head's gradients (of the
                # batch sum; Adam does not see the constant factor)
                gc.confidence_loss(self.conf_x, self.loss, self.conf_w, self.conf_alpha,
                                   out=(self.conf_c, self.conf_loss, self.conf_grads))
            mark("train_pass")
        elif self.loss_mode == "fused":
            # the loss pass folded into the compositing kernel's output stage:
            # loss, channel means and the elementwise gradient part written
            # as the spectrum is written; the backward adds the channel-mean
            # term
            spec, loss, _, mgrad, scale = blend_loss(self.ws, self.attr, target, self.lambda_ch, n_sets=self.B,
                                                     is_complex=True, out=self.spec, partial=self.dpart)
            mark("blend")
            mark("loss")
            backward_l2(self.ws, sc, self.attr, self.rx, spec, None, mgrad, scale, partial=self.dpart,
                        is_complex=True, n_sets=self.B, d_attr=self.d_attr, out=self.ggrads)
        else:
            spec = blend(self.ws, self.attr, n_sets=self.B, is_complex=True, out=self.spec)
            mark("blend")
            if self.loss_mode == "partial":
                # one pass over (spectrum, target): loss, channel means and
                # the elementwise gradient; the backward adds the
                # channel-mean term
                loss, _, mgrad, scale = loss_stats(spec, target, True, self.lambda_ch, partial=self.dpart)
                mark("loss")
                backward_l2(self.ws, sc, self.attr, self.rx, spec, None, mgrad, scale, partial=self.dpart,
                            is_complex=True, n_sets=self.B, d_attr=self.d_attr, out=self.ggrads)
            elif self.loss_mode == "target":
                # the backward forms the elementwise part from (spec, target)
                loss, _, mgrad, scale = loss_stats(spec, target, True, self.lambda_ch)
                mark("loss")
                backward_l2(self.ws, sc, self.attr, self.rx, spec, target, mgrad, scale, is_complex=True,
                            n_sets=self.B, d_attr=self.d_attr, out=self.ggrads)
            else:
                loss, _, dspec = loss_spectrum(spec, target, True, self.lambda_ch)
                mark("loss")
                backward(self.ws, sc, self.attr, self.rx, spec, dspec, is_complex=True, n_sets=self.B,
                         d_attr=self.d_attr, out=self.ggrads)
        if self.loss_mode != "train_pass":
            mark("render_bwd")
        self.mgrads = gm.backward(self.net, self.E_bf, sc["mean"], self._rows(tx), self.d_attr, self.state,
                                  self.mgrads, clear_d_attr=True)
        if geo_side:
            main.wait_stream(self._side)  # the scene gradients
        if self.densify_stats:
            gd.stats(self.ggrads["d_mean"], self.live_list[0], self.live_count, self.grad_acc, self.grad_cnt)
        mark("mlp_bwd")
        self.step_count += 1
        r = self.rates
        segs, final = [], []
        for k, lr, sh in (("W1", r.mlp, self.net.bf["W1"]), ("b1", r.mlp, None), ("W2", r.mlp, self.net.bf["W2"]),
                          ("b2", r.mlp, None), ("W3", r.mlp, self.net.bf["W3"]), ("b3", r.mlp, None)):
            m, v = self._moment(k, self.net.w[k])
            segs.append((self.net.w[k], self.mgrads[k], m, v, sh, lr))
            final.append(lr)
        m, v = self._moment("E", self.E)
        segs.append((self.E, self.mgrads["E"], m, v, self.E_bf, r.embedding))
        final.append(r.embedding)
        if self.confidence:
            for k in ("W1", "b1", "w2", "b2"):
                m, v = self._moment("conf_" + k, self.conf_w[k])
                segs.append((self.conf_w[k], self.conf_grads[k], m, v, None, r.mlp))
                final.append(r.mlp)
        if self.train_geometry:
            for k, lr, lr1 in (("mean", r.position, r.position_final), ("log_scale", r.scaling, r.scaling),
                               ("quat", r.rotation, r.rotation), ("opacity_logit", r.opacity, r.opacity)):
                m, v = self._moment(k, sc[k])
                segs.append((sc[k], self.ggrads["d_" + k], m, v, None, lr))
                final.append(lr1)
        gm.adam_step_scheduled(segs, final, self.total_steps, self.step_dev, skip_if=self.ws.overflow_word(0),
                               skip_count=self.skipped)
        mark("adam")
        return loss

    def skipped_steps(self) -> int:
        """Steps left out because the render's pair buffer overflowed
        (synchronises).  A caller that sees a non-zero count raises the
        pair capacity (Params.pair_capacity) and rebuilds the scene."""
        return int(self.skipped.item())


class FixedAttributeScene:
    """The comparison without the network: one learned complex attribute
    vector per Gaussian, shared by every transmitter (geometry fixed)."""

    def __init__(self, scene: dict, rx, batch: int, grid: Grid = Grid(), params: Params = Params(), lr: float = 0.005,
                 lambda_ch: float = 1.0, device="cuda"):
        dev = torch.device(device)
        self.dev, self.grid, self.params, self.lr, self.B, self.lambda_ch = dev, grid, params, lr, batch, lambda_ch
        self.n = n = scene["opacity_logit"].shape[0]
        self.g = {k: torch.tensor(np.asarray(v, np.float32), device=dev) for k, v in scene.items()}
        self.rx = torch.tensor(np.asarray(rx, np.float32).reshape(1, 3), device=dev)
        self.attr = torch.zeros(n, F, 2, device=dev)
        self.m = torch.zeros_like(self.attr)
        self.v = torch.zeros_like(self.attr)
        self.ws = Workspace(n, 1, grid, params, device=dev)
        self.spec = torch.empty(batch, F, grid.H, grid.W, 2, device=dev)
        self.step_count = 0
        self.skipped = torch.zeros(1, dtype=torch.int32, device=dev)

    def render(self, tx=None) -> torch.Tensor:
        prepare(self.g, self.rx, grid=self.grid, params=self.params, workspace=self.ws)
        # one attribute set (stride 0) blended B times
        return blend(self.ws, self.attr, n_sets=self.B, is_complex=True, out=self.spec)

    def train_step(self, tx, target) -> torch.Tensor:
        spec = self.render()
        loss, _, dspec = loss_spectrum(spec, target, True, self.lambda_ch)
        # shared attributes: the backward sums the attribute gradient over sets
        g = backward(self.ws, self.g, self.attr, self.rx, spec, dspec, is_complex=True, n_sets=self.B)
        self.step_count += 1
        gm.adam_step([(self.attr, g["d_attr"], self.m, self.v, None, self.lr)], self.step_count,
                     skip_if=self.ws.overflow_word(0), skip_count=self.skipped)
        return loss
