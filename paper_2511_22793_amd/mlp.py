"""Python binding of the attribute network and the fused Adam step
(argument marshalling around gs_mlp_* and gs_adam_step)."""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from ._lib import GsAdamSegment, GsMlp, GsMlpGrads, GsMlpRows, GsMlpState, check, lib

EMB, ENC, IN_PAD, HID, F = 32, 51, 96, 64, 64
WEIGHTS = ("W1", "b1", "W2", "b2", "W3", "b3")
BF16_WEIGHTS = ("W1", "W2", "W3")


def bf16_bits(x: np.ndarray) -> np.ndarray:
    """Host-side round-to-nearest-even float -> bfloat16 bit patterns (uint16),
    for loading initial weights and embeddings."""
    x32 = np.ascontiguousarray(x, dtype=np.float32)
    b = x32.view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16).astype(np.uint16)
    nan = np.isnan(x32)
    r[nan] = ((x32.view(np.uint32)[nan] >> 16) | 0x40).astype(np.uint16)
    return r


def _p(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class AttributeNet:
    """FP32 master weights, their BF16 copies on the device and the encoding
    box.  weights: dict of numpy arrays in [out, in] layout."""

    def __init__(self, weights: dict, box_lo, box_hi, r_near: float = 0.2, device="cuda"):
        self.device = torch.device(device)
        self.w = {k: torch.tensor(np.asarray(weights[k], np.float32), device=self.device) for k in WEIGHTS}
        self.bf = {k: torch.from_numpy(bf16_bits(weights[k]).view(np.int16)).to(self.device) for k in BF16_WEIGHTS}
        self.box_lo, self.box_hi, self.r_near = list(box_lo), list(box_hi), float(r_near)
        # subcarriers: W3 has 2F rows (F amplitudes, F phases), F in {32, 64}
        self.F = int(self.w["W3"].shape[0]) // 2
        if self.F not in (32, 64) or tuple(self.w["W3"].shape) != (2 * self.F, HID):
            raise ValueError("W3 must be [2F, 64] with F = 32 or 64")

    def c(self) -> GsMlp:
        m = GsMlp()
        m.W1, m.b1 = _p(self.bf["W1"]), _p(self.w["b1"])
        m.W2, m.b2 = _p(self.bf["W2"]), _p(self.w["b2"])
        m.W3, m.b3 = _p(self.bf["W3"]), _p(self.w["b3"])
        for k in range(3):
            m.box_lo[k], m.box_hi[k] = self.box_lo[k], self.box_hi[k]
        m.r_near = self.r_near
        m.n_chan = self.F
        return m


class Rows:
    """Rows (set, Gaussian): list [S, L] or shared [L], counts on the device."""

    def __init__(self, tx: torch.Tensor, lst: torch.Tensor, count: torch.Tensor, row_cap: int, grid_x: int = 0):
        self.tx, self.list, self.count, self.row_cap, self.grid_x = tx, lst, count, row_cap, grid_x
        self.S = tx.shape[0]
        self.shared = lst.dim() == 1

    def c(self) -> GsMlpRows:
        r = GsMlpRows()
        r.n_sets, r.tx, r.list = self.S, _p(self.tx), _p(self.list)
        r.list_stride = 0 if self.shared else self.list.shape[1]
        r.count, r.count_stride = _p(self.count), 0 if self.count.numel() == 1 else 1
        r.row_cap, r.grid_x = self.row_cap, self.grid_x
        return r


class State:
    """Scratch of the network calls for S sets and row_cap rows per set."""

    def __init__(self, S: int, row_cap: int, training: bool = True, n_partial: int = 16, device="cuda",
                 n_chan: int = F):
        dev = torch.device(device)
        u16 = torch.int16
        self.cb = torch.empty(S, HID, device=dev)
        self.genc = torch.empty(S, 64, dtype=u16, device=dev)
        self.training = training
        if training:
            self.h1 = torch.empty(S, row_cap, HID, dtype=u16, device=dev)
            self.h2 = torch.empty(S, row_cap, HID, dtype=u16, device=dev)
            self.do = torch.empty(S, row_cap, 2 * n_chan, dtype=u16, device=dev)  # rows of 2F d_o values
            self.dz2 = torch.empty(S, row_cap, HID, dtype=u16, device=dev)
            self.dz1 = torch.empty(S, row_cap, HID, dtype=u16, device=dev)
            self.dc = torch.empty(S, HID, device=dev)
            self.wT = torch.empty(EMB * HID + HID * HID + HID * 2 * F, dtype=u16, device=dev)
            self.partial = torch.empty(n_partial, 2 * F * HID + HID * HID + HID * EMB, device=dev)
        self.n_partial = n_partial

    def c(self) -> GsMlpState:
        s = GsMlpState()
        s.cb, s.genc = _p(self.cb), _p(self.genc)
        if self.training:
            s.save_h1, s.save_h2, s.save_do = _p(self.h1), _p(self.h2), _p(self.do)
            s.save_dz2, s.save_dz1, s.dc = _p(self.dz2), _p(self.dz1), _p(self.dc)
            s.wT, s.partial, s.n_partial = _p(self.wT), _p(self.partial), self.n_partial
        return s


def _stream(dev):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def embed(net: AttributeNet, E_bf: torch.Tensor, Z1: Optional[torch.Tensor] = None) -> torch.Tensor:
    n = E_bf.shape[0]
    if Z1 is None:
        Z1 = torch.empty(n, HID, device=E_bf.device)
    m = net.c()
    check(lib().gs_mlp_embed(ctypes.byref(m), _p(E_bf), n, _p(Z1), _stream(E_bf.device)), "gs_mlp_embed")
    return Z1


def forward(net: AttributeNet, Z1: torch.Tensor, mean: torch.Tensor, rows: Rows, attr: torch.Tensor,
            state: State) -> torch.Tensor:
    """attr: [S, n, F, 2] float32, written for the listed rows."""
    n = mean.shape[1]
    m, r, s = net.c(), rows.c(), state.c()
    if not state.training:
        s.save_h1 = s.save_h2 = None
    check(lib().gs_mlp_forward(ctypes.byref(m), _p(Z1), _p(mean), n, ctypes.byref(r), _p(attr), n * 2 * net.F,
                               ctypes.byref(s), _stream(mean.device)), "gs_mlp_forward")
    return attr


def backward(net: AttributeNet, E_bf: torch.Tensor, mean: torch.Tensor, rows: Rows, d_attr: torch.Tensor,
             state: State, grads: Optional[dict] = None, clear_d_attr: bool = False) -> dict:
    n = mean.shape[1]
    dev = mean.device
    if grads is None:
        grads = {"W1": torch.empty(HID, IN_PAD, device=dev), "b1": torch.empty(HID, device=dev),
                 "W2": torch.empty(HID, HID, device=dev), "b2": torch.empty(HID, device=dev),
                 "W3": torch.empty(2 * net.F, HID, device=dev), "b3": torch.empty(2 * net.F, device=dev),
                 "E": torch.empty(n, EMB, device=dev)}
    g = GsMlpGrads(_p(grads["W1"]), _p(grads["b1"]), _p(grads["W2"]), _p(grads["b2"]), _p(grads["W3"]),
                   _p(grads["b3"]), _p(grads["E"]))
    m, r, s = net.c(), rows.c(), state.c()
    check(lib().gs_mlp_backward(ctypes.byref(m), _p(E_bf), _p(mean), n, ctypes.byref(r), _p(d_attr), n * 2 * net.F,
                                int(clear_d_attr), ctypes.byref(s), ctypes.byref(g), _stream(dev)),
          "gs_mlp_backward")
    return grads


def adam_step(segments, step: int, beta1=0.9, beta2=0.999, eps=1e-15, skip_if=None,
              skip_count: Optional[torch.Tensor] = None):
    """segments: list of (param, grad, m, v, bf16_shadow or None, lr).
    skip_if: device address (int) of a guard word; when it holds a non-zero
    value at run time nothing is updated and skip_count (int32 device
    tensor) is incremented."""
    arr = (GsAdamSegment * len(segments))()
    dev = segments[0][0].device
    for k, (p, g, m, v, sh, lr) in enumerate(segments):
        arr[k] = GsAdamSegment(_p(p), _p(g), _p(m), _p(v), _p(sh), p.numel(), float(lr))
    check(lib().gs_adam_step(arr, len(segments), int(step), beta1, beta2, eps,
                             None if skip_if is None else ctypes.c_void_p(skip_if), _p(skip_count), _stream(dev)),
          "gs_adam_step")


def adam_step_scheduled(segments, lr_final, total_steps: int, step_counter: torch.Tensor, beta1=0.9, beta2=0.999,
                        eps=1e-15, skip_if=None, skip_count: Optional[torch.Tensor] = None):
    """adam_step() with the step number read from (and advanced in)
    step_counter (int32 device tensor of completed steps) and rate k decaying
    log-linearly from segments[k] lr to lr_final[k] over total_steps, on the
    device (capturable)."""
    arr = (GsAdamSegment * len(segments))()
    dev = segments[0][0].device
    for k, (p, g, m, v, sh, lr) in enumerate(segments):
        arr[k] = GsAdamSegment(_p(p), _p(g), _p(m), _p(v), _p(sh), p.numel(), float(lr))
    fin = (ctypes.c_float * len(segments))(*[float(x) for x in lr_final])
    check(lib().gs_adam_step_scheduled(arr, fin, len(segments), int(total_steps), _p(step_counter), beta1, beta2,
                                       eps, None if skip_if is None else ctypes.c_void_p(skip_if), _p(skip_count),
                                       _stream(dev)), "gs_adam_step_scheduled")
