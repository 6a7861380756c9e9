"""Binding of gs_confidence_loss (include/gsparc.h): the confidence head
C = 1 + exp(g(x_rx)) and the confidence-weighted loss of Sec. 4.2, Eq. (6).
Argument marshalling only; the computation runs in the HIP kernel."""
from __future__ import annotations

import ctypes

import torch

from ._lib import check, lib

ALPHA = 0.3     # the paper's regularisation coefficient
HIDDEN = 32     # 3 -> 32 -> 1


def _f32(t: torch.Tensor, shape, name: str) -> torch.Tensor:
    if not t.is_cuda or t.dtype != torch.float32 or tuple(t.shape) != tuple(shape):
        raise ValueError("%s: float32 CUDA tensor of shape %s expected" % (name, tuple(shape)))
    return t.contiguous()


def init_weights(seed: int = 0, device="cuda") -> dict:
    """Initial head weights: W1 [32, 3] He-normal, w2 [32] small normal,
    zero biases (C = 1 + exp(g) starts near 2)."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    return {"W1": (torch.randn(HIDDEN, 3, generator=g) * (2.0 / 3.0) ** 0.5).to(device),
            "b1": torch.zeros(HIDDEN, device=device),
            "w2": (torch.randn(HIDDEN, generator=g) * 0.05).to(device),
            "b2": torch.zeros(1, device=device)}


def confidence_loss(x_rx: torch.Tensor, task_loss: torch.Tensor, weights: dict, alpha: float = ALPHA,
                    scratch: torch.Tensor = None, out: tuple = None):
    """x_rx [n, 3], task_loss [n]; weights W1 [32, 3], b1 [32], w2 [32], b2 [1]
    (float32, device).  Returns (conf [n], loss [n], grads) with grads the
    gradients of loss.sum() with respect to W1, b1, w2, b2; conf is also the
    factor on the task loss gradient.  scratch: device memory for the
    multi-workgroup sums above 4096 samples (allocated here when None).
    out: optional (conf, loss, grads) to write into (same shapes)."""
    n = x_rx.shape[0]
    x = _f32(x_rx, (n, 3), "x_rx")
    L = _f32(task_loss, (n,), "task_loss")
    W1 = _f32(weights["W1"], (HIDDEN, 3), "W1")
    b1 = _f32(weights["b1"], (HIDDEN,), "b1")
    w2 = _f32(weights["w2"], (HIDDEN,), "w2")
    b2 = _f32(weights["b2"], (1,), "b2")
    dev = x.device
    if out is not None:
        conf, loss, grads = out
        _f32(conf, (n,), "conf")
        _f32(loss, (n,), "loss")
        for k, t in (("W1", W1), ("b1", b1), ("w2", w2), ("b2", b2)):
            _f32(grads[k], tuple(t.shape), "grads[%s]" % k)
    else:
        conf = torch.empty(n, device=dev)
        loss = torch.empty(n, device=dev)
        grads = {"W1": torch.empty_like(W1), "b1": torch.empty_like(b1), "w2": torch.empty_like(w2),
                 "b2": torch.empty_like(b2)}
    p = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    nb = int(lib().gs_confidence_scratch_bytes(int(n)))
    if scratch is None and nb:
        scratch = torch.empty(nb // 4, dtype=torch.float32, device=dev)
    if scratch is not None and scratch.numel() * scratch.element_size() < nb:
        raise ValueError("scratch: at least %d bytes needed" % nb)
    check(lib().gs_confidence_loss(p(x), p(L), int(n), p(W1), p(b1), p(w2), p(b2), float(alpha), p(conf), p(loss),
                                   p(grads["W1"]), p(grads["b1"]), p(grads["w2"]), p(grads["b2"]),
                                   p(scratch) if scratch is not None else None,
                                   scratch.numel() * scratch.element_size() if scratch is not None else 0,
                                   ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)),
          "gs_confidence_loss")
    return conf, loss, grads
