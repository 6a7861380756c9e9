"""Binding of gs_emission_forward / gs_emission_backward (include/gsparc.h):
the paper's own emission form, one 3 -> 16 -> 2 network per Gaussian
(Sec. 4.1, Eq. (1)).  Argument marshalling only; the computation runs in the
HIP kernels."""
from __future__ import annotations

import ctypes

import torch

from ._lib import check, lib

NPARAM = 98      # hidden width 16: W1 [16][3], b1 [16], W2 [2][16], b2 [2]; 6 H + 2 for width H
R_NEAR = 0.2


def _dev(t: torch.Tensor, name: str, shape=None) -> torch.Tensor:
    if not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous() or (shape and tuple(t.shape) != shape):
        raise ValueError("%s: contiguous float32 CUDA tensor%s expected" % (name, " of shape %s" % (shape,) if shape else ""))
    return t


def _width(params: torch.Tensor, n: int) -> int:
    """Hidden width H from the parameter rows 6 H + 2 (H in 8, 16, 64)."""
    H = (params.shape[0] - 2) // 6
    if params.dim() != 2 or 6 * H + 2 != params.shape[0] or H not in (8, 16, 64) or params.shape[1] < n:
        raise ValueError("params: [6 H + 2, stride >= n] with H in 8, 16, 64 expected")
    return H


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream(dev):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def emission_forward(params: torch.Tensor, mean: torch.Tensor, rx: torch.Tensor, tx: torch.Tensor,
                     r_near: float = R_NEAR) -> torch.Tensor:
    """params [6 H + 2, stride] (parameter-major, stride >= n; H = 16 gives
    the paper's 98), mean [3, n] (the
    scene's layout), rx/tx [Q, 3] -> attr [Q, n, 2] (Re, Im of one complex
    channel)."""
    n = mean.shape[1]
    _dev(params, "params")
    H = _width(params, n)
    _dev(mean, "mean", (3, n))
    Q = rx.shape[0]
    _dev(rx, "rx", (Q, 3))
    _dev(tx, "tx", (Q, 3))
    attr = torch.empty(Q, n, 2, device=mean.device)
    check(lib().gs_emission_forward(_p(params), params.shape[1], H, _p(mean), n, _p(rx), _p(tx), Q, float(r_near),
                                    _p(attr), 2 * n, _stream(mean.device)), "gs_emission_forward")
    return attr


def emission_backward(params: torch.Tensor, mean: torch.Tensor, rx: torch.Tensor, tx: torch.Tensor,
                      d_attr: torch.Tensor, r_near: float = R_NEAR):
    """Gradients of sum(d_attr * attr) with respect to params ([6 H + 2, stride])
    and mean ([3, n]), summed over the queries."""
    n = mean.shape[1]
    Q = rx.shape[0]
    _dev(d_attr, "d_attr", (Q, n, 2))
    _dev(params, "params")
    _dev(mean, "mean", (3, n))
    _dev(rx, "rx", (Q, 3))
    _dev(tx, "tx", (Q, 3))
    d_params = torch.empty_like(params)
    d_mean = torch.empty_like(mean)
    check(lib().gs_emission_backward(_p(params), params.shape[1], _width(params, n), _p(mean), n, _p(rx), _p(tx), Q, float(r_near),
                                     _p(d_attr), 2 * n, _p(d_params), _p(d_mean), _stream(mean.device)),
          "gs_emission_backward")
    return d_params, d_mean
