"""Bindings of the densification entry points (include/gsparc.h): gradient
statistics, the plan (clone / split / prune, Algorithm 1), the new scene,
gathers of other per-Gaussian arrays and the opacity reset.  Argument
marshalling only; the computation runs in the HIP kernels."""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional

import torch

from ._lib import GsDensifyParams, GsScene, check, lib
from .render import Workspace, _ptr


@dataclass
class DensifyParams:
    """Thresholds of Algorithm 1's densify branch.  The paper gives none;
    these defaults are readings: tau_grad on the mean |dL/dmu| over live
    steps, epsilon r_scene as an absolute scale, N = 2 children, sigma_min,
    r_max in pixels of the equirectangular grid."""
    grad_threshold: float = 2e-4
    clone_extent: float = 0.05
    split_n: int = 2
    opacity_min: float = 0.005
    radius_max: float = 40.0

    def c(self) -> GsDensifyParams:
        return GsDensifyParams(float(self.grad_threshold), float(self.clone_extent), int(self.split_n),
                               float(self.opacity_min), float(self.radius_max))


def _stream(dev):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def stats(d_mean: torch.Tensor, live_list: torch.Tensor, live_count: torch.Tensor, acc: torch.Tensor,
          cnt: torch.Tensor):
    """acc[i] += |d_mean[:, i]|, cnt[i] += 1 for the live Gaussians."""
    n = d_mean.shape[1]
    check(lib().gs_densify_stats(_ptr(d_mean), n, _ptr(live_list), _ptr(live_count), _ptr(acc), _ptr(cnt),
                                 _stream(d_mean.device)), "gs_densify_stats")


def screen_radius(ws: Workspace, q: int = 0, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    out = torch.empty(ws.n, device=ws.buf.device) if out is None else out
    g, p = ws.grid.c(), ws.params.c()
    check(lib().gs_screen_radius(ctypes.c_void_p(ws.ptr), ws.nbytes, ws.n, ws.nq, ctypes.byref(g), ctypes.byref(p),
                                 int(q), _ptr(out), _stream(out.device)), "gs_screen_radius")
    return out


def plan(scene: dict, acc: torch.Tensor, cnt: torch.Tensor, radius: Optional[torch.Tensor], prm: DensifyParams):
    """(src, kind, n_out): device slot arrays of capacity n * N and the new
    count (host int: one synchronisation)."""
    n = scene["opacity_logit"].shape[0]
    dev = acc.device
    capn = n * prm.split_n
    src = torch.empty(capn, dtype=torch.int32, device=dev)
    kind = torch.empty(capn, dtype=torch.int32, device=dev)
    n_out = torch.empty(1, dtype=torch.int32, device=dev)
    nb = int(lib().gs_densify_scratch_bytes(n))
    scr = torch.empty(nb + 256, dtype=torch.uint8, device=dev)
    sp = scr.data_ptr() + (-scr.data_ptr()) % 256
    p = prm.c()
    check(lib().gs_densify_plan(n, _ptr(scene["log_scale"]), _ptr(scene["opacity_logit"]), _ptr(acc), _ptr(cnt),
                                _ptr(radius) if radius is not None else None, ctypes.byref(p), _ptr(src), _ptr(kind),
                                capn, _ptr(n_out), ctypes.c_void_p(sp), nb, _stream(dev)), "gs_densify_plan")
    return src, kind, int(n_out.item())


def apply(scene: dict, src: torch.Tensor, kind: torch.Tensor, n_out: int, xi: torch.Tensor, split_n: int) -> dict:
    """The new scene arrays; xi [n, split_n, 3] standard normals."""
    n = scene["opacity_logit"].shape[0]
    dev = src.device
    out = {"mean": torch.empty(3, n_out, device=dev), "log_scale": torch.empty(3, n_out, device=dev),
           "quat": torch.empty(4, n_out, device=dev), "opacity_logit": torch.empty(n_out, device=dev)}
    sc = GsScene(n, _ptr(scene["mean"]), _ptr(scene["log_scale"]), _ptr(scene["quat"]), _ptr(scene["opacity_logit"]))
    check(lib().gs_densify_apply(n, n_out, _ptr(src), _ptr(kind), ctypes.byref(sc), _ptr(xi.contiguous()),
                                 int(split_n), _ptr(out["mean"]), _ptr(out["log_scale"]), _ptr(out["quat"]),
                                 _ptr(out["opacity_logit"]), _stream(dev)), "gs_densify_apply")
    return out


def gather(arr: torch.Tensor, src: torch.Tensor, kind: torch.Tensor, n: int, n_out: int, comps: int,
           zero_new: bool) -> torch.Tensor:
    """arr viewed as [comps][n][width] 32-bit words (any 4-byte dtype, or
    16-bit with an even row width) -> [comps][n_out][width] in the new order."""
    arr = arr.contiguous()
    words = arr.numel() * arr.element_size() // 4
    width = words // (comps * n)
    if width * comps * n != words:
        raise ValueError("array is not [comps][n][width] in 32-bit words")
    shape = list(arr.shape)
    axis = 1 if comps > 1 else 0
    shape[axis] = n_out
    out = torch.empty(shape, dtype=arr.dtype, device=arr.device)
    check(lib().gs_densify_gather(n, n_out, _ptr(src), _ptr(kind), _ptr(arr), _ptr(out), int(comps), int(width),
                                  1 if zero_new else 0, _stream(arr.device)), "gs_densify_gather")
    return out


def opacity_reset(opacity_logit: torch.Tensor, cap: float = 0.01):
    check(lib().gs_opacity_reset(opacity_logit.shape[0], _ptr(opacity_logit), float(cap),
                                 _stream(opacity_logit.device)), "gs_opacity_reset")
