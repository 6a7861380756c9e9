"""Python binding of the renderer: argument marshalling around the C ABI.

Every step runs in the HIP library; PyTorch only provides device memory and
the current stream.  Shapes follow include/gsparc.h:
  scene     dict of float32 CUDA tensors mean [3,n], log_scale [3,n],
            quat [4,n], opacity_logit [n]
  attr      [n,F] / [n,F,2] (shared by all queries) or [B,n,F] / [B,n,F,2]
  rx, tx    [B,3] float32 CUDA tensors (tx may be None)
  output    [B,F,H,W] (real) or [B,F,H,W,2] (complex, re/im interleaved)
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field
from typing import Optional

import torch

from ._lib import (GS_OPT_BLEND_PER_GROUP, GS_OPT_BWD_PER_GROUP, GS_OPT_FORWARD_ONLY, GS_TRAIN_DEFER_GEOMETRY,
                   GS_TRAIN_WRITE_SPECTRUM, GsAttrs,
                   GsFlags, GsGrid, GsL2Grad, GsLayout, GsParams, GsQueries, GsScene, GsTrainTarget, check, lib)

DEFAULT_VIEW = (0.0, 1.0, 0.0, 0.0, 0.0, 1.0, 1.0, 0.0, 0.0)


@dataclass
class Params:
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    T_min: float = 1e-4
    dilation: float = 0.3
    r_near: float = 0.2
    atten_power: float = 2.0
    atten_ref: int = 0
    margin: float = 1e-3
    pair_capacity: int = 0
    chan_group: int = 0
    forward_only: bool = False
    bwd_per_group: bool = False  # backward per set and channel group even over shared geometry
    blend_per_group: bool = False  # compositing per set and channel group even over shared geometry

    def c(self) -> GsParams:
        return GsParams(self.alpha_min, self.alpha_max, self.T_min, self.dilation, self.r_near, self.atten_power,
                        int(self.atten_ref), self.margin, int(self.pair_capacity), int(self.chan_group),
                        (GS_OPT_FORWARD_ONLY if self.forward_only else 0)
                        | (GS_OPT_BWD_PER_GROUP if self.bwd_per_group else 0)
                        | (GS_OPT_BLEND_PER_GROUP if self.blend_per_group else 0))


@dataclass
class Grid:
    H: int = 90
    W: int = 360
    tile_h: int = 16
    tile_w: int = 16
    view: tuple = field(default=DEFAULT_VIEW)

    def c(self) -> GsGrid:
        g = GsGrid()
        g.H, g.W, g.tile_h, g.tile_w = self.H, self.W, self.tile_h, self.tile_w
        for k in range(9):
            g.view[k] = float(self.view[k])
        return g


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check_f32(name, t, shape=None):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise ValueError("%s must be a contiguous float32 CUDA tensor" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))


def layout(n: int, n_queries: int, grid: Grid, params: Params) -> GsLayout:
    L = GsLayout()
    g, p = grid.c(), params.c()
    check(lib().gs_workspace_layout(n, n_queries, ctypes.byref(g), ctypes.byref(p), ctypes.byref(L)),
          "gs_workspace_layout")
    return L


class Workspace:
    """Caller-owned device workspace of one (n, B, grid, params) shape."""

    def __init__(self, n: int, n_queries: int, grid: Grid, params: Params, device=None):
        self.n, self.nq, self.grid, self.params = n, n_queries, grid, params
        self.layout = layout(n, n_queries, grid, params)
        self.buf = torch.empty(self.layout.total + 256, dtype=torch.uint8, device=device or "cuda")
        base = self.buf.data_ptr()
        self.offset = (-base) % 256
        self.ptr = base + self.offset
        self.nbytes = self.layout.total

    def fits(self, n, n_queries, grid, params):
        return (n, n_queries, grid, params) == (self.n, self.nq, self.grid, self.params)

    def view(self, field_name: str, q: int, count: int, dtype=torch.int32) -> torch.Tensor:
        """Device tensor over `count` elements of a sub-buffer of query q."""
        L = self.layout
        off = getattr(L, field_name) + q * getattr(L, _STRIDE[field_name])
        itemsize = torch.empty((), dtype=dtype).element_size()
        b = self.buf[self.offset + off:self.offset + off + count * itemsize]
        return b.view(dtype)

    def overflow_word(self, q: int = 0) -> int:
        """Device address of query q's pair-overflow word (for Adam's guard)."""
        g, p = self.grid.c(), self.params.c()
        w = ctypes.c_void_p()
        check(lib().gs_overflow_word(ctypes.c_void_p(self.ptr), self.nbytes, self.n, self.nq, ctypes.byref(g),
                                     ctypes.byref(p), q, ctypes.byref(w)), "gs_overflow_word")
        return w.value

    def check(self, stream=None) -> int:
        """gs_check: synchronises; GS_OK, GS_ERR_CAPACITY (a pair buffer
        overflowed) or GS_ERR_NONFINITE (invalid Gaussians were dropped)."""
        g, p = self.grid.c(), self.params.c()
        st = stream if stream is not None else torch.cuda.current_stream().cuda_stream
        return int(lib().gs_check(ctypes.c_void_p(self.ptr), self.nbytes, self.n, self.nq, ctypes.byref(g),
                                  ctypes.byref(p), ctypes.c_void_p(st)))

    def flags(self, stream=None):
        out = (GsFlags * self.nq)()
        g, p = self.grid.c(), self.params.c()
        st = stream if stream is not None else torch.cuda.current_stream().cuda_stream
        check(lib().gs_read_flags(ctypes.c_void_p(self.ptr), self.nbytes, self.n, self.nq, ctypes.byref(g),
                                  ctypes.byref(p), out, ctypes.c_void_p(st)), "gs_read_flags")
        return [dict(n_visible=f.n_visible, n_pairs=f.n_pairs, overflow=f.overflow, n_invalid=f.n_invalid)
                for f in out]


_STRIDE = {"flags": "flags_stride", "rec": "rec_stride", "rect": "rect_stride", "status": "status_stride",
           "tinfo": "tinfo_stride", "order": "order_stride", "keys": "keys_stride",
           "pair_keys": "pair_keys_stride", "pair_list": "pair_list_stride", "ranges": "ranges_stride",
           "T_final": "pix_stride", "n_last": "pix_stride", "n_contrib": "pix_stride"}


def _scene_c(scene: dict) -> GsScene:
    n = scene["opacity_logit"].shape[0]
    _check_f32("mean", scene["mean"], (3, n))
    _check_f32("log_scale", scene["log_scale"], (3, n))
    _check_f32("quat", scene["quat"], (4, n))
    _check_f32("opacity_logit", scene["opacity_logit"], (n,))
    return GsScene(n, _ptr(scene["mean"]), _ptr(scene["log_scale"]), _ptr(scene["quat"]),
                   _ptr(scene["opacity_logit"]))


def _attrs_c(attr: torch.Tensor, n: int, B: int, is_complex: bool) -> GsAttrs:
    _check_f32("attr", attr)
    per_query = attr.dim() == (4 if is_complex else 3)
    shape = attr.shape[1:] if per_query else attr.shape
    if shape[0] != n or (is_complex and shape[-1] != 2):
        raise ValueError("attr shape %s does not match n=%d complex=%s" % (tuple(attr.shape), n, is_complex))
    if per_query and attr.shape[0] != B:
        raise ValueError("attr has %d query slices, expected %d" % (attr.shape[0], B))
    F = shape[1]
    stride = attr[0].numel() if per_query else 0
    return GsAttrs(F, int(is_complex), _ptr(attr), stride)


def forward(scene: dict, attr: torch.Tensor, rx: torch.Tensor, tx: Optional[torch.Tensor] = None,
            grid: Grid = Grid(), params: Params = Params(), is_complex: bool = False,
            workspace: Optional[Workspace] = None, out: Optional[torch.Tensor] = None):
    """Renders B queries; returns (spectrum, workspace)."""
    sc = _scene_c(scene)
    n = sc.n
    _check_f32("rx", rx)
    B = rx.shape[0]
    if rx.shape != (B, 3):
        raise ValueError("rx must be [B,3]")
    if tx is not None:
        _check_f32("tx", tx, (B, 3))
    a = _attrs_c(attr, n, B, is_complex)
    F = a.n_chan
    shape = (B, F, grid.H, grid.W, 2) if is_complex else (B, F, grid.H, grid.W)
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=rx.device)
    else:
        _check_f32("out", out, shape)
    if workspace is None or not workspace.fits(n, B, grid, params):
        workspace = Workspace(n, B, grid, params, device=rx.device)
    q = GsQueries(B, _ptr(rx), _ptr(tx))
    g, p = grid.c(), params.c()
    stream = torch.cuda.current_stream(rx.device).cuda_stream
    check(lib().gs_render_forward(ctypes.byref(sc), ctypes.byref(a), ctypes.byref(q), ctypes.byref(g),
                                  ctypes.byref(p), _ptr(out), ctypes.c_void_p(workspace.ptr), workspace.nbytes,
                                  ctypes.c_void_p(stream)), "gs_render_forward")
    return out, workspace


def prepare(scene: dict, rx: torch.Tensor, tx: Optional[torch.Tensor] = None, grid: Grid = Grid(),
            params: Params = Params(), workspace: Optional[Workspace] = None) -> Workspace:
    """Projection, depth sort and tile binning of B queries into a workspace."""
    sc = _scene_c(scene)
    _check_f32("rx", rx)
    B = rx.shape[0]
    if tx is not None:
        _check_f32("tx", tx, (B, 3))
    if workspace is None or not workspace.fits(sc.n, B, grid, params):
        workspace = Workspace(sc.n, B, grid, params, device=rx.device)
    q = GsQueries(B, _ptr(rx), _ptr(tx))
    g, p = grid.c(), params.c()
    stream = torch.cuda.current_stream(rx.device).cuda_stream
    check(lib().gs_render_prepare(ctypes.byref(sc), ctypes.byref(q), ctypes.byref(g), ctypes.byref(p),
                                  ctypes.c_void_p(workspace.ptr), workspace.nbytes, ctypes.c_void_p(stream)),
          "gs_render_prepare")
    return workspace


def fit_pair_capacity(scene: dict, rx: torch.Tensor, tx: Optional[torch.Tensor] = None, grid: Grid = Grid(),
                      params: Params = Params(), headroom: float = 2.0) -> Params:
    """Params whose pair_capacity fits these queries of a static scene: one
    prepare with the default capacity (n min(tiles, 64) + 4096 pairs per
    query, several times what scenes of the benchmark's kind need), then
    headroom times the largest measured pair count plus 4096.  The workspace
    of a static serving scene shrinks accordingly; a scene whose geometry
    changes keeps the default (an overflow is detected and flagged, see
    gs_read_flags)."""
    from dataclasses import replace
    ws = prepare(scene, rx, tx=tx, grid=grid, params=replace(params, pair_capacity=0))
    fl = ws.flags()
    if any(f["overflow"] for f in fl):
        return replace(params, pair_capacity=0)
    need = max(f["n_pairs"] for f in fl)
    return replace(params, pair_capacity=int(headroom * need) + 4096)


def blend(workspace: Workspace, attr: torch.Tensor, n_sets: Optional[int] = None, is_complex: bool = False,
          out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Compositing over a prepared workspace.  attr: [n_sets, n, F(,2)] (or
    [n, F(,2)] with n_sets = 1 per prepared query)."""
    _check_f32("attr", attr)
    n, B = workspace.n, workspace.nq
    per_set = attr.dim() == (4 if is_complex else 3)
    S = attr.shape[0] if per_set else (n_sets if n_sets is not None else B)
    if n_sets is not None and n_sets != S:
        raise ValueError("n_sets %d does not match attr" % n_sets)
    a = _attrs_c(attr, n, S, is_complex)
    shape = (S, a.n_chan, workspace.grid.H, workspace.grid.W) + ((2,) if is_complex else ())
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=attr.device)
    else:
        _check_f32("out", out, shape)
    g, p = workspace.grid.c(), workspace.params.c()
    stream = torch.cuda.current_stream(attr.device).cuda_stream
    check(lib().gs_render_blend(ctypes.byref(a), n, B, S, ctypes.byref(g), ctypes.byref(p), _ptr(out),
                                ctypes.c_void_p(workspace.ptr), workspace.nbytes, ctypes.c_void_p(stream)),
          "gs_render_blend")
    return out


def blend_loss(workspace: Workspace, attr: torch.Tensor, target: torch.Tensor, lambda_ch: float = 1.0,
               n_sets: Optional[int] = None, is_complex: bool = False, out: Optional[torch.Tensor] = None,
               partial: Optional[torch.Tensor] = None):
    """blend() with loss_stats() fused into the compositing kernel's output
    stage (gs_render_blend_loss): returns (spectrum, loss per set, h_hat,
    mean_grad, scale); `partial`, when given, receives scale (spectrum -
    target) from the same pass."""
    _check_f32("attr", attr)
    n, B = workspace.n, workspace.nq
    per_set = attr.dim() == (4 if is_complex else 3)
    S = attr.shape[0] if per_set else (n_sets if n_sets is not None else B)
    if n_sets is not None and n_sets != S:
        raise ValueError("n_sets %d does not match attr" % n_sets)
    a = _attrs_c(attr, n, S, is_complex)
    F, H, W = a.n_chan, workspace.grid.H, workspace.grid.W
    C = 2 if is_complex else 1
    shape = (S, F, H, W) + ((2,) if is_complex else ())
    dev = attr.device
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=dev)
    else:
        _check_f32("out", out, shape)
    _check_f32("target", target, shape)
    if partial is not None:
        _check_f32("partial", partial, shape)
    loss = torch.empty(S, device=dev)
    hhat = torch.empty((S, F, 2) if is_complex else (S, F), device=dev)
    mgrad = torch.empty(S, F * C, device=dev)
    gr = workspace.grid
    tiles = -(-gr.H // gr.tile_h) * -(-gr.W // gr.tile_w)
    nacc = S * F * C * 3
    nbytes = -(-nacc * 4 // 256) * 256 + nacc * tiles * (gr.tile_h * gr.tile_w // 64) * 4
    scratch = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    base = scratch.data_ptr()
    off = (-base) % 256
    g, p = workspace.grid.c(), workspace.params.c()
    stream = torch.cuda.current_stream(dev).cuda_stream
    check(lib().gs_render_blend_loss(ctypes.byref(a), n, B, S, ctypes.byref(g), ctypes.byref(p), _ptr(out),
                                     ctypes.c_void_p(workspace.ptr), workspace.nbytes, _ptr(target),
                                     float(lambda_ch), _ptr(loss), _ptr(hhat), _ptr(mgrad), _ptr(partial),
                                     ctypes.c_void_p(base + off), scratch.numel() - off, ctypes.c_void_p(stream)),
          "gs_render_blend_loss")
    return out, loss, hhat, mgrad, 2.0 / (F * H * W * S)


def backward(workspace: Workspace, scene: dict, attr: torch.Tensor, rx: torch.Tensor, spectrum: torch.Tensor,
             d_spectrum: torch.Tensor, tx: Optional[torch.Tensor] = None, is_complex: bool = False,
             n_sets: Optional[int] = None, d_attr: Optional[torch.Tensor] = None, out: Optional[dict] = None) -> dict:
    """Gradients of a forward (or prepare + blend) call that used `workspace`.
    Returns d_mean, d_log_scale, d_quat, d_opacity_logit, d_attr."""
    sc = _scene_c(scene)
    n = sc.n
    B = rx.shape[0]
    per_set = attr.dim() == (4 if is_complex else 3)
    S = n_sets if n_sets is not None else (attr.shape[0] if per_set else B)
    a = _attrs_c(attr, n, S, is_complex)
    _check_f32("spectrum", spectrum)
    _check_f32("d_spectrum", d_spectrum, tuple(spectrum.shape))
    dev = rx.device
    g = out if out is not None else {
        "d_mean": torch.empty(3, n, device=dev), "d_log_scale": torch.empty(3, n, device=dev),
        "d_quat": torch.empty(4, n, device=dev), "d_opacity_logit": torch.empty(n, device=dev)}
    # a caller-provided d_attr must be all zero: it is accumulated into, not cleared
    flags = 1 if d_attr is not None else 0
    g["d_attr"] = d_attr if d_attr is not None else torch.empty_like(attr)
    q = GsQueries(B, _ptr(rx), _ptr(tx))
    gr, p = workspace.grid.c(), workspace.params.c()
    stream = torch.cuda.current_stream(dev).cuda_stream
    check(lib().gs_render_backward(ctypes.byref(sc), ctypes.byref(a), ctypes.byref(q), S, ctypes.byref(gr),
                                   ctypes.byref(p), _ptr(spectrum), _ptr(d_spectrum), _ptr(g["d_mean"]),
                                   _ptr(g["d_log_scale"]), _ptr(g["d_quat"]), _ptr(g["d_opacity_logit"]),
                                   _ptr(g["d_attr"]), flags, ctypes.c_void_p(workspace.ptr), workspace.nbytes,
                                   ctypes.c_void_p(stream)), "gs_render_backward")
    return g


def backward_l2(workspace: Workspace, scene: dict, attr: torch.Tensor, rx: torch.Tensor, spectrum: torch.Tensor,
                target: Optional[torch.Tensor], mean_grad: torch.Tensor, scale: float,
                partial: Optional[torch.Tensor] = None, tx: Optional[torch.Tensor] = None,
                is_complex: bool = False, n_sets: Optional[int] = None, d_attr: Optional[torch.Tensor] = None,
                out: Optional[dict] = None) -> dict:
    """backward() for dL/dspectrum = E + mean_grad (the loss of
    loss_stats()), assembled inside the kernel: E = partial when given,
    else scale (spectrum - target)."""
    sc = _scene_c(scene)
    n = sc.n
    B = rx.shape[0]
    per_set = attr.dim() == (4 if is_complex else 3)
    S = n_sets if n_sets is not None else (attr.shape[0] if per_set else B)
    a = _attrs_c(attr, n, S, is_complex)
    _check_f32("spectrum", spectrum)
    if partial is not None:
        _check_f32("partial", partial, tuple(spectrum.shape))
    else:
        _check_f32("target", target, tuple(spectrum.shape))
    _check_f32("mean_grad", mean_grad)
    if mean_grad.numel() != S * a.n_chan * (2 if is_complex else 1):
        raise ValueError("mean_grad must hold n_sets * F * c values")
    dev = rx.device
    g = out if out is not None else {
        "d_mean": torch.empty(3, n, device=dev), "d_log_scale": torch.empty(3, n, device=dev),
        "d_quat": torch.empty(4, n, device=dev), "d_opacity_logit": torch.empty(n, device=dev)}
    flags = 1 if d_attr is not None else 0
    g["d_attr"] = d_attr if d_attr is not None else torch.empty_like(attr)
    q = GsQueries(B, _ptr(rx), _ptr(tx))
    gr, p = workspace.grid.c(), workspace.params.c()
    lg = GsL2Grad(_ptr(partial), _ptr(target), _ptr(mean_grad), float(scale))
    stream = torch.cuda.current_stream(dev).cuda_stream
    check(lib().gs_render_backward_l2(ctypes.byref(sc), ctypes.byref(a), ctypes.byref(q), S, ctypes.byref(gr),
                                      ctypes.byref(p), _ptr(spectrum), ctypes.byref(lg), _ptr(g["d_mean"]),
                                      _ptr(g["d_log_scale"]), _ptr(g["d_quat"]), _ptr(g["d_opacity_logit"]),
                                      _ptr(g["d_attr"]), flags, ctypes.c_void_p(workspace.ptr), workspace.nbytes,
                                      ctypes.c_void_p(stream)), "gs_render_backward_l2")
    return g


def live(workspace: Workspace, lst: Optional[torch.Tensor] = None, count: Optional[torch.Tensor] = None):
    """Gaussians reaching some pixel, per prepared query: (list [B, n] int32
    (valid prefix of length count[b]), count [B] int32 on the device)."""
    n, B = workspace.n, workspace.nq
    dev = workspace.buf.device
    if lst is None:
        lst = torch.empty(B, n, dtype=torch.int32, device=dev)
    if count is None:
        count = torch.empty(B, dtype=torch.int32, device=dev)
    g, p = workspace.grid.c(), workspace.params.c()
    stream = torch.cuda.current_stream(dev).cuda_stream
    check(lib().gs_render_live(n, B, ctypes.byref(g), ctypes.byref(p), ctypes.c_void_p(workspace.ptr),
                               workspace.nbytes, _ptr(lst), n, _ptr(count), ctypes.c_void_p(stream)),
          "gs_render_live")
    return lst, count


def loss_spectrum(spectrum: torch.Tensor, target: torch.Tensor, is_complex: bool, lambda_ch: float = 1.0):
    """Spectrum L2 + Eq. (4) on the spatial means.  spectrum, target:
    [B,F,H,W(,2)].  Returns (loss per set [B], h_hat [B,F(,2)], d_spectrum)
    with d_spectrum the gradient of the mean over sets."""
    _check_f32("spectrum", spectrum)
    _check_f32("target", target, tuple(spectrum.shape))
    B, F, H, W = spectrum.shape[:4]
    C = 2 if is_complex else 1
    dev = spectrum.device
    loss = torch.empty(B, device=dev)
    hhat = torch.empty((B, F, 2) if is_complex else (B, F), device=dev)
    d = torch.empty_like(spectrum)
    scratch = torch.empty(B * F * C * 3 * 4 + 256, dtype=torch.uint8, device=dev)
    base = scratch.data_ptr()
    off = (-base) % 256
    stream = torch.cuda.current_stream(dev).cuda_stream
    check(lib().gs_loss_spectrum(_ptr(spectrum), _ptr(target), B, F, int(is_complex), H, W, float(lambda_ch),
                                 _ptr(loss), _ptr(hhat), _ptr(d), ctypes.c_void_p(base + off),
                                 scratch.numel() - off, ctypes.c_void_p(stream)), "gs_loss_spectrum")
    return loss, hhat, d


def loss_stats(spectrum: torch.Tensor, target: torch.Tensor, is_complex: bool, lambda_ch: float = 1.0,
               partial: Optional[torch.Tensor] = None):
    """The loss of loss_spectrum() in one pass: (loss per set [B], h_hat
    [B,F(,2)], mean_grad [B,F*c], scale) for backward_l2(); when `partial`
    (layout of the spectrum) is given, the same pass writes the elementwise
    gradient part scale (spectrum - target) into it."""
    _check_f32("spectrum", spectrum)
    _check_f32("target", target, tuple(spectrum.shape))
    B, F, H, W = spectrum.shape[:4]
    C = 2 if is_complex else 1
    dev = spectrum.device
    loss = torch.empty(B, device=dev)
    hhat = torch.empty((B, F, 2) if is_complex else (B, F), device=dev)
    mgrad = torch.empty(B, F * C, device=dev)
    scratch = torch.empty(B * F * C * 3 * 4 + 256, dtype=torch.uint8, device=dev)
    base = scratch.data_ptr()
    off = (-base) % 256
    stream = torch.cuda.current_stream(dev).cuda_stream
    if partial is not None:
        _check_f32("partial", partial, tuple(spectrum.shape))
    check(lib().gs_loss_spectrum_stats(_ptr(spectrum), _ptr(target), B, F, int(is_complex), H, W, float(lambda_ch),
                                       _ptr(loss), _ptr(hhat), _ptr(mgrad), _ptr(partial), ctypes.c_void_p(base + off),
                                       scratch.numel() - off, ctypes.c_void_p(stream)), "gs_loss_spectrum_stats")
    return loss, hhat, mgrad, 2.0 / (F * H * W * B)


def spatial_mean(spectrum: torch.Tensor, is_complex: bool, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Eq. (2): the coherent spatial mean of each channel, [B,F(,2)]."""
    _check_f32("spectrum", spectrum)
    B, F, H, W = spectrum.shape[:4]
    shape = (B, F, 2) if is_complex else (B, F)
    if out is None:
        out = torch.empty(shape, device=spectrum.device)
    else:
        _check_f32("out", out, shape)
    stream = torch.cuda.current_stream(spectrum.device).cuda_stream
    check(lib().gs_spatial_mean(_ptr(spectrum), B, F, int(is_complex), H, W, _ptr(out), ctypes.c_void_p(stream)),
          "gs_spatial_mean")
    return out


class TrainScratch:
    """Caller-owned scratch of train_pass() for (n_sets, F, grid)."""

    def __init__(self, n_sets: int, n_chan: int, grid: Grid, device=None):
        g = grid.c()
        self.key = (n_sets, n_chan, grid)
        self.nbytes = int(lib().gs_train_scratch_bytes(n_sets, n_chan, ctypes.byref(g)))
        if self.nbytes == 0:
            raise ValueError("no training scratch size for these shapes")
        self.buf = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=device or "cuda")
        base = self.buf.data_ptr()
        self.ptr = base + (-base) % 256


def train_pass(workspace: Workspace, scene: dict, attr: torch.Tensor, rx: torch.Tensor, live_list: torch.Tensor,
               live_count: torch.Tensor, target: torch.Tensor, target_mean: torch.Tensor, lambda_ch: float = 1.0,
               spectrum: Optional[torch.Tensor] = None, write_spectrum: bool = False,
               d_attr: Optional[torch.Tensor] = None, out: Optional[dict] = None,
               scratch: Optional[TrainScratch] = None, loss: Optional[torch.Tensor] = None,
               h_hat: Optional[torch.Tensor] = None, grad_scale: Optional[torch.Tensor] = None,
               defer_geometry: bool = False):
    """Fused compositing + loss + backward over S complex attribute sets
    sharing the workspace's one prepared receiver (gs_render_train), after
    live().  attr [S,n,F,2]; target [S,F,H,W,2]; target_mean [S,F,2]
    (spatial_mean of the target); grad_scale: optional device float c, every
    gradient then that of c L.  defer_geometry: the scene gradients are left
    to train_geometry() (GS_TRAIN_DEFER_GEOMETRY).  Returns (loss [S],
    h_hat [S,F,2], gradients dict, spectrum)."""
    sc = _scene_c(scene)
    n = sc.n
    if attr.dim() != 4:
        raise ValueError("attr must be [S, n, F, 2]")
    S = attr.shape[0]
    a = _attrs_c(attr, n, S, True)
    F, H, W = a.n_chan, workspace.grid.H, workspace.grid.W
    dev = attr.device
    shape = (S, F, H, W, 2)
    _check_f32("target", target, shape)
    _check_f32("target_mean", target_mean, (S, F, 2))
    if grad_scale is not None and (not grad_scale.is_cuda or grad_scale.dtype != torch.float32 or
                                   grad_scale.numel() < 1):
        raise ValueError("grad_scale: a float32 CUDA tensor expected")
    if spectrum is None:
        spectrum = torch.empty(shape, device=dev)
    else:
        _check_f32("spectrum", spectrum, shape)
    if scratch is None or scratch.key != (S, F, workspace.grid):
        scratch = TrainScratch(S, F, workspace.grid, device=dev)
    loss = torch.empty(S, device=dev) if loss is None else loss
    h_hat = torch.empty(S, F, 2, device=dev) if h_hat is None else h_hat
    g = out if out is not None else {
        "d_mean": torch.empty(3, n, device=dev), "d_log_scale": torch.empty(3, n, device=dev),
        "d_quat": torch.empty(4, n, device=dev), "d_opacity_logit": torch.empty(n, device=dev)}
    flags = ((1 if d_attr is not None else 0) | (GS_TRAIN_WRITE_SPECTRUM if write_spectrum else 0) |
             (GS_TRAIN_DEFER_GEOMETRY if defer_geometry else 0))
    g["d_attr"] = d_attr if d_attr is not None else torch.empty_like(attr)
    tt = GsTrainTarget(_ptr(target), _ptr(target_mean), float(lambda_ch), _ptr(loss), _ptr(h_hat),
                       _ptr(grad_scale) if grad_scale is not None else None)
    q = GsQueries(1, _ptr(rx), None)
    gr, p = workspace.grid.c(), workspace.params.c()
    stream = torch.cuda.current_stream(dev).cuda_stream
    check(lib().gs_render_train(ctypes.byref(sc), ctypes.byref(a), ctypes.byref(q), S, ctypes.byref(gr),
                                ctypes.byref(p), _ptr(live_list), _ptr(live_count), ctypes.byref(tt),
                                _ptr(spectrum), _ptr(g["d_mean"]), _ptr(g["d_log_scale"]), _ptr(g["d_quat"]),
                                _ptr(g["d_opacity_logit"]), _ptr(g["d_attr"]), flags,
                                ctypes.c_void_p(workspace.ptr), workspace.nbytes, ctypes.c_void_p(scratch.ptr),
                                scratch.nbytes, ctypes.c_void_p(stream)), "gs_render_train")
    return loss, h_hat, g, spectrum


def train_geometry(workspace: Workspace, scene: dict, rx: torch.Tensor, out: dict):
    """The scene gradients of a train_pass(defer_geometry=True) on the same
    workspace (gs_render_train_geometry), on the current stream: out's
    d_mean [3,n], d_log_scale [3,n], d_quat [4,n], d_opacity_logit [n]."""
    sc = _scene_c(scene)
    n = sc.n
    for k, shape in (("d_mean", (3, n)), ("d_log_scale", (3, n)), ("d_quat", (4, n)), ("d_opacity_logit", (n,))):
        _check_f32(k, out[k], shape)
    q = GsQueries(1, _ptr(rx), None)
    gr, p = workspace.grid.c(), workspace.params.c()
    stream = torch.cuda.current_stream(out["d_mean"].device).cuda_stream
    check(lib().gs_render_train_geometry(ctypes.byref(sc), ctypes.byref(q), ctypes.byref(gr), ctypes.byref(p),
                                         _ptr(out["d_mean"]), _ptr(out["d_log_scale"]), _ptr(out["d_quat"]),
                                         _ptr(out["d_opacity_logit"]), ctypes.c_void_p(workspace.ptr),
                                         workspace.nbytes, ctypes.c_void_p(stream)), "gs_render_train_geometry")
    return out


def loss_l1_ssim(spectrum: torch.Tensor, target: torch.Tensor, lambda_1: float = 0.2, grad: bool = True):
    """Eq. (5) on real spectra [S,F,H,W]: returns (loss [S], ssim [S], l1 [S],
    dL/dspectrum of the mean over sets, or None)."""
    _check_f32("spectrum", spectrum)
    _check_f32("target", target, tuple(spectrum.shape))
    if spectrum.dim() != 4:
        raise ValueError("spectrum must be [S, F, H, W] (real)")
    S, F, H, W = spectrum.shape
    dev = spectrum.device
    loss, ssim, l1 = (torch.empty(S, device=dev) for _ in range(3))
    d = torch.empty_like(spectrum) if grad else None
    nbytes = int(lib().gs_loss_l1_ssim_scratch_bytes(S, F, H, W))
    scratch = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    base = scratch.data_ptr()
    off = (-base) % 256
    stream = torch.cuda.current_stream(dev).cuda_stream
    check(lib().gs_loss_l1_ssim(_ptr(spectrum), _ptr(target), S, F, H, W, float(lambda_1), _ptr(loss), _ptr(ssim),
                                _ptr(l1), _ptr(d), ctypes.c_void_p(base + off), nbytes, ctypes.c_void_p(stream)),
          "gs_loss_l1_ssim")
    return loss, ssim, l1, d
