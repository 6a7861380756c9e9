"""CPU oracle for the hemispherical RF splatting renderer.

TEST INFRASTRUCTURE ONLY. The product path never imports this package: only
the test suite, the smoke check and the CPU-baseline leg of the benchmark do.
It shares no code with the GPU library; the only common dependency is the
seeded input generator module ``synth``.

Contents
  * ``oracle.c`` -- FP64 projection (Sec. 3.2, Sec. 4.2), depth order,
    per-pixel untiled compositing (Eq. (3)), independent tile binning and a
    tiled variant; loaded here through ctypes.
  * ``torch_ref`` -- an independent dense FP64 PyTorch-CPU implementation of
    the same forward, differentiated by autograd (gradient reference).
  * ``confidence_ref`` -- FP64 confidence head and the confidence-weighted
    loss (Eq. (6)) with its gradients.
  * ``emission_ref`` -- FP64 per-Gaussian 3 -> 16 -> 2 emission networks
    (the paper's own form of Eq. (1)) with their gradients.
  * ``mlp_ref`` -- FP64 attribute network with BF16 rounding emulation,
    losses and Adam.

The parameter defaults follow the readings stated in the C file header:
alpha_min = 1/255, alpha_max = 0.99, T_min = 1e-4, dilation 0.3 px^2,
r_near = 0.2 m, 1/d^2 attenuation referenced to the receiver.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

ST_VISIBLE, ST_NEAR, ST_FAINT, ST_OFFGRID, ST_INVALID = range(5)
# record fields (must match the enum in oracle.c)
REC_FIELDS = ["px", "py", "ca", "cb", "cc", "sigma", "att", "ex", "ey",
              "s00", "s01", "s11", "dist", "qmax", "az", "el"]

DEFAULTS = dict(alpha_min=1.0 / 255.0, alpha_max=0.99, T_min=1e-4, dilation=0.3,
                r_near=0.2, atten_power=2.0, atten_ref=0, margin=1e-3)

# Receiver frame: world z is up; (x', y', z') = (y_w, z_w, x_w), so the
# azimuth is atan2(y_w, x_w) and the elevation asin(z_w / r).
DEFAULT_VIEW = np.array([[0.0, 1.0, 0.0], [0.0, 0.0, 1.0], [1.0, 0.0, 0.0]])


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (FP64, no FP contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-Wall", "-o", tmp, SRC, "-lm", "-lpthread"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        i32 = ctypes.c_int
        L.orc_r32.restype = ctypes.c_float
        L.orc_r32.argtypes = [ctypes.c_float] * 6
        L.orc_project.restype = i32
        L.orc_project.argtypes = [i32, P, P, P, P, P, P, P, i32, i32, P, P, P, P, P]
        L.orc_order.restype = i32
        L.orc_order.argtypes = [i32, P, P, P]
        L.orc_render.restype = i32
        L.orc_render.argtypes = [i32, P, P, i32, P, i32, i32, i32, i32, P, P, i32, P, P, P, P, P, P, P, i32]
        L.orc_bin.restype = ctypes.c_long
        L.orc_bin.argtypes = [i32, P, P, i32, i32, i32, i32, P, P, ctypes.c_long]
        L.orc_render_tiled.restype = i32
        L.orc_render_tiled.argtypes = [i32, P, P, P, i32, i32, P, i32, i32, i32, i32, P, P, P, P, i32]
        L.orc_tiles_of.restype = i32
        L.orc_tiles_of.argtypes = [P, i32, i32, i32, i32, P, P, P]
        L.orc_nrec.restype = i32
        assert L.orc_nrec() == len(REC_FIELDS)
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def params(**kw) -> np.ndarray:
    d = dict(DEFAULTS)
    d.update(kw)
    # the renderer's parameters are single-precision numbers: use the same values
    v = np.array([d["alpha_min"], d["alpha_max"], d["T_min"], d["dilation"], d["r_near"],
                  d["atten_power"], float(d["atten_ref"]), d["margin"]], dtype=np.float64)
    return v.astype(np.float32).astype(np.float64)


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def _nthreads(n):
    return n if n else min(os.cpu_count() or 1, 64)


def r32(mean_xyz, rx) -> float:
    return lib().orc_r32(*[float(v) for v in mean_xyz], *[float(v) for v in rx])


def project(scene: dict, rx, H: int, W: int, prm=None, tx=None, view=None) -> dict:
    """Per-Gaussian FP64 records, FP32 distance keys, integer support
    rectangles (c0, c1, r0, r1) and cull status."""
    prm = params() if prm is None else prm
    mean, ls, q, o = (_f32(scene[k]) for k in ("mean", "log_scale", "quat", "opacity_logit"))
    n = o.shape[0]
    rx = _f32(rx).reshape(3)
    tx = rx if tx is None else _f32(tx).reshape(3)
    V = np.ascontiguousarray(DEFAULT_VIEW if view is None else view, dtype=np.float64)
    rec = np.zeros((n, len(REC_FIELDS)), np.float64)
    key = np.zeros(n, np.float32)
    rect = np.zeros((n, 4), np.int32)
    status = np.zeros(n, np.int32)
    nvis = lib().orc_project(n, _p(mean), _p(ls), _p(q), _p(o), _p(rx), _p(tx), _p(V), H, W,
                             _p(prm), _p(rec), _p(key), _p(rect), _p(status))
    out = {k: rec[:, i] for i, k in enumerate(REC_FIELDS)}
    out.update(rec=rec, r32=key, rect=rect, status=status, nvis=nvis, n=n)
    return out


def depth_order(proj: dict) -> np.ndarray:
    n = proj["n"]
    order = np.zeros(max(n, 1), np.int32)
    m = lib().orc_order(n, _p(proj["r32"]), _p(proj["status"]), _p(order))
    return order[:m].copy()


def composite(proj: dict, order: np.ndarray, attr, H: int, W: int, prm=None, pixels=None,
              nthreads: int = 0) -> dict:
    """Per-pixel compositing over `order` (no tiles). attr: [n, F] real or
    [n, F, 2] complex. Returns out [F,H,W] (complex128 when complex), absacc,
    T_final, n_contrib, ambig, ambig_kind (bits: 1 alpha_min, 2 alpha_max,
    4 the stop, 8 the seam), flip_bound [F,H,W] (the change a flip of the
    ambiguous decisions can cause; 0 on unambiguous pixels) and live [n]
    (bit 0: taken at an unambiguous pixel; bit 1: taken at, or a decision in
    doubt at, an ambiguous pixel)."""
    prm = params() if prm is None else prm
    attr = _f32(attr)
    n = proj["n"]
    cplx = attr.ndim == 3
    F = attr.shape[1]
    C = 2 if cplx else 1
    assert attr.shape[0] == n
    out = np.zeros((F, H, W, C), np.float64)
    absacc = np.zeros((F, H, W), np.float64)
    Tf = np.ones((H, W), np.float64)
    nc = np.zeros((H, W), np.int32)
    amb = np.zeros((H, W), np.uint8)
    flipb = np.zeros((F, H, W), np.float64)
    live = np.zeros(max(n, 1), np.uint8)
    order = np.ascontiguousarray(order, dtype=np.int32)
    if pixels is None:
        pix, npix = None, 0
    else:
        pix = np.ascontiguousarray(pixels, dtype=np.int32)
        npix = pix.shape[0]
    rc = lib().orc_render(n, _p(proj["rec"]), _p(order), order.shape[0], _p(attr), F, int(cplx), H, W,
                          _p(prm), None if pix is None else _p(pix), npix, _p(out), _p(Tf), _p(nc),
                          _p(absacc), _p(amb), _p(flipb), _p(live), _nthreads(nthreads))
    assert rc == 0
    val = out[..., 0] + 1j * out[..., 1] if cplx else out[..., 0]
    return dict(out=val, absacc=absacc, T_final=Tf, n_contrib=nc, ambig=amb.astype(bool), ambig_kind=amb,
                flip_bound=flipb, live=live[:n])


def render(scene: dict, attr, rx, H: int, W: int, prm=None, tx=None, view=None, pixels=None,
           nthreads: int = 0) -> dict:
    """The oracle proper: project, order by (r32, index), composite every
    pixel over every Gaussian."""
    proj = project(scene, rx, H, W, prm, tx=tx, view=view)
    order = depth_order(proj)
    res = composite(proj, order, attr, H, W, prm, pixels=pixels, nthreads=nthreads)
    res.update(proj=proj, order=order)
    return res


def tile_grid(H, W, tw, th):
    return (W + tw - 1) // tw, (H + th - 1) // th


def bin_tiles(proj: dict, order: np.ndarray, H: int, W: int, tw: int = 16, th: int = 16,
              rect=None):
    """Per-tile Gaussian lists (tile id = ty * TX + tx), each in `order`'s
    order. Returns (tile_off [T+1] int32, list [P] int32)."""
    rect = proj["rect"] if rect is None else np.ascontiguousarray(rect, dtype=np.int32)
    TX, TY = tile_grid(H, W, tw, th)
    off = np.zeros(TX * TY + 1, np.int32)
    order = np.ascontiguousarray(order, dtype=np.int32)
    P = lib().orc_bin(order.shape[0], _p(order), _p(rect), H, W, tw, th, _p(off), None, 0)
    lst = np.zeros(max(P, 1), np.int32)
    P2 = lib().orc_bin(order.shape[0], _p(order), _p(rect), H, W, tw, th, _p(off), _p(lst), P)
    assert P2 == P
    return off, lst[:P].copy()


def tiles_of(rect_row, H, W, tw=16, th=16):
    """Tile set of one rectangle as a sorted list of tile ids."""
    r = np.ascontiguousarray(rect_row, dtype=np.int32)
    ty0 = np.zeros(1, np.int32)
    ty1 = np.zeros(1, np.int32)
    rng = np.zeros(4, np.int32)
    nr = lib().orc_tiles_of(_p(r), W, H, tw, th, _p(ty0), _p(ty1), _p(rng))
    TX, _ = tile_grid(H, W, tw, th)
    out = []
    for ty in range(int(ty0[0]), int(ty1[0]) + 1):
        for k in range(nr):
            out.extend(ty * TX + tx for tx in range(int(rng[2 * k]), int(rng[2 * k + 1]) + 1))
    return sorted(out)


def composite_tiled(proj: dict, tile_off, tile_list, attr, H: int, W: int, tw=16, th=16, prm=None,
                    nthreads: int = 0) -> dict:
    prm = params() if prm is None else prm
    attr = _f32(attr)
    n = proj["n"]
    cplx = attr.ndim == 3
    F = attr.shape[1]
    C = 2 if cplx else 1
    out = np.zeros((F, H, W, C), np.float64)
    Tf = np.ones((H, W), np.float64)
    nc = np.zeros((H, W), np.int32)
    tile_off = np.ascontiguousarray(tile_off, dtype=np.int32)
    tile_list = np.ascontiguousarray(tile_list if len(tile_list) else np.zeros(1), dtype=np.int32)
    rc = lib().orc_render_tiled(n, _p(proj["rec"]), _p(tile_off), _p(tile_list), tw, th, _p(attr), F,
                                int(cplx), H, W, _p(prm), _p(out), _p(Tf), _p(nc), _nthreads(nthreads))
    assert rc == 0
    val = out[..., 0] + 1j * out[..., 1] if cplx else out[..., 0]
    return dict(out=val, T_final=Tf, n_contrib=nc)


def parity_error(x, ref, absacc):
    """e = |x - ref| / max(A, 1e-30), A the absolute-sum magnitude."""
    return np.abs(np.asarray(x) - np.asarray(ref)) / np.maximum(absacc, 1e-30)
