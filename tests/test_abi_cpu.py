"""The C-ABI library loads on a machine without a GPU, exports every symbol
that include/gsparc.h declares, and rejects bad arguments on the host before
enqueuing anything (no device call is made by these tests)."""
import ctypes
import os
import re

import pytest

from paper_2511_22793_amd import _lib
from paper_2511_22793_amd._lib import GsAttrs, GsGrid, GsLayout, GsParams, GsQueries, GsScene

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "gsparc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(gs_[a-z_]+)\s*\(", text))
    return sorted(names)


def test_every_declared_symbol_is_exported_and_bound():
    L = _lib.lib()
    names = declared_symbols()
    assert len(names) >= 6
    for name in names:
        assert hasattr(L, name), name
        assert name in _lib.SIGNATURES, "binding missing for %s" % name


def grid(H=90, W=360, th=16, tw=16):
    g = GsGrid()
    _lib.lib().gs_default_grid(ctypes.byref(g), H, W)
    g.tile_h, g.tile_w = th, tw
    return g


def params(**kw):
    p = GsParams()
    _lib.lib().gs_default_params(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_defaults():
    p = params()
    assert p.alpha_min == pytest.approx(1 / 255) and p.alpha_max == pytest.approx(0.99)
    assert p.T_min == pytest.approx(1e-4) and p.dilation == pytest.approx(0.3) and p.r_near == pytest.approx(0.2)
    g = grid()
    assert list(g.view) == [0, 1, 0, 0, 0, 1, 1, 0, 0] and (g.tile_h, g.tile_w) == (16, 16)


@pytest.mark.parametrize("n,B,H,W", [(2048, 1, 90, 360), (100_000, 64, 90, 360), (300_000, 4, 180, 720)])
def test_layout(n, B, H, W):
    out = GsLayout()
    st = _lib.lib().gs_workspace_layout(n, B, ctypes.byref(grid(H, W)), ctypes.byref(params()), ctypes.byref(out))
    assert st == _lib.GS_OK
    assert out.tiles_x == (W + 15) // 16 and out.tiles_y == (H + 15) // 16
    assert out.total % 256 == 0 and out.total > n * B * 48
    T = out.tiles_x * out.tiles_y
    assert out.pair_capacity == n * min(T, 64) + 4096
    for f in ("flags", "rec", "rect", "order", "pair_list", "ranges", "T_final"):
        assert getattr(out, f) % 256 == 0


@pytest.mark.parametrize("bad", [dict(n=0), dict(B=0), dict(th=10, tw=10), dict(th=32, tw=32), dict(H=0)])
def test_layout_rejects(bad):
    a = dict(n=100, B=1, H=90, W=360, th=16, tw=16)
    a.update(bad)
    out = GsLayout()
    st = _lib.lib().gs_workspace_layout(a["n"], a["B"], ctypes.byref(grid(a["H"], a["W"], a["th"], a["tw"])),
                                        ctypes.byref(params()), ctypes.byref(out))
    assert st == _lib.GS_ERR_INVALID_ARG


def test_layout_rejects_key_overflow():
    # depth rank bits + tile bits must fit a 32-bit pair key
    out = GsLayout()
    st = _lib.lib().gs_workspace_layout(1 << 28, 1, ctypes.byref(grid(2048, 4096)), ctypes.byref(params()),
                                        ctypes.byref(out))
    assert st == _lib.GS_ERR_CAPACITY


FAKE = ctypes.c_void_p(0x10000)  # never dereferenced: validation fails first


def _forward(scene, attrs, queries, g, p, out, ws, nbytes):
    return _lib.lib().gs_render_forward(scene, attrs, queries, g, p, out, ws, nbytes, None)


def _valid_args(n=100):
    sc = GsScene(n, FAKE, FAKE, FAKE, FAKE)
    at = GsAttrs(1, 0, FAKE, 0)
    q = GsQueries(1, FAKE, None)
    return sc, at, q


def test_forward_rejects_null_and_bad_sizes_on_host():
    sc, at, q = _valid_args()
    g, p = grid(), params()
    L = _lib.lib()
    assert _forward(None, ctypes.byref(at), ctypes.byref(q), ctypes.byref(g), ctypes.byref(p), FAKE, FAKE, 1) == \
        _lib.GS_ERR_INVALID_ARG
    bad = GsScene(100, None, FAKE, FAKE, FAKE)
    assert _forward(ctypes.byref(bad), ctypes.byref(at), ctypes.byref(q), ctypes.byref(g), ctypes.byref(p), FAKE,
                    FAKE, 1) == _lib.GS_ERR_INVALID_ARG
    bad_at = GsAttrs(0, 0, FAKE, 0)
    assert _forward(ctypes.byref(sc), ctypes.byref(bad_at), ctypes.byref(q), ctypes.byref(g), ctypes.byref(p),
                    FAKE, FAKE, 1) == _lib.GS_ERR_INVALID_ARG
    bad_q = GsQueries(0, FAKE, None)
    assert _forward(ctypes.byref(sc), ctypes.byref(at), ctypes.byref(bad_q), ctypes.byref(g), ctypes.byref(p),
                    FAKE, FAKE, 1) == _lib.GS_ERR_INVALID_ARG
    bad_p = params(alpha_max=1.5)
    assert _forward(ctypes.byref(sc), ctypes.byref(at), ctypes.byref(q), ctypes.byref(g), ctypes.byref(bad_p),
                    FAKE, FAKE, 1) == _lib.GS_ERR_INVALID_ARG
    assert L.gs_status_string(_lib.GS_ERR_WORKSPACE)


def test_forward_rejects_small_or_misaligned_workspace_on_host():
    sc, at, q = _valid_args()
    g, p = grid(), params()
    out = GsLayout()
    assert _lib.lib().gs_workspace_layout(100, 1, ctypes.byref(g), ctypes.byref(p), ctypes.byref(out)) == 0
    args = (ctypes.byref(sc), ctypes.byref(at), ctypes.byref(q), ctypes.byref(g), ctypes.byref(p), FAKE)
    assert _forward(*args, FAKE, out.total - 1) == _lib.GS_ERR_WORKSPACE
    assert _forward(*args, ctypes.c_void_p(0x10010), out.total) == _lib.GS_ERR_WORKSPACE
    assert _forward(*args, None, out.total) == _lib.GS_ERR_WORKSPACE


def test_python_binding_fails_loudly_without_library(monkeypatch):
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", "/nonexistent/libgsparc.so")
    with pytest.raises(RuntimeError, match="not built"):
        _lib.lib()


def test_kernel_timing_api_on_host():
    # enabling, disabling and reading with no launch recorded needs no device
    L = _lib.lib()
    tot, cnt = ctypes.c_double(), ctypes.c_int64()
    assert L.gs_timing_enable(0) == _lib.GS_OK
    assert L.gs_timing_read(0, ctypes.byref(tot), ctypes.byref(cnt)) == _lib.GS_OK and cnt.value == 0
    assert L.gs_timing_read(1, ctypes.byref(tot), ctypes.byref(cnt)) == _lib.GS_OK and tot.value == 0.0
    assert L.gs_timing_read(2, ctypes.byref(tot), ctypes.byref(cnt)) == _lib.GS_OK and cnt.value == 0
    assert L.gs_timing_read(3, ctypes.byref(tot), ctypes.byref(cnt)) == _lib.GS_ERR_INVALID_ARG
    assert L.gs_timing_read(0, None, ctypes.byref(cnt)) == _lib.GS_ERR_INVALID_ARG


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr


def _train(sc, at, q, S, g, p, tt, flags=0, ws_bytes=None, scratch_bytes=None):
    L = _lib.lib()
    out = GsLayout()
    assert L.gs_workspace_layout(sc.n, q.count, ctypes.byref(g), ctypes.byref(p), ctypes.byref(out)) == 0
    ws_bytes = out.total if ws_bytes is None else ws_bytes
    need = L.gs_train_scratch_bytes(S, at.n_chan, ctypes.byref(g))
    scratch_bytes = need if scratch_bytes is None else scratch_bytes
    return L.gs_render_train(ctypes.byref(sc), ctypes.byref(at), ctypes.byref(q), S, ctypes.byref(g),
                             ctypes.byref(p), FAKE, FAKE, tt, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, flags,
                             ctypes.c_void_p(0x100000), ws_bytes, ctypes.c_void_p(0x200000), scratch_bytes, None)


def test_train_pass_rejects_bad_arguments_on_host():
    sc = GsScene(100, FAKE, FAKE, FAKE, FAKE)
    q = GsQueries(1, FAKE, None)
    g, p = grid(), params()
    at = GsAttrs(8, 1, FAKE, 100 * 16)
    tt = ctypes.byref(_lib.GsTrainTarget(FAKE, FAKE, 1.0, FAKE, FAKE))
    L = _lib.lib()
    # scratch size: GV partials per (64-pixel group, column range) dominate
    need = L.gs_train_scratch_bytes(4, 8, ctypes.byref(g))
    assert need >= 138 * 4 * 64 * 64 * 4 and need % 256 == 0
    assert L.gs_train_scratch_bytes(0, 8, ctypes.byref(g)) == 0
    assert _train(sc, at, q, 4, g, p, None) == _lib.GS_ERR_INVALID_ARG
    assert _train(sc, GsAttrs(8, 0, FAKE, 800), q, 4, g, p, tt) == _lib.GS_ERR_INVALID_ARG      # real attributes
    assert _train(sc, GsAttrs(4, 1, FAKE, 800), q, 4, g, p, tt) == _lib.GS_ERR_INVALID_ARG      # 2F not 16k
    assert _train(sc, at, GsQueries(2, FAKE, None), 4, g, p, tt) == _lib.GS_ERR_INVALID_ARG     # two receivers
    assert _train(sc, at, q, 4, g, params(atten_ref=1), tt) == _lib.GS_ERR_INVALID_ARG
    assert _train(sc, at, q, 4, g, params(options=_lib.GS_OPT_FORWARD_ONLY), tt) == _lib.GS_ERR_INVALID_ARG
    assert _train(sc, at, q, 4, g, p, tt, flags=8) == _lib.GS_ERR_INVALID_ARG
    bad_tt = ctypes.byref(_lib.GsTrainTarget(FAKE, None, 1.0, FAKE, FAKE))
    assert _train(sc, at, q, 4, g, p, bad_tt) == _lib.GS_ERR_INVALID_ARG
    assert _train(sc, at, q, 4, g, p, tt, scratch_bytes=need - 1) == _lib.GS_ERR_WORKSPACE
    assert _train(sc, at, q, 4, g, p, tt, ws_bytes=100) == _lib.GS_ERR_WORKSPACE


def test_train_geometry_rejects_bad_arguments_on_host():
    L = _lib.lib()
    sc = GsScene(100, FAKE, FAKE, FAKE, FAKE)
    q = GsQueries(1, FAKE, None)
    g, p = grid(), params()
    out = GsLayout()
    assert L.gs_workspace_layout(100, 1, ctypes.byref(g), ctypes.byref(p), ctypes.byref(out)) == 0

    def call(sc_=sc, q_=q, p_=p, d=FAKE, ws=ctypes.c_void_p(0x100000), nb=out.total):
        return L.gs_render_train_geometry(ctypes.byref(sc_), ctypes.byref(q_), ctypes.byref(g), ctypes.byref(p_), d,
                                          FAKE, FAKE, FAKE, ws, nb, None)
    assert call(d=None) == _lib.GS_ERR_INVALID_ARG
    assert call(sc_=GsScene(100, None, FAKE, FAKE, FAKE)) == _lib.GS_ERR_INVALID_ARG
    assert call(q_=GsQueries(2, FAKE, None)) == _lib.GS_ERR_INVALID_ARG          # one receiver only
    assert call(p_=params(options=_lib.GS_OPT_FORWARD_ONLY)) == _lib.GS_ERR_INVALID_ARG
    assert call(nb=out.total - 1) == _lib.GS_ERR_WORKSPACE
    assert call(ws=ctypes.c_void_p(0x100010)) == _lib.GS_ERR_WORKSPACE           # not 256-byte aligned


def test_spatial_mean_rejects_bad_arguments_on_host():
    L = _lib.lib()
    assert L.gs_spatial_mean(None, 1, 1, 0, 4, 4, FAKE, None) == _lib.GS_ERR_INVALID_ARG
    assert L.gs_spatial_mean(FAKE, 1, 0, 0, 4, 4, FAKE, None) == _lib.GS_ERR_INVALID_ARG
    assert L.gs_spatial_mean(ctypes.c_void_p(0x10004), 1, 1, 1, 4, 4, FAKE, None) == _lib.GS_ERR_INVALID_ARG
    assert L.gs_spatial_mean(FAKE, 1, 70000, 0, 4, 4, FAKE, None) == _lib.GS_ERR_CAPACITY


def test_l1_ssim_rejects_bad_arguments_on_host():
    L = _lib.lib()
    need = L.gs_loss_l1_ssim_scratch_bytes(2, 3, 90, 360)
    assert need == 2 * 3 * 12 * 6 * 2 * 4 + (-(2 * 3 * 12 * 6 * 2 * 4) % 256)
    args = lambda **kw: dict(dict(sp=FAKE, tg=FAKE, S=2, F=3, H=90, W=360, lam=0.2, sc=ctypes.c_void_p(0x100000),
                                  nb=need), **kw)

    def call(a):
        return L.gs_loss_l1_ssim(a["sp"], a["tg"], a["S"], a["F"], a["H"], a["W"], a["lam"], FAKE, None, None, None,
                                 a["sc"], a["nb"], None)
    assert call(args(sp=None)) == _lib.GS_ERR_INVALID_ARG
    assert call(args(lam=1.5)) == _lib.GS_ERR_INVALID_ARG
    assert call(args(H=0)) == _lib.GS_ERR_INVALID_ARG
    assert call(args(nb=need - 1)) == _lib.GS_ERR_WORKSPACE
    assert call(args(sc=ctypes.c_void_p(0x100010))) == _lib.GS_ERR_WORKSPACE
    assert call(args(S=300, F=300)) == _lib.GS_ERR_CAPACITY


def test_confidence_rejects_bad_arguments_on_host():
    L = _lib.lib()
    assert L.gs_confidence_scratch_bytes(4096) == 0
    need = L.gs_confidence_scratch_bytes(4097)
    assert need == 17 * 192 * 4  # 17 chunks of 256 samples, one workgroup each: their partials
    assert L.gs_confidence_scratch_bytes(1 << 24) == 1024 * 192 * 4
    w = [FAKE] * 4

    def call(n, sc=ctypes.c_void_p(0x100000), nb=None, alpha=0.3):
        return L.gs_confidence_loss(FAKE, FAKE, n, *w, alpha, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, sc,
                                    need if nb is None else nb, None)
    assert call(0) == _lib.GS_ERR_INVALID_ARG
    assert call(10, alpha=-1.0) == _lib.GS_ERR_INVALID_ARG
    assert call((1 << 24) + 1) == _lib.GS_ERR_CAPACITY
    assert call(4097, sc=None) == _lib.GS_ERR_WORKSPACE
    assert call(4097, nb=need - 1) == _lib.GS_ERR_WORKSPACE
    assert call(4097, sc=ctypes.c_void_p(0x100010)) == _lib.GS_ERR_WORKSPACE
