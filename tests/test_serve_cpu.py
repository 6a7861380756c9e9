"""Host side of batched serving: the uneven serving mix, the forward-only
workspace and the batch entry points' argument checks (no device call)."""
import ctypes

import numpy as np
import pytest

import synth
from paper_2511_22793_amd import _lib
from paper_2511_22793_amd._lib import GsBatchInfo, GsBatchJob, GsLayout, GsQueries

from test_abi_cpu import FAKE, _valid_args, grid, params


def test_serving_mix_shape():
    mix = synth.serving_mix()
    assert len(mix) == 8
    assert sum(m["n_queries"] for m in mix) == 256 and min(m["n_queries"] for m in mix) >= 1
    for m in mix:
        assert m["n"] in (10_000, 30_000, 80_000, 150_000, 200_000)
        assert (m["H"], m["W"]) in ((90, 360), (180, 720))
        assert m["F"] in (1, 16, 64) and m["complex"] == (m["F"] > 1)
    assert mix == synth.serving_mix()  # seeded
    small = synth.serving_mix(n_queries=5, n_scenes=5, seed=7)
    assert sum(m["n_queries"] for m in small) == 5 and min(m["n_queries"] for m in small) == 1


def test_serving_arrays_follow_mix():
    mix = synth.serving_mix(n_queries=6, n_scenes=2, seed=3)
    arrs = synth.serving_arrays(mix, n_scale=0.01)
    for m, (sc, attr, rx, cplx, H, W) in zip(mix, arrs):
        n = int(round(m["n"] * 0.01))
        assert sc["mean"].shape == (3, n) and rx.shape == (m["n_queries"], 3)
        assert attr.shape == ((n, m["F"], 2) if cplx else (n, m["F"]))
        assert (H, W) == (m["H"], m["W"])


def _layout(p, n=100_000, B=4):
    out = GsLayout()
    assert _lib.lib().gs_workspace_layout(n, B, ctypes.byref(grid()), ctypes.byref(p), ctypes.byref(out)) == 0
    return out


def test_forward_only_workspace_is_smaller_and_rejects_backward():
    full = _layout(params())
    fwd = _layout(params(options=_lib.GS_OPT_FORWARD_ONLY))
    # the per-pair gradient accumulators (32 B per pair) are gone
    assert full.total - fwd.total >= 4 * full.pair_capacity * 32
    assert fwd.pair_list == full.pair_list and fwd.T_final == full.T_final
    # unknown option bits are rejected; the backward-decomposition bit is known
    assert _lib.lib().gs_workspace_layout(100, 1, ctypes.byref(grid()), ctypes.byref(params(options=8)),
                                          ctypes.byref(GsLayout())) == _lib.GS_ERR_INVALID_ARG
    assert _lib.lib().gs_workspace_layout(100, 1, ctypes.byref(grid()),
                                          ctypes.byref(params(options=_lib.GS_OPT_BWD_PER_GROUP)),
                                          ctypes.byref(GsLayout())) == _lib.GS_OK
    sc, at, q = _valid_args()
    p = params(options=_lib.GS_OPT_FORWARD_ONLY)
    st = _lib.lib().gs_render_backward(ctypes.byref(sc), ctypes.byref(at), ctypes.byref(q), 1,
                                       ctypes.byref(grid()), ctypes.byref(p), FAKE, FAKE, FAKE, FAKE, FAKE, FAKE,
                                       FAKE, 0, FAKE, 1 << 40, None)
    assert st == _lib.GS_ERR_INVALID_ARG
    st = _lib.lib().gs_render_live(100, 1, ctypes.byref(grid()), ctypes.byref(p), FAKE, 1 << 40, FAKE, 100, FAKE,
                                   None)
    assert st == _lib.GS_ERR_INVALID_ARG


def _jobs(k=2):
    jobs = (GsBatchJob * k)()
    for i in range(k):
        sc, at, q = _valid_args(100 * (i + 1))
        jobs[i].scene, jobs[i].attrs, jobs[i].queries = sc, at, q
        jobs[i].grid, jobs[i].params = grid(), params(options=_lib.GS_OPT_FORWARD_ONLY)
        jobs[i].spectrum = FAKE
        jobs[i].workspace = ctypes.c_void_p(0x100000)
        jobs[i].workspace_bytes = 1 << 40
    return jobs


def test_batch_plan_bytes():
    L = _lib.lib()
    assert L.gs_batch_plan_bytes(0) == 0
    assert L.gs_batch_plan_bytes(8) % 256 == 0 and L.gs_batch_plan_bytes(8) > L.gs_batch_plan_bytes(1) >= 256


def test_batch_rejects_on_host():
    L = _lib.lib()
    jobs = _jobs()
    info = GsBatchInfo()
    plan = ctypes.c_void_p(0x200000)
    nb = L.gs_batch_plan_bytes(2)
    assert L.gs_batch_plan(None, 2, plan, nb, ctypes.byref(info), None) == _lib.GS_ERR_INVALID_ARG
    assert L.gs_batch_plan(jobs, 0, plan, nb, ctypes.byref(info), None) == _lib.GS_ERR_INVALID_ARG
    assert L.gs_batch_plan(jobs, 2, plan, nb, None, None) == _lib.GS_ERR_INVALID_ARG
    assert L.gs_batch_plan(jobs, 2, ctypes.c_void_p(0x200010), nb, ctypes.byref(info), None) == \
        _lib.GS_ERR_WORKSPACE
    assert L.gs_batch_plan(jobs, 2, plan, nb - 1, ctypes.byref(info), None) == _lib.GS_ERR_WORKSPACE
    assert L.gs_batch_run(jobs, 2, plan, nb, 0, None, None) == _lib.GS_ERR_INVALID_ARG
    bad = _jobs()
    bad[1].workspace_bytes = 16
    assert L.gs_batch_run(bad, 2, plan, nb, 1024, None, None) == _lib.GS_ERR_WORKSPACE
    bad = _jobs()
    bad[0].queries = GsQueries(0, FAKE, None)
    assert L.gs_batch_run(bad, 2, plan, nb, 1024, None, None) == _lib.GS_ERR_INVALID_ARG
