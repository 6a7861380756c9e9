"""The allocation-free loss entry point (gs_loss_spectrum_noalloc) against
gs_loss_spectrum with caller scratch, through the C ABI: two calls in a row,
the second with a smaller input, so the device array keeps the first call's
sums when the second starts.  Loss and spatial means agree to FP32
summation order (both sum with float atomics); the gradient is elementwise
from those sums.  Also: sizes beyond the array are rejected on the host."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2511_22793_amd import _lib
from paper_2511_22793_amd.render import loss_spectrum

pytestmark = pytest.mark.gpu


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _noalloc(spec, tgt, is_complex, lam):
    B, F, H, W = spec.shape[:4]
    dev = spec.device
    loss = torch.full((B,), float("nan"), device=dev)
    hhat = torch.full((B, F, 2) if is_complex else (B, F), float("nan"), device=dev)
    d = torch.full_like(spec, float("nan"))
    stream = torch.cuda.current_stream(dev).cuda_stream
    st = _lib.lib().gs_loss_spectrum_noalloc(_ptr(spec), _ptr(tgt), B, F, int(is_complex), H, W, float(lam),
                                             _ptr(loss), _ptr(hhat), _ptr(d), ctypes.c_void_p(stream))
    assert st == _lib.GS_OK, st
    return loss, hhat, d


def _close(a, b, what, rtol=2e-5):
    a = a.double().cpu().numpy()
    b = b.double().cpu().numpy()
    scale = max(float(np.abs(b).max()), 1e-30)
    err = float(np.abs(a - b).max())
    assert err <= rtol * scale, "%s: max err %.3g vs scale %.3g" % (what, err, scale)


@pytest.mark.parametrize("cases", [[(16, 64, True, 90, 360), (4, 16, True, 45, 90)],
                                   [(8, 1, False, 90, 360), (2, 3, False, 17, 33)]])
def test_noalloc_loss_matches_scratch_entry_point_twice(cases):
    g = torch.Generator(device="cuda").manual_seed(5)
    for (B, F, cplx, H, W) in cases:
        shape = (B, F, H, W, 2) if cplx else (B, F, H, W)
        spec = torch.randn(shape, device="cuda", generator=g)
        tgt = torch.randn(shape, device="cuda", generator=g) * 0.5 + 0.1
        ref = loss_spectrum(spec, tgt, cplx, 1.0)
        got = _noalloc(spec, tgt, cplx, 1.0)
        torch.cuda.synchronize()
        for name, a, b in zip(("loss", "h_hat", "d_spectrum"), got, ref):
            assert torch.isfinite(a).all(), name
            _close(a, b, "%s B=%d F=%d %dx%d" % (name, B, F, H, W))


def test_noalloc_rejects_sizes_beyond_its_array():
    spec = torch.zeros(4, 1, 1, 1, 2, device="cuda")
    loss = torch.zeros(4, device="cuda")
    # n_sets * F * c * 3 > 65536 floats: rejected before any pointer is used
    B, F = 1, (65536 // 6) + 1
    st = _lib.lib().gs_loss_spectrum_noalloc(_ptr(spec), _ptr(spec), B, F, 1, 1, 1, 1.0, _ptr(loss), _ptr(loss),
                                             _ptr(spec), None)
    assert st == _lib.GS_ERR_CAPACITY
