"""GPU attribute network (BF16 matrix cores) and fused Adam against the oracle.

Comparison protocol.  FP32 accumulation on the matrix cores and FP64
accumulation in the oracle round to BF16 differently only when a value lies
next to a BF16 rounding boundary.  So each layer is checked *re-anchored*: the
oracle recomputes it in FP64 from the GPU's own BF16 inputs of that layer;
BF16 codes must then be equal except for one-ulp differences at values whose
FP64 result lies within 1e-5 (relative) of a rounding boundary, and
continuous outputs must agree to 2e-5 relative.  An end-to-end comparison with
the unanchored oracle checks the whole chain to the BF16 flip bound.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import mlp_ref
from paper_2511_22793_amd import mlp as gm

pytestmark = pytest.mark.gpu

LO, HI = [-5.0, -5.0, 0.0], [5.0, 5.0, 3.0]


def bits_to_f64(t):
    b = t.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


def near_boundary(v, scale, rel=1e-5):
    """True where FP64 value v lies within rel * scale of a BF16 rounding
    boundary (scale: magnitude of the terms that formed v)."""
    v = np.asarray(v, np.float64)
    r = mlp_ref.bf16(v)
    _, e = np.frexp(np.where(r == 0, v, r))
    ulp = np.ldexp(1.0, e - 8)  # BF16 keeps 8 significant bits
    frac = np.abs(v - r) / ulp  # 0.5 at a boundary
    return np.abs(frac - 0.5) * ulp <= rel * np.maximum(scale, 1e-30)


def check_codes(gpu, ref_pre, label, max_frac=0.01, scale=None):
    """gpu: BF16 values; ref_pre: FP64 values before rounding."""
    ref = mlp_ref.bf16(ref_pre)
    diff = gpu != ref
    if diff.any():
        amb = near_boundary(ref_pre, np.abs(ref_pre) if scale is None else scale)
        assert np.all(amb[diff]), "%s: %d BF16 codes differ away from a rounding boundary" % (label, int((diff & ~amb).sum()))
        ulps = np.abs(gpu[diff] - ref[diff]) / np.maximum(np.abs(ref[diff]) * 2.0 ** -7, 1e-38)
        assert ulps.max() <= 1.01, "%s: code differs by more than one ulp" % label
    assert diff.mean() <= max_frac, "%s: %.3g of codes differ" % (label, diff.mean())


def test_mfma_operand_layout_probe():
    # the operand layout the network kernels assume, checked by a test-only
    # probe library (tests/probe) on small integers (exact in BF16 and FP32)
    import ctypes
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "probe", "libgsprobe.so")
    probe = ctypes.CDLL(path)
    probe.probe_mfma_bf16.restype = ctypes.c_int
    rng = np.random.default_rng(0)
    A = rng.integers(-8, 9, size=(16, 32)).astype(np.float32)
    B = rng.integers(-8, 9, size=(32, 16)).astype(np.float32)
    Ab = torch.from_numpy(gm.bf16_bits(A).view(np.int16)).cuda()
    Bb = torch.from_numpy(gm.bf16_bits(B).view(np.int16)).cuda()
    C = torch.empty(16, 16, device="cuda")
    torch.cuda.synchronize()
    assert probe.probe_mfma_bf16(ctypes.c_void_p(Ab.data_ptr()), ctypes.c_void_p(Bb.data_ptr()),
                                 ctypes.c_void_p(C.data_ptr())) == 0
    assert np.array_equal(C.cpu().numpy(), A @ B)


def setup(n=300, S=3, seed=0, shared=True, F=64):
    w = mlp_ref.init(seed)
    rng = np.random.default_rng(seed + 1)
    w["b1"] = rng.normal(0, 0.1, 64)
    w["b2"] = rng.normal(0, 0.1, 64)
    w["b3"] = rng.normal(0, 0.3, 2 * F)
    if F != 64:  # a network with F complex subcarriers: W3 [2F, 64]
        w["W3"] = rng.normal(0, np.sqrt(2.0 / 64), size=(2 * F, 64))
    E = synth.embeddings(n, seed=seed + 2)
    sc = synth.scene(n, seed=seed + 3)
    tx = synth.points(S, seed=seed + 4)
    net = gm.AttributeNet(w, LO, HI, 0.2)
    E_bf = torch.from_numpy(gm.bf16_bits(E).view(np.int16)).cuda()
    mean = torch.from_numpy(sc["mean"]).cuda()
    # rows: a seeded subset of Gaussians (shared by all sets, or one per set)
    if shared:
        lst = np.sort(rng.choice(n, size=n // 2, replace=False)).astype(np.uint32)
        L = torch.from_numpy(lst.view(np.int32)).cuda()
        cnt = torch.tensor([len(lst)], dtype=torch.int32).cuda()
        lists = [lst] * S
    else:
        lists = [np.sort(rng.choice(n, size=n // 2 - 7 * s, replace=False)).astype(np.uint32) for s in range(S)]
        arr = np.zeros((S, n // 2), np.uint32)
        for s in range(S):
            arr[s, :len(lists[s])] = lists[s]
        L = torch.from_numpy(arr.view(np.int32)).cuda()
        cnt = torch.tensor([len(x) for x in lists], dtype=torch.int32).cuda()
    rows = gm.Rows(torch.from_numpy(tx).cuda(), L, cnt, row_cap=n // 2)
    return dict(w=w, E=E, sc=sc, tx=tx, net=net, E_bf=E_bf, mean=mean, rows=rows, lists=lists, n=n, S=S, F=F)


@pytest.mark.parametrize("shared,F", [(True, 64), (False, 64), (True, 32)])
def test_forward_layers_reanchored_and_end_to_end(shared, F):
    d = setup(shared=shared, F=F)
    n, S = d["n"], d["S"]
    st = gm.State(S, n // 2)
    for t in (st.h1, st.h2):  # rows past a set's count are never written: keep them defined
        t.zero_()
    Z1 = gm.embed(d["net"], d["E_bf"])
    attr = torch.zeros(S, n, F, 2, device="cuda")
    gm.forward(d["net"], Z1, d["mean"], d["rows"], attr, st)
    torch.cuda.synchronize()
    w = d["w"]
    W1r, W2r, W3r = mlp_ref.bf16(w["W1"]), mlp_ref.bf16(w["W2"]), mlp_ref.bf16(w["W3"])
    Er = mlp_ref.bf16(d["E"])
    g = mlp_ref.bf16(mlp_ref.fourier(d["tx"], LO, HI))
    h1g, h2g = bits_to_f64(st.h1), bits_to_f64(st.h2)
    A = attr.cpu().numpy().astype(np.float64)
    full = mlp_ref.forward(w["W1"], w["b1"], w["W2"], w["b2"], w["W3"], w["b3"], d["E"], d["tx"], d["sc"]["mean"],
                           0.2, LO, HI, F=F)
    for s in range(S):
        lst = d["lists"][s]
        m = len(lst)
        x = np.concatenate([Er[lst], np.repeat(g[s][None], m, 0), np.zeros((m, 13))], 1)
        z1 = x @ W1r.T + w["b1"]
        check_codes(h1g[s, :m], np.maximum(z1, 0.0), "h1")
        z2 = h1g[s, :m] @ W2r.T + w["b2"]
        check_codes(h2g[s, :m], np.maximum(z2, 0.0), "h2")
        o = h2g[s, :m] @ W3r.T + w["b3"]
        dd = np.maximum(np.linalg.norm(d["sc"]["mean"][:, lst].T.astype(np.float64) - d["tx"][s].astype(np.float64), axis=1), 0.2)
        amp = 1 / (1 + np.exp(-(o[:, :F] - np.log(dd)[:, None])))
        ref = np.stack([amp * np.cos(o[:, F:]), amp * np.sin(o[:, F:])], -1)
        err = np.abs(A[s, lst] - ref) / np.maximum(amp[..., None], 1e-6)
        assert err.max() <= 2e-5, "attr re-anchored err %.3g" % err.max()
        # end to end against the unanchored oracle: BF16 flip bound
        e2 = np.abs(A[s, lst] - full["attr"][s, lst]) / np.maximum(full["amp"][s, lst][..., None], 1e-6)
        assert e2.max() <= 5e-2 and np.mean(e2 > 1e-4) <= 0.05
    # rows not listed stay untouched
    mask = np.ones(n, bool)
    mask[d["lists"][0]] = False
    assert np.all(A[0, mask] == 0)


@pytest.mark.parametrize("F", [64, 32])
def test_backward_reanchored(F):
    d = setup(n=256, S=3, seed=5, F=F)
    n, S = d["n"], d["S"]
    st = gm.State(S, n // 2, n_partial=8, n_chan=F)
    for t in (st.h1, st.h2, st.do, st.dz2, st.dz1):
        t.zero_()
    Z1 = gm.embed(d["net"], d["E_bf"])
    attr = torch.zeros(S, n, F, 2, device="cuda")
    gm.forward(d["net"], Z1, d["mean"], d["rows"], attr, st)
    rng = np.random.default_rng(9)
    dA = rng.normal(size=(S, n, F, 2)).astype(np.float32)
    gr = gm.backward(d["net"], d["E_bf"], d["mean"], d["rows"], torch.from_numpy(dA).cuda(), st)
    torch.cuda.synchronize()
    w = d["w"]
    W1r, W2r, W3r = mlp_ref.bf16(w["W1"]), mlp_ref.bf16(w["W2"]), mlp_ref.bf16(w["W3"])
    Er = mlp_ref.bf16(d["E"])
    g = mlp_ref.bf16(mlp_ref.fourier(d["tx"], LO, HI))
    h1g, h2g = bits_to_f64(st.h1), bits_to_f64(st.h2)
    dog, dz2g, dz1g = bits_to_f64(st.do), bits_to_f64(st.dz2), bits_to_f64(st.dz1)
    ref = {k: 0.0 for k in ("W3", "W2", "W1e", "b3", "b2")}
    dc = np.zeros((S, 64))
    dE = np.zeros((n, 32))
    lst = d["lists"][0]
    m = len(lst)
    for s in range(S):
        o = h2g[s, :m] @ W3r.T + w["b3"]
        dd = np.maximum(np.linalg.norm(d["sc"]["mean"][:, lst].T.astype(np.float64) - d["tx"][s].astype(np.float64), axis=1), 0.2)
        amp = 1 / (1 + np.exp(-(o[:, :F] - np.log(dd)[:, None])))
        ph = o[:, F:]
        gre, gim = dA[s, lst, :, 0].astype(np.float64), dA[s, lst, :, 1].astype(np.float64)
        do = np.concatenate([(gre * np.cos(ph) + gim * np.sin(ph)) * amp * (1 - amp),
                             amp * (-gre * np.sin(ph) + gim * np.cos(ph))], 1)
        mag = np.abs(gre) + np.abs(gim)
        do_scale = np.concatenate([mag * amp * (1 - amp), amp * mag], 1)
        check_codes(dog[s, :m], do, "d_o", max_frac=0.02, scale=do_scale)
        dz2 = (dog[s, :m] @ W3r) * (h2g[s, :m] > 0)
        check_codes(dz2g[s, :m], dz2, "dZ2", max_frac=0.02)
        dz1 = (dz2g[s, :m] @ W2r) * (h1g[s, :m] > 0)
        check_codes(dz1g[s, :m], dz1, "dZ1", max_frac=0.02)
        ref["W3"] = ref["W3"] + dog[s, :m].T @ h2g[s, :m]
        ref["W2"] = ref["W2"] + dz2g[s, :m].T @ h1g[s, :m]
        ref["W1e"] = ref["W1e"] + dz1g[s, :m].T @ Er[lst]
        ref["b3"] = ref["b3"] + do.sum(0)
        ref["b2"] = ref["b2"] + dz2.sum(0)
        dc[s] = dz1.sum(0)
        dE[lst] += dz1g[s, :m] @ W1r[:, :32]

    def close(got, want, label, tol=2e-4):
        got = got.cpu().numpy().astype(np.float64)
        scale = np.abs(want).max()
        assert np.abs(got - want).max() <= tol * scale + 1e-9, "%s err %.3g scale %.3g" % (
            label, np.abs(got - want).max(), scale)

    close(gr["W3"], ref["W3"], "dW3")
    close(gr["W2"], ref["W2"], "dW2")
    close(gr["W1"][:, :32], ref["W1e"], "dW1e")
    close(gr["W1"][:, 32:83], dc.T @ g, "dW1t", tol=2e-3)
    close(gr["b1"], dc.sum(0), "db1", tol=2e-3)
    close(gr["b3"], ref["b3"], "db3")
    close(gr["b2"], ref["b2"], "db2", tol=2e-3)
    close(gr["E"], dE, "dE")
    assert np.all(gr["W1"].cpu().numpy()[:, 83:] == 0)
    # end to end against the unanchored oracle (flip bound)
    full = mlp_ref.forward(w["W1"], w["b1"], w["W2"], w["b2"], w["W3"], w["b3"], d["E"], d["tx"], d["sc"]["mean"],
                           0.2, LO, HI, F=F)
    dmask = np.zeros_like(dA, dtype=np.float64)
    dmask[:, lst] = dA[:, lst]
    gfull = mlp_ref.backward(full, dmask, F=F)
    for k in ("W1", "W2", "W3", "b3", "E"):
        want = gfull[k]
        got = gr[k].cpu().numpy()
        assert np.abs(got - want).max() <= 2e-2 * np.abs(want).max(), k


def test_adam_matches_oracle_and_refreshes_bf16():
    rng = np.random.default_rng(11)
    shapes = [(1000,), (64, 96), (37,)]
    ps = [rng.normal(size=s).astype(np.float32) for s in shapes]
    state = [(np.zeros(s), np.zeros(s)) for s in shapes]
    tp = [torch.from_numpy(p.copy()).cuda() for p in ps]
    tm = [torch.zeros(s, device="cuda") for s in shapes]
    tv = [torch.zeros(s, device="cuda") for s in shapes]
    sh = torch.zeros(64, 96, dtype=torch.int16, device="cuda")
    lrs = [1e-3, 5e-3, 1.6e-4]
    ref = [p.astype(np.float64) for p in ps]
    for t in range(1, 6):
        gs_ = [rng.normal(size=s).astype(np.float32) for s in shapes]
        segs = [(tp[k], torch.from_numpy(gs_[k]).cuda(), tm[k], tv[k], sh if k == 1 else None, lrs[k]) for k in range(3)]
        gm.adam_step(segs, t)
        for k in range(3):
            ref[k], m, v = mlp_ref.adam(ref[k], gs_[k].astype(np.float64), state[k][0], state[k][1], t, lrs[k])
            state[k] = (m, v)
    torch.cuda.synchronize()
    for k in range(3):
        assert np.allclose(tp[k].cpu().numpy(), ref[k], rtol=1e-5, atol=1e-6)
    assert np.array_equal(sh.cpu().numpy().view(np.uint16), gm.bf16_bits(tp[1].cpu().numpy()))
