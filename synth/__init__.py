"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only draws random numbers and lays them out; it holds none of the
renderer's arithmetic (no projection, no compositing, no activation). Every
array is float32 because that is the precision the renderer receives; the
oracle widens them to float64 itself.

Workload shapes follow the synthetic stand-ins for the paper's scenes
(Sec. 5: an indoor room a few metres across, a fixed receiver or transmitter,
tens of subcarriers around 2.4 GHz, up to ~1e5 Gaussians):

* means uniform in a 10 x 10 x 3 m box [-5,5] x [-5,5] x [0,3], z up, the
  receiver at the floor centre (0, 0, 0);
* log-scales N(-1.5, 0.5) per axis;
* quaternions uniform on the unit 3-sphere (normalised N(0, I4)), stored
  (w, x, y, z);
* opacity logits N(0, 1);
* one scalar RSS attribute per Gaussian, U(0, 1).

Layout: Gaussian parameters are structure-of-arrays, ``mean[3][n]``,
``log_scale[3][n]``, ``quat[4][n]``, ``opacity_logit[n]``; attributes are
``attr[n][F]`` (real) or ``attr[n][F][2]`` (complex, interleaved re/im).
"""
from __future__ import annotations

import numpy as np

BOX_LO = np.array([-5.0, -5.0, 0.0])
BOX_HI = np.array([5.0, 5.0, 3.0])

SEED_SCENE = 0
SEED_QUERIES = 1
SEED_PERTURB = 2
SEED_GT_SCENE = 3
SEED_SERVING = 4


def scene(n: int, seed: int = SEED_SCENE, lo=BOX_LO, hi=BOX_HI,
          log_scale_mean: float = -1.5, log_scale_sd: float = 0.5) -> dict:
    """Random Gaussians: SoA float32 arrays (see module docstring)."""
    rng = np.random.default_rng(seed)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    mean = (lo[:, None] + (hi - lo)[:, None] * rng.random((3, n))).astype(np.float32)
    log_scale = rng.normal(log_scale_mean, log_scale_sd, size=(3, n)).astype(np.float32)
    q = rng.normal(size=(4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    quat = q.astype(np.float32)
    opacity_logit = rng.normal(0.0, 1.0, size=n).astype(np.float32)
    return {"mean": np.ascontiguousarray(mean), "log_scale": np.ascontiguousarray(log_scale),
            "quat": np.ascontiguousarray(quat), "opacity_logit": opacity_logit}


def rss_attrs(n: int, seed: int = SEED_SCENE + 100) -> np.ndarray:
    """One real attribute per Gaussian, U(0, 1): float32 [n, 1]."""
    rng = np.random.default_rng(seed)
    return rng.random((n, 1)).astype(np.float32)


def channel_attrs(n: int, f: int, complex_: bool, seed: int = SEED_SCENE + 200,
                  scale: float = 1.0) -> np.ndarray:
    """F channels per Gaussian. Real: U(0,1) [n, F]; complex: unit-disk-ish
    N(0, 0.5) re/im interleaved [n, F, 2]."""
    rng = np.random.default_rng(seed)
    if complex_:
        return (scale * rng.normal(0.0, 0.5, size=(n, f, 2))).astype(np.float32)
    return (scale * rng.random((n, f))).astype(np.float32)


def points(b: int, seed: int = SEED_QUERIES, lo=BOX_LO, hi=BOX_HI) -> np.ndarray:
    """b positions uniform in the box: float32 [b, 3]."""
    rng = np.random.default_rng(seed)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    return (lo + (hi - lo) * rng.random((b, 3))).astype(np.float32)


def subset(n: int, k: int, seed: int) -> np.ndarray:
    """k distinct Gaussian indices out of n, sorted: int64 [k]."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=k, replace=False))


def perturbation(n: int, seed: int = SEED_PERTURB) -> dict:
    """Additive perturbation draws used to build a target scene: means
    +N(0, 0.05 m), log-scales +N(0, 0.1), logits +N(0, 0.3), attributes
    +N(0, 0.05). Returned as raw draws; the caller adds them."""
    rng = np.random.default_rng(seed)
    return {"mean": rng.normal(0.0, 0.05, size=(3, n)).astype(np.float32),
            "log_scale": rng.normal(0.0, 0.1, size=(3, n)).astype(np.float32),
            "opacity_logit": rng.normal(0.0, 0.3, size=n).astype(np.float32),
            "attr_sd": 0.05,
            "rng": rng}


def embeddings(n: int, dim: int = 32, seed: int = SEED_SCENE + 300, sd: float = 0.1) -> np.ndarray:
    """Per-Gaussian embedding N(0, sd^2 I): float32 [n, dim]."""
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, sd, size=(n, dim)).astype(np.float32)


def mlp_init(sizes, seed: int = SEED_SCENE + 400, gain: float = 1.0) -> list:
    """He-style normal init for a stack of linear layers: list of
    (W [out, in] float32, b [out] float32)."""
    rng = np.random.default_rng(seed)
    layers = []
    for fan_in, fan_out in zip(sizes[:-1], sizes[1:]):
        w = rng.normal(0.0, gain * np.sqrt(2.0 / fan_in), size=(fan_out, fan_in)).astype(np.float32)
        b = np.zeros(fan_out, dtype=np.float32)
        layers.append((w, b))
    return layers


def uniform(shape, lo: float, hi: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return (lo + (hi - lo) * rng.random(shape)).astype(np.float32)


def normal(shape, sd: float, seed: int, mean: float = 0.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.normal(mean, sd, size=shape).astype(np.float32)


def serving_mix(n_queries: int = 256, n_scenes: int = 8, sizes=(10_000, 30_000, 80_000, 150_000, 200_000),
                grids=((90, 360), (180, 720)), chans=(1, 16, 64), seed: int = SEED_SERVING) -> list:
    """An uneven serving batch: n_scenes scenes whose Gaussian count, grid
    (1 or 0.5 degree) and channel count are drawn uniformly from the given
    sets, and n_queries receivers each assigned to a uniformly drawn scene
    (every scene keeps at least one).  One channel is a real RSS value, more
    are complex subcarriers.  Returns one dict per scene: n, H, W, F,
    complex, n_queries, scene_seed, query_seed, attr_seed."""
    rng = np.random.default_rng(seed)
    n = rng.choice(np.asarray(sizes), size=n_scenes)
    g = rng.integers(0, len(grids), size=n_scenes)
    f = rng.choice(np.asarray(chans), size=n_scenes)
    owner = rng.integers(0, n_scenes, size=n_queries)
    counts = np.bincount(owner, minlength=n_scenes)
    for s_ in range(n_scenes):  # move a query from the largest group to an empty one
        if counts[s_] == 0:
            counts[np.argmax(counts)] -= 1
            counts[s_] = 1
    out = []
    for s_ in range(n_scenes):
        H, W = grids[g[s_]]
        out.append({"n": int(n[s_]), "H": int(H), "W": int(W), "F": int(f[s_]), "complex": bool(f[s_] > 1),
                    "n_queries": int(counts[s_]), "scene_seed": seed * 1000 + s_,
                    "query_seed": seed * 1000 + 100 + s_, "attr_seed": seed * 1000 + 200 + s_})
    return out


def serving_arrays(mix: list, n_scale: float = 1.0) -> list:
    """Host arrays of a serving mix: per scene (scene, attr, rx, complex, H,
    W), the scene recipe of the other workloads with n scaled by n_scale,
    shared attributes and receivers uniform in the room."""
    out = []
    for m in mix:
        n = max(1, int(round(m["n"] * n_scale)))
        out.append((scene(n, seed=m["scene_seed"]), channel_attrs(n, m["F"], m["complex"], seed=m["attr_seed"]),
                    points(m["n_queries"], seed=m["query_seed"]), m["complex"], m["H"], m["W"]))
    return out


def ground_truth_attributes(scene: dict, rho: np.ndarray, tx: np.ndarray, r_near: float = 0.2,
                            f_c: float = 2.4e9, df: float = 312.5e3, nf: int = 64) -> np.ndarray:
    """Target emissions for the learned-attribute workloads (a stand-in for
    measured channels): Gaussian reflectivity rho_i times the baseband delay
    phase and free-space loss of the transmitter leg (the multipath model
    reduced to one bounce per Gaussian),
    c_i[k] = rho_i exp(-j 2 pi (f_k - f_c) d_i / c0) / max(d_i, r_near),
    f_k = f_c + (k - (nf-1)/2) df.  Returns [S, n, nf, 2] float32."""
    c0 = 299_792_458.0
    m = np.asarray(scene["mean"], np.float64).T
    d = np.linalg.norm(m[None] - np.asarray(tx, np.float64)[:, None], axis=-1)      # [S, n]
    fk = (np.arange(nf) - (nf - 1) / 2.0) * df
    ph = -2.0 * np.pi * fk[None, None, :] * d[..., None] / c0
    a = np.asarray(rho, np.float64)[None, :, None] / np.maximum(d, r_near)[..., None]
    return np.stack([a * np.cos(ph), a * np.sin(ph)], -1).astype(np.float32)
