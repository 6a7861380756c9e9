"""Oracle: adaptive densification, pruning and opacity reset (Sec. 4.2,
Algorithm 1's densify branch).  Test infrastructure: only tests/ may use it.

The paper gives the steps but no thresholds; the readings:
* the gradient statistic is the mean of |dL/dmu_i| over the steps in which
  Gaussian i was live (reached some pixel);
* "max(Sigma_i) <= epsilon r_scene" compares the largest per-axis scale
  exp(log_scale) with clone_extent = epsilon r_scene;
* "split into N children, scale Sigma_i / (0.8 N)": children's per-axis
  scale divided by 0.8 N (log_scale - log(0.8 N)), positions sampled from
  the parent, mu + R(q) (s * xi) with xi standard normals;
* the prune runs over the densified set: a parent is dropped when faint
  (sigmoid(opacity_logit) < opacity_min) or large (screen radius > r_max);
  its clone is dropped only when faint, split children likewise (new
  Gaussians have no screen radius yet); a split parent always leaves;
* the opacity reset caps sigma at 0.01 (in logit space).

The decisions are integer outcomes of floating-point comparisons: they are
taken in FP32, the kernels' precision (statistic acc / cnt, exp of the
largest log scale, the sigmoid); the displaced means in FP64.
"""
import numpy as np

KEEP, CLONE = -1, -2


def stats(d_mean, live, acc, cnt):
    """acc[i] += |d_mean[:, i]| and cnt[i] += 1 for every i in `live`
    (d_mean [3][n]).  Returns new (acc, cnt) (FP64, int)."""
    acc = np.asarray(acc, np.float64).copy()
    cnt = np.asarray(cnt, np.int64).copy()
    g = np.asarray(d_mean, np.float64)
    for i in np.asarray(live, np.int64):
        acc[i] += np.sqrt(g[0, i] ** 2 + g[1, i] ** 2 + g[2, i] ** 2)
        cnt[i] += 1
    return acc, cnt


def decisions(log_scale, opacity_logit, acc, cnt, radius, grad_threshold, clone_extent, opacity_min, radius_max):
    """Per Gaussian (densify, small, faint, large), in FP32."""
    f = np.float32
    ls = np.asarray(log_scale, f)
    acc32 = np.asarray(acc, f)
    cnt32 = np.asarray(cnt, f)
    with np.errstate(divide="ignore", invalid="ignore"):
        mean_g = np.where(cnt32 > 0, acc32 / np.maximum(cnt32, f(1)), f(0))
    densify = (np.asarray(cnt) > 0) & (mean_g >= f(grad_threshold))
    small = np.exp(ls.max(axis=0)) <= f(clone_extent)
    op = f(1) / (f(1) + np.exp(-np.asarray(opacity_logit, f)))
    faint = op < f(opacity_min)
    large = np.zeros_like(faint) if radius is None else np.asarray(radius, f) > f(radius_max)
    return densify, small, faint, large


def plan(log_scale, opacity_logit, acc, cnt, radius, grad_threshold, clone_extent, split_n, opacity_min,
         radius_max):
    """The new set's slots in parent order: (src, kind) int arrays."""
    densify, small, faint, large = decisions(log_scale, opacity_logit, acc, cnt, radius, grad_threshold,
                                             clone_extent, opacity_min, radius_max)
    src, kind = [], []
    for i in range(len(faint)):
        if not densify[i]:
            if not (faint[i] or large[i]):
                src.append(i)
                kind.append(KEEP)
        elif small[i]:
            if not (faint[i] or large[i]):
                src.append(i)
                kind.append(KEEP)
            if not faint[i]:
                src.append(i)
                kind.append(CLONE)
        elif not faint[i]:
            for k in range(split_n):
                src.append(i)
                kind.append(k)
    return np.asarray(src, np.int64), np.asarray(kind, np.int64)


def quat_to_R(q):
    """Rotation of the unit quaternion (w, x, y, z), normalised first."""
    w, x, y, z = np.asarray(q, np.float64) / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def apply(scene, src, kind, xi, split_n):
    """The new scene (FP64): parents copied; child k of parent i at
    mu_i + R(q_i) (exp(log_scale_i) * xi[i, k]), log scale minus
    log(0.8 split_n).  scene arrays in the scene's layout ([3][n] ...);
    xi [n][split_n][3]."""
    mean = np.asarray(scene["mean"], np.float64)
    ls = np.asarray(scene["log_scale"], np.float64)
    quat = np.asarray(scene["quat"], np.float64)
    op = np.asarray(scene["opacity_logit"], np.float64)
    m = len(src)
    out = {"mean": np.zeros((3, m)), "log_scale": np.zeros((3, m)), "quat": np.zeros((4, m)),
           "opacity_logit": np.zeros(m)}
    for j, (i, k) in enumerate(zip(src, kind)):
        mu, l = mean[:, i].copy(), ls[:, i].copy()
        if k >= 0:
            mu = mu + quat_to_R(quat[:, i]) @ (np.exp(l) * np.asarray(xi[i, k], np.float64))
            l = l - np.log(0.8 * split_n)
        out["mean"][:, j] = mu
        out["log_scale"][:, j] = l
        out["quat"][:, j] = quat[:, i]
        out["opacity_logit"][j] = op[i]
    return out


def gather(arr, src, kind, zero_new):
    """arr [comps][n][width] -> [comps][len(src)][width] in the new order,
    rows of clones and children zero when zero_new."""
    a = np.asarray(arr)
    out = a[:, src, :].copy()
    if zero_new:
        out[:, np.asarray(kind) != KEEP, :] = 0
    return out


def opacity_reset(opacity_logit, cap=0.01):
    """sigma <- min(sigma, cap) in logit space."""
    return np.minimum(np.asarray(opacity_logit, np.float64), np.log(cap / (1.0 - cap)))
