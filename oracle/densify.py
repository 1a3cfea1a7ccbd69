"""Densification of the GES training loop, plain numpy -- TEST INFRASTRUCTURE ONLY.

Only tests/, the package's smoke check and the benchmark's CPU baseline may use this module.

GES keeps the densification of Gaussian splatting (Sec. 5.2: other design choices kept; App. B.2: from
iteration 500 to 15,000, every 100 iterations, gradient threshold 0.0003, percent dense 0.01, opacity reset
every 3,000).  The paper gives the numbers, not the operations; the readings taken:
* statistic: per iteration, every visible splat adds the norm of its mean-2D gradient in normalised device
  coordinates, ||(dL/du * W/2, dL/dv * H/2)|| (u, v in pixels), to an accumulator and 1 to a count;
* selection: splats whose mean statistic (accumulator / count, 0 when never visible) is >= the threshold;
* clone: a selected splat whose largest scale exp(log_scale) is <= percent_dense * extent is copied (the
  test is taken on the largest log-scale against ln(percent_dense * extent), and the mean statistic as
  accumulator / count, both in binary64, so GPU and oracle decide identically);
* split: a selected splat whose largest scale is above that is replaced by two children with means
  mu + R(q) (s * z_k) for given standard normal draws z_k (k = 0, 1; R(q) the rotation of the normalised
  quaternion, s the scales) and log-scales reduced by ln 1.6; every other parameter is copied;
* order: the unsplit splats in their order, then the clones in the order of their sources, then the two
  children of each split splat in the order of their sources;
* optimiser moments: kept splats keep theirs; clones and children start from zero;
* opacity reset: every opacity becomes min(opacity, 0.01) (taken on the logit) with its moments cleared.
"""
from __future__ import annotations

import math

import numpy as np

SPLIT_SCALE_DIV = 1.6   # 0.8 * 2 children
RESET_OPACITY = 0.01


def ndc_grad_norm(g_u: np.ndarray, g_v: np.ndarray, width: int, height: int) -> np.ndarray:
    """||(dL/du * W/2, dL/dv * H/2)|| in binary64."""
    a = np.asarray(g_u, np.float64) * (width / 2.0)
    b = np.asarray(g_v, np.float64) * (height / 2.0)
    return np.sqrt(a * a + b * b)


def accumulate(accum, count, g_u, g_v, visible, width, height):
    """New (accum, count) after one iteration's statistics."""
    add = np.where(visible, ndc_grad_norm(g_u, g_v, width, height), 0.0)
    return np.asarray(accum, np.float64) + add, np.asarray(count, np.float64) + visible.astype(np.float64)


def _rotation(q):
    w, x, y, z = np.asarray(q, np.float64) / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def classify(accum, count, log_scales, grad_threshold, scale_threshold):
    """Per splat: 0 kept as is, 1 cloned, 2 split."""
    n = len(accum)
    out = np.zeros(n, np.int8)
    log_bound = math.log(scale_threshold)
    for i in range(n):
        c = float(count[i])
        mean = float(accum[i]) / c if c > 0 else 0.0
        if not mean >= grad_threshold:
            continue
        lmax = max(float(v) for v in log_scales[i])
        out[i] = 1 if lmax <= log_bound else 2
    return out


def densify(arrays: dict, moments: list[dict], accum, count, normals, grad_threshold, scale_threshold):
    """Densified copies of the splat arrays and moments; normals [n, 2, 3] standard normal draws."""
    kind = classify(accum, count, arrays["log_scales"], grad_threshold, scale_threshold)
    n = len(kind)
    rows = {k: [] for k in arrays}
    mrows = [{k: [] for k in m} for m in moments]
    # unsplit splats (kept and cloned sources), in order, with their moments
    for i in range(n):
        if kind[i] != 2:
            for k in arrays:
                rows[k].append(np.asarray(arrays[k][i], np.float64))
            for m, mr in zip(moments, mrows):
                for k in m:
                    mr[k].append(np.asarray(m[k][i], np.float64))
    # clones, then split children, with zero moments
    new = []
    for i in range(n):
        if kind[i] == 1:
            new.append({k: np.asarray(arrays[k][i], np.float64) for k in arrays})
    for i in range(n):
        if kind[i] == 2:
            s = np.exp(np.asarray(arrays["log_scales"][i], np.float64))
            R = _rotation(arrays["quats"][i])
            for c in range(2):
                child = {k: np.asarray(arrays[k][i], np.float64) for k in arrays}
                child["means"] = np.asarray(arrays["means"][i], np.float64) + R @ (s * np.asarray(normals[i, c],
                                                                                                    np.float64))
                child["log_scales"] = np.asarray(arrays["log_scales"][i], np.float64) - math.log(SPLIT_SCALE_DIV)
                new.append(child)
    for child in new:
        for k in arrays:
            rows[k].append(child[k])
        for m, mr in zip(moments, mrows):
            for k in m:
                mr[k].append(np.zeros_like(np.asarray(m[k][0], np.float64)))
    out = {k: np.array(v) if v else np.zeros((0,) + np.asarray(arrays[k]).shape[1:]) for k, v in rows.items()}
    outm = [{k: np.array(v) if v else np.zeros((0,) + np.asarray(moments[j][k]).shape[1:]) for k, v in mr.items()}
            for j, mr in enumerate(mrows)]
    return out, outm, kind


def opacity_reset(opacity_logits, exp_avg, exp_avg_sq):
    """min(opacity, 0.01) on the logit; the opacity moments cleared."""
    bound = math.log(RESET_OPACITY / (1.0 - RESET_OPACITY))
    return np.minimum(np.asarray(opacity_logits, np.float64), bound), np.zeros_like(exp_avg), np.zeros_like(exp_avg_sq)
