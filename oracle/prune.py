"""Shape reset and shape/opacity pruning of the GES training loop, plain numpy -- TEST INFRASTRUCTURE ONLY.

Only tests/, the package's smoke check and the benchmark's CPU baseline may use this module.

The paper controls the splat count by pruning on the shape parameter instead of a variable density
mechanism (Sec. 4.4), prunes every 100 iterations and resets the shape every 1,000 (Sec. 5.2; App. B.2), and
keeps the opacity pruning of Gaussian splatting.  It names the intervals and thresholds, not the
operations.  Readings:
* pruning removes every splat whose opacity sigmoid(logit) is below min_opacity or whose beta is below
  min_beta, and keeps the others in their original order, together with their optimiser moments;
* the opacity test is taken on the logit: sigmoid(x) < t  <=>  x < ln(t / (1 - t)), with the bound
  evaluated in binary64 and the binary32 logit widened to binary64 (a comparison, so both sides take the
  same decision);
* shape reset sets every beta to its initial value (2, the Gaussian) and clears beta's Adam moments.
"""
from __future__ import annotations

import math

import numpy as np

PARAMS = ("means", "log_scales", "quats", "opacity_logits", "sh", "beta")


def opacity_logit_bound(min_opacity: float) -> float:
    """The logit below which sigmoid(logit) < min_opacity (-inf for a bound of 0)."""
    if min_opacity <= 0.0:
        return -math.inf
    if min_opacity >= 1.0:
        return math.inf
    return math.log(min_opacity / (1.0 - min_opacity))


def keep_mask(opacity_logits: np.ndarray, beta: np.ndarray, min_opacity: float, min_beta: float) -> np.ndarray:
    """True for every splat that survives pruning, decided one splat at a time."""
    bound = opacity_logit_bound(min_opacity)
    n = len(beta)
    keep = np.zeros(n, bool)
    for i in range(n):
        x = float(np.float32(opacity_logits[i]))
        b = float(np.float32(beta[i]))
        keep[i] = (not x < bound) and (not b < min_beta)
    return keep


def prune(arrays: dict, moments: list[dict], min_opacity: float, min_beta: float):
    """Copies of ``arrays`` and of each moment dict (same keys) without the pruned splats, order kept."""
    keep = keep_mask(np.asarray(arrays["opacity_logits"]).ravel(), np.asarray(arrays["beta"]).ravel(),
                     min_opacity, min_beta)
    idx = [i for i in range(len(keep)) if keep[i]]
    out = {k: np.asarray(v)[idx] for k, v in arrays.items()}
    outm = [{k: np.asarray(v)[idx] for k, v in m.items()} for m in moments]
    return out, outm, keep


def shape_reset(beta: np.ndarray, exp_avg: np.ndarray, exp_avg_sq: np.ndarray, value: float = 2.0):
    """Every beta set to ``value``; its two Adam moments cleared."""
    return np.full_like(beta, value), np.zeros_like(exp_avg), np.zeros_like(exp_avg_sq)
