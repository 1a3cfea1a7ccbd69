"""Central finite differences of the binary64 oracle (test infrastructure).

The loss is the linear functional <g, image> for a fixed random g, so its gradient is exactly what the
backward pass returns for dL/dimage = g.  Each scalar parameter theta is perturbed by
h = 1e-6 max(1, |theta|) in binary64; a perturbation that changes any decision (which pairs are
composited, where a pixel terminates, which alphas are clamped) is excluded and counted.
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as O
from oracle import preprocess_f64 as PF

PARAMS = ["means", "log_scales", "quats", "opacity_logits", "sh", "beta"]


def render_loss(arrays64, sh_degree, cam, falloff, base_rec, g, rho=0.1):
    P = PF.to_params(arrays64)
    out = PF.preprocess(P, sh_degree, cam, falloff, rho, base_rec.clamp_bits)
    rec = PF.record_from(out, base_rec)
    orc = O.Oracle({k: np.zeros((1,) + v.shape[1:], np.float32) for k, v in arrays64.items()}, sh_degree, cam,
                   falloff=falloff, rho=rho)
    res = orc.render_untiled(rec, O.MODE_F64)
    return float((res["img"] * g).sum()), res["stats"]["decision_hash"]


def central_fd(arrays, sh_degree, cam, falloff, g, picks, rho=0.1):
    """picks: list of (name, index tuple).  Returns list of (fd value or None if excluded)."""
    arrays64 = {k: np.asarray(v, np.float64).copy() for k, v in arrays.items()}
    orc = O.Oracle(arrays, sh_degree, cam, falloff=falloff, rho=rho)
    base = orc.preprocess(O.MODE_F64)
    _, h0 = render_loss(arrays64, sh_degree, cam, falloff, base, g, rho)
    out = []
    for name, idx in picks:
        x0 = arrays64[name][idx]
        h = 1e-6 * max(1.0, abs(x0))
        vals, ok = [], True
        for sgn in (1.0, -1.0):
            arrays64[name][idx] = x0 + sgn * h
            L, hh = render_loss(arrays64, sh_degree, cam, falloff, base, g, rho)
            ok = ok and hh == h0
            vals.append(L)
        arrays64[name][idx] = x0
        out.append((vals[0] - vals[1]) / (2 * h) if ok else None)
    return out, base


def random_picks(arrays, visible, count, seed):
    rng = np.random.default_rng(seed)
    vis = np.nonzero(visible)[0]
    picks = []
    for k in range(count):
        name = PARAMS[k % len(PARAMS)]
        i = int(rng.choice(vis))
        shape = arrays[name].shape[1:]
        picks.append((name, (i,) + tuple(int(rng.integers(0, s)) for s in shape)))
    return picks
