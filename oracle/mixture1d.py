"""The paper's 1-D mixture simulation, plain numpy in binary64 -- TEST INFRASTRUCTURE ONLY.

Only tests/, the package's smoke check and the benchmark's CPU baseline may use this module.

Four mixture models fitted to six 1-D signals (Sec. 3.2; App. A.3):
  GMM (Eq. gaussianmixture):  g(x) = sum_i w_i exp(-(x - mu_i)^2 / (2 s_i^2 + eps))
  DoG (variance ratio nu = 4): d(x) = sum_i w_i [exp(-(x - mu_i)^2 / (2 s_i^2 + eps))
                                                 - exp(-(x - mu_i)^2 / (2 s_i^2 / nu + eps))]
  LoG:                         l(x) = sum_i w_i (1 - (x - mu_i)^2 / s_i^2) exp(-(x - mu_i)^2 / (2 s_i^2 + eps))
  GEF (Eq. genmixture):        h(x) = sum_i w_i exp(-|x - mu_i|^beta_i / (2 s_i^2 + eps))
with eps = 1e-8, trained by Adam on the mean squared error over a linspace grid; a run whose final loss is
not finite counts as a NaN run.

Readings (the paper leaves these open): every component has its own beta; the parameters of a component
are (w_raw, mu, s, beta), with w = w_raw for unrestricted weights and w = softplus(w_raw) = ln(1 + e^w_raw)
for positive ones; at x = mu the GEF term's derivatives with respect to mu and beta are taken as 0 (the
limits of |d|^(beta-1) sign(d) for beta > 1 and of |d|^beta ln|d|); the gradient of every parameter is the
analytic derivative of the loss (the chain rule written out below, one component at a time).
"""
from __future__ import annotations

import numpy as np

from oracle import optim as OP

EPS = 1e-8
NU = 4.0
MODELS = ("gmm", "dog", "log", "gef")


def weight(w_raw, positive):
    """w and dw/dw_raw."""
    w_raw = np.asarray(w_raw, np.float64)
    if not positive:
        return w_raw, np.ones_like(w_raw)
    # softplus, written to stay finite for large |w_raw|
    w = np.where(w_raw > 30.0, w_raw, np.log1p(np.exp(np.minimum(w_raw, 30.0))))
    return w, 1.0 / (1.0 + np.exp(-w_raw))


def components(kind: str, x, theta, positive: bool):
    """Per-component values c_i(x) [M, N] and their derivatives [M, N, 4] w.r.t. (w_raw, mu, s, beta)."""
    x = np.asarray(x, np.float64)[:, None]
    theta = np.asarray(theta, np.float64)
    w_raw, mu, s, beta = theta[:, 0], theta[:, 1], theta[:, 2], theta[:, 3]
    w, dw = weight(w_raw, positive)
    d = x - mu
    d2 = d * d
    grad = np.zeros(d.shape + (4,))
    with np.errstate(all="ignore"):
        if kind in ("gmm", "dog", "log"):
            S1 = 2.0 * s * s + EPS
            E1 = np.exp(-d2 / S1)
            dE1_dmu = E1 * 2.0 * d / S1                 # d/dmu of exp(-(x-mu)^2/S1)
            dE1_ds = E1 * d2 * 4.0 * s / (S1 * S1)
            if kind == "gmm":
                base, dbase_dmu, dbase_ds = E1, dE1_dmu, dE1_ds
            elif kind == "dog":
                S2 = 2.0 * s * s / NU + EPS
                E2 = np.exp(-d2 / S2)
                base = E1 - E2
                dbase_dmu = dE1_dmu - E2 * 2.0 * d / S2
                dbase_ds = dE1_ds - E2 * d2 * (4.0 * s / NU) / (S2 * S2)
            else:
                P = 1.0 - d2 / (s * s)
                base = P * E1
                dbase_dmu = (2.0 * d / (s * s)) * E1 + P * dE1_dmu
                dbase_ds = (2.0 * d2 / (s * s * s)) * E1 + P * dE1_ds
            dbase_db = np.zeros_like(base)
        elif kind == "gef":
            S = 2.0 * s * s + EPS
            ad = np.abs(d)
            a = ad ** beta
            base = np.exp(-a / S)
            at_mu = ad == 0.0
            # d|d|^beta/dmu = -beta |d|^(beta-1) sign(d); d|d|^beta/dbeta = |d|^beta ln|d|  (0 at d = 0)
            da_dmu = np.where(at_mu, 0.0, -beta * ad ** (beta - 1.0) * np.sign(d))
            da_db = np.where(at_mu, 0.0, a * np.log(np.where(at_mu, 1.0, ad)))
            dbase_dmu = -base * da_dmu / S
            dbase_ds = base * a * 4.0 * s / (S * S)
            dbase_db = -base * da_db / S
        else:
            raise ValueError(kind)
        c = w * base
        grad[..., 0] = dw * base
        grad[..., 1] = w * dbase_dmu
        grad[..., 2] = w * dbase_ds
        grad[..., 3] = w * dbase_db
    return c, grad


def loss_and_grad(kind, x, y, theta, positive):
    """MSE = mean (model - y)^2 and its gradient [N, 4] (beta's is zero except for GEF)."""
    c, g = components(kind, x, theta, positive)
    r = c.sum(axis=1) - np.asarray(y, np.float64)
    M = len(r)
    with np.errstate(all="ignore"):
        loss = float(np.mean(r * r))
        grad = (2.0 / M) * np.einsum("m,mnk->nk", r, g)
    return loss, grad


def fit(kind, x, y, theta0, positive, epochs, lr, b1=0.9, b2=0.999, eps=1e-8):
    """Adam on the MSE for ``epochs`` steps; returns the final parameters and the loss of each epoch (taken
    before that epoch's update) and the loss after the last update."""
    theta = np.array(theta0, np.float64)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    losses = []
    for t in range(1, epochs + 1):
        loss, g = loss_and_grad(kind, x, y, theta, positive)
        losses.append(loss)
        theta, m, v = OP.adam_step(theta, g, m, v, t, lr, b1, b2, eps)
    final, _ = loss_and_grad(kind, x, y, theta, positive)
    return theta, losses, final
