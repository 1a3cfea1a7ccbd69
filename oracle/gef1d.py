"""1-D generalized exponential function and the paper's 1-D setup -- TEST INFRASTRUCTURE ONLY.

* GEF f(x | mu, alpha, beta, A) = A exp(-(|x - mu| / alpha)^beta)   (Sec. 3.1, Eq. gef)
* Theorem 1 (App. A.2): the L1 error of a square wave of amplitude A and width L
  approximated by A exp(-t^2/alpha^2) versus A exp(-(|t|/alpha)^beta); computed by
  quadrature over t >= 0 and doubled (symmetry).
* Mixtures (App. A.3): Gaussian mixture Eq. gaussianmixture and the generalized
  mixture Eq. genmixture, which coincide when every beta = 2.
* The six 1-D test signals of App. A.3.
* The approximate shape modification phi_rho(beta) = 2 / (1 + exp(-(rho beta - 2 rho)))
  (Sec. 4.2, Eq. approx) and the exact ratio Gamma(3/beta)/Gamma(1/beta) (Eq. probablity).
* The boundary-error bounds of App. B.1: (4 - pi)/pi and (pi - 2)/pi.
"""
from __future__ import annotations

import math

import numpy as np


def gef(x, mu=0.0, alpha=1.0, beta=2.0, A=1.0):
    return A * np.exp(-(np.abs(np.asarray(x, np.float64) - mu) / alpha) ** beta)


def phi_bar(beta, rho=0.1):
    beta = np.asarray(beta, np.float64)
    return 2.0 / (1.0 + np.exp(-(rho * beta - 2.0 * rho)))


def phi_exact(beta):
    return math.gamma(3.0 / beta) / math.gamma(1.0 / beta)


def _trapz(y, x):
    return float(np.sum((y[1:] + y[:-1]) * np.diff(x)) / 2.0)


def square_error(f, L=2.0, A=1.0, t_max=50.0, n=2_000_001):
    """E_f = int |S(t) - f(t)| dt for the square wave S = A on |t| < L/2 (Theorem 1)."""
    # integrate the two pieces separately so the jump of S sits on a grid boundary
    t1 = np.linspace(0.0, L / 2.0, n // 2)
    t2 = np.linspace(L / 2.0, t_max, n // 2)
    e1 = _trapz(np.abs(A - f(t1)), t1)
    e2 = _trapz(np.abs(f(t2)), t2)
    return 2.0 * (e1 + e2)


def theorem1_errors(alpha, beta, L=2.0, A=1.0):
    eg = square_error(lambda t: A * np.exp(-(t * t) / (alpha * alpha)), L, A)
    ef = square_error(lambda t: A * np.exp(-(np.abs(t) / alpha) ** beta), L, A)
    return eg, ef


def gmm(x, w, mu, sigma, eps=1e-8):
    x = np.asarray(x, np.float64)[:, None]
    return np.sum(w * np.exp(-((x - mu) ** 2) / (2.0 * sigma ** 2 + eps)), axis=1)


def gef_mixture(x, w, mu, sigma, beta, eps=1e-8):
    x = np.asarray(x, np.float64)[:, None]
    return np.sum(w * np.exp(-(np.abs(x - mu) ** beta) / (2.0 * sigma ** 2 + eps)), axis=1)


def signal(kind: str, x, width: float):
    x = np.asarray(x, np.float64)
    inside = (x > -width / 2.0) & (x < width / 2.0)
    if kind == "square":
        return inside.astype(np.float64)
    if kind == "triangle":
        return np.where(inside, width / 2.0 - np.abs(x), 0.0)
    if kind == "parabolic":
        return np.where(inside, (width / 2.0) ** 2 - x * x, 0.0)
    if kind == "half_sinusoid":
        return np.where(inside, np.sin((x + width / 2.0) * math.pi / width), 0.0)
    if kind == "exponential":
        return np.where(inside, np.exp(-np.abs(x)), 0.0)
    if kind == "gaussian":
        return np.exp(-(x * x) / (2.0 * width * width))
    raise ValueError(kind)


ETA_SQUARE_LARGER = (4.0 - math.pi) / math.pi
ETA_CIRCLE_LARGER = (math.pi - 2.0) / math.pi
