"""Structural-similarity term of the GES training loss, plain numpy in binary64 -- TEST INFRASTRUCTURE ONLY.

Only tests/, the package's smoke check and the benchmark's CPU baseline may use this module.

The training loss adds lambda_ssim L_ssim to the L1 and frequency-modulated terms, with lambda_ssim = 0.2 and
lambda_L1 = 1 - lambda_ssim - lambda_omega (Sec. 4.4, Eq. final; App. B.2).  The paper does not spell
SSIM out; this module takes the Gaussian-weighted SSIM of Wang et al. (2004):
  mu_x = w * x,  s_x = w * x^2 - mu_x^2,  s_xy = w * (x y) - mu_x mu_y   (and likewise for y),
  SSIM = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_x + s_y + C2)),
  L_ssim = 1 - mean of SSIM over every pixel and colour channel.
Readings: w is the 11x11 outer product of a sampled Gaussian with sigma 1.5 normalised to unit sum; each
colour channel is filtered on its own; the image is padded with zeros so the SSIM map has the image's size;
C1 = 0.01^2 and C2 = 0.03^2 (dynamic range 1).

Gradient (chain rule through the five local statistics): with A = dSSIM/dmu_x, B = dSSIM/d(w * x^2) and
Cxy = dSSIM/d(w * x y) at every pixel p, the derivative of sum_p SSIM(p) with respect to x(q) is
(w * A)(q) + 2 x(q) (w * B)(q) + y(q) (w * Cxy)(q), the filter again zero-padded (w is symmetric, so the
adjoint of the filter is the filter).
"""
from __future__ import annotations

import numpy as np

RADIUS, SIGMA = 5, 1.5
C1, C2 = 0.01 ** 2, 0.03 ** 2


def window() -> np.ndarray:
    """The 11x11 window: outer product of the normalised 1-D Gaussian."""
    k = np.arange(-RADIUS, RADIUS + 1, dtype=np.float64)
    g = np.exp(-(k * k) / (2.0 * SIGMA * SIGMA))
    g /= g.sum()
    return np.outer(g, g)


def local_mean(a: np.ndarray) -> np.ndarray:
    """w * a for a 2-D array: every output is the 121-tap weighted sum over the zero-padded input."""
    w = window()
    H, W = a.shape
    pad = np.zeros((H + 2 * RADIUS, W + 2 * RADIUS))
    pad[RADIUS:RADIUS + H, RADIUS:RADIUS + W] = a
    out = np.zeros((H, W))
    for dy in range(2 * RADIUS + 1):
        for dx in range(2 * RADIUS + 1):
            out += w[dy, dx] * pad[dy:dy + H, dx:dx + W]
    return out


def _stats(x, y):
    mx, my = local_mean(x), local_mean(y)
    sx = local_mean(x * x) - mx * mx
    sy = local_mean(y * y) - my * my
    sxy = local_mean(x * y) - mx * my
    return mx, my, sx, sy, sxy


def ssim_map(img: np.ndarray, target: np.ndarray) -> np.ndarray:
    """SSIM at every pixel and channel of two [H, W, 3] images."""
    img, target = np.asarray(img, np.float64), np.asarray(target, np.float64)
    out = np.zeros(img.shape)
    for c in range(img.shape[2]):
        mx, my, sx, sy, sxy = _stats(img[..., c], target[..., c])
        out[..., c] = ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sx + sy + C2))
    return out


def ssim_loss_and_grad(img: np.ndarray, target: np.ndarray):
    """L_ssim = 1 - mean SSIM and its derivative with respect to the rendered image [H, W, 3]."""
    img, target = np.asarray(img, np.float64), np.asarray(target, np.float64)
    N = img.size
    grad = np.zeros(img.shape)
    total = 0.0
    for c in range(img.shape[2]):
        x, y = img[..., c], target[..., c]
        mx, my, sx, sy, sxy = _stats(x, y)
        n1, n2 = 2 * mx * my + C1, 2 * sxy + C2
        d1, d2 = mx * mx + my * my + C1, sx + sy + C2
        s = n1 * n2 / (d1 * d2)
        total += s.sum()
        # partial derivatives of SSIM with respect to mu_x, w * x^2 and w * x y at each pixel
        dA = 2 * my * n2 / (d1 * d2) - 2 * mx * s / d1 + 2 * mx * s / d2 - 2 * my * n1 / (d1 * d2)
        dB = -s / d2
        dC = 2 * n1 / (d1 * d2)
        grad[..., c] = local_mean(dA) + 2 * x * local_mean(dB) + y * local_mean(dC)
    return 1.0 - total / N, -grad / N
