"""Frequency-modulated loss of GES (Sec. 4.3), plain numpy -- TEST INFRASTRUCTURE ONLY.

Definitions:
* DoG_omega(I) = G(I, sigma1) - G(I, sigma2), sigma2 = 0.1 + 10 omega, sigma1 = 2 sigma2
  (Sec. 4.3, Eq. mask), applied to the grey level of the target after an area
  down-sampling by 0.2 (App. B.2: the image Laplacian scale factor), the mask then
  up-sampled back with nearest-neighbour lookup.
* M_omega = 1(|DoG_omega|/max|DoG_omega| > 0.5)  (threshold eps = 0.5).
* For 0 < omega <= 0.5 the mask is 1 - M_(omega + 0.5) (Sec. 4.3, last paragraph), M_(omega + 0.5) being the
  direct mask of the range 0.5 < omega + 0.5 <= 1.  omega = 0 is taken as the limit from above,
  1 - (direct mask at 0.5): the direct definition itself degenerates there (sigma2 = 0.1 gives a response
  below the flat-image floor on any image).
* L = lambda_1 mean|I - I_gt| + lambda_omega mean(|I - I_gt| M_omega)  (Eq. laplace, Eq. final;
  the SSIM term is not part of this loss).
Readings: the blur is a normalised sampled Gaussian of radius ceil(3 sigma) with
replicated borders; "normalised" divides by the maximum absolute response; grey
is the mean of R, G, B; the down-sampling averages each 5x5 block (partial blocks
at the border average the pixels they hold); a maximum response below 1e-5 (a
flat image up to rounding) gives an empty mask.
"""
from __future__ import annotations

import math

import numpy as np

SCALE_INV = 5  # 1 / 0.2
ZERO_RESPONSE = 1e-5


def gaussian_weights(sigma: float) -> np.ndarray:
    R = int(math.ceil(3.0 * sigma))
    k = np.arange(-R, R + 1, dtype=np.float64)
    w = np.exp(-(k * k) / (2.0 * sigma * sigma))
    return w / w.sum()


def blur(img: np.ndarray, sigma: float) -> np.ndarray:
    """Separable Gaussian blur of a 2-D array with replicated borders."""
    w = gaussian_weights(sigma)
    R = (len(w) - 1) // 2
    H, W = img.shape
    out = np.zeros_like(img, dtype=np.float64)
    xs = np.arange(W)
    for k in range(-R, R + 1):
        out += w[k + R] * img[:, np.clip(xs + k, 0, W - 1)]
    out2 = np.zeros_like(out)
    ys = np.arange(H)
    for k in range(-R, R + 1):
        out2 += w[k + R] * out[np.clip(ys + k, 0, H - 1), :]
    return out2


def downsample(grey: np.ndarray) -> np.ndarray:
    H, W = grey.shape
    Hl, Wl = (H + SCALE_INV - 1) // SCALE_INV, (W + SCALE_INV - 1) // SCALE_INV
    out = np.zeros((Hl, Wl))
    for y in range(Hl):
        for x in range(Wl):
            out[y, x] = grey[y * SCALE_INV:(y + 1) * SCALE_INV, x * SCALE_INV:(x + 1) * SCALE_INV].mean()
    return out


def dog_response(target: np.ndarray, omega: float) -> np.ndarray:
    """Normalised |DoG_omega| of the target's grey level, at the down-sampled resolution."""
    grey = np.asarray(target, np.float64).mean(axis=2)
    low = downsample(grey)
    s2 = 0.1 + 10.0 * omega
    s1 = 2.0 * s2
    resp = np.abs(blur(low, s1) - blur(low, s2))
    m = resp.max()
    # a response below 1e-5 is rounding noise of a flat image: no band-pass content, empty mask
    return resp / m if m > ZERO_RESPONSE else np.zeros_like(resp)


def freq_mask(target: np.ndarray, omega: float, eps: float = 0.5) -> np.ndarray:
    """M_omega as uint8 [H,W]."""
    if omega <= 0.5:
        return (1 - _direct_mask(target, omega + 0.5, eps)).astype(np.uint8)
    return _direct_mask(target, omega, eps)


def _direct_mask(target: np.ndarray, omega: float, eps: float) -> np.ndarray:
    """1(normalised |DoG_omega| > eps), up-sampled to the target's size."""
    H, W = target.shape[:2]
    low = dog_response(target, omega) > eps
    ys = np.arange(H) // SCALE_INV
    xs = np.arange(W) // SCALE_INV
    return low[ys[:, None], xs[None, :]].astype(np.uint8)


def loss_and_grad(img: np.ndarray, target: np.ndarray, mask: np.ndarray | None, lam_l1: float, lam_w: float):
    """L and dL/dI for L = lam_l1 mean|I-T| + lam_w mean(|I-T| M), mean over H*W*3; sign(0) = 0."""
    d = np.asarray(img, np.float64) - np.asarray(target, np.float64)
    n = d.size
    m = np.zeros(d.shape[:2]) if mask is None else mask.astype(np.float64)
    w = lam_l1 + lam_w * m[:, :, None]
    L = float((w * np.abs(d)).sum() / n)
    g = w * np.sign(d) / n
    return L, g
