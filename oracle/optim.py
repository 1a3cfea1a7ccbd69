"""Optimiser of the GES training step (App. B.2), plain numpy in binary64 -- TEST INFRASTRUCTURE ONLY.

Only tests/, the package's smoke check and the benchmark's CPU baseline may use this module.

* Adam (Kingma & Ba, 2015, Algorithm 1) on every parameter group, with the bias corrections applied to
  the step: m <- b1 m + (1 - b1) g;  v <- b2 v + (1 - b2) g^2;
  p <- p - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps), at step t >= 1.
* Per-group learning rates of App. B.2: feature (all SH coefficients) 0.0025, opacity 0.05, shape (beta)
  0.001, rotation 0.001, scaling 0.005; position from 0.00016 down to 0.0000016 over 30,000 steps.
* Position learning-rate schedule: log-linear interpolation between the initial and final rates over
  max_steps (constant afterwards), times an optional delay factor that ramps from delay_mult to 1 along a
  quarter sine over delay_steps (no delay when delay_steps = 0).

Readings (the paper names the rates but not these details): Adam's b1 = 0.9, b2 = 0.999 and eps = 1e-15;
one feature rate for every SH coefficient; the position rates are used as given (a caller may scale them
by a scene extent); the delay multiplier 0.01 has no effect with delay_steps = 0.
"""
from __future__ import annotations

import math

import numpy as np

BETA1, BETA2, EPS = 0.9, 0.999, 1e-15
# App. B.2 learning rates per parameter group
LR = dict(means=0.00016, sh=0.0025, opacity_logits=0.05, beta=0.001, quats=0.001, log_scales=0.005)
LR_POS_FINAL = 0.0000016
LR_POS_MAX_STEPS = 30000
LR_DELAY_MULT = 0.01


def adam_step(p, g, m, v, t, lr, b1=BETA1, b2=BETA2, eps=EPS):
    """One Adam update of a parameter array at step t >= 1; returns new (p, m, v) in binary64."""
    p = np.asarray(p, np.float64)
    g = np.asarray(g, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1.0 - b2) * g * g
    m_hat = m / (1.0 - b1 ** t)
    v_hat = v / (1.0 - b2 ** t)
    return p - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


def expon_lr(step, lr_init, lr_final, max_steps, delay_steps=0, delay_mult=1.0):
    """Log-linear learning rate from lr_init (step 0) to lr_final (step max_steps), with optional delay."""
    if lr_init == lr_final:
        base = lr_init
    else:
        tau = min(max(step / max_steps, 0.0), 1.0)
        base = math.exp((1.0 - tau) * math.log(lr_init) + tau * math.log(lr_final))
    if delay_steps > 0:
        ramp = min(max(step / delay_steps, 0.0), 1.0)
        base *= delay_mult + (1.0 - delay_mult) * math.sin(0.5 * math.pi * ramp)
    return base


def position_lr(step, scale=1.0):
    """Position learning rate of App. B.2 at a step (optionally times a scene extent)."""
    return scale * expon_lr(step, LR["means"], LR_POS_FINAL, LR_POS_MAX_STEPS)
