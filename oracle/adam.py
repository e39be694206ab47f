"""Bias-corrected Adam, the optimiser of the cited 3D-GS training (Sec. III).

Reading used: beta = (0.9, 0.999), eps = 1e-15, dense (every Gaussian, every
step), per-group learning rates; step t counts from 1:

    m = b1 m + (1 - b1) g;  v = b2 v + (1 - b2) g^2
    p = p - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
"""
from __future__ import annotations

import numpy as np

BETA1 = 0.9
BETA2 = 0.999
EPS = 1e-15

# group -> learning rate (the 3D-GS defaults; the means rate scales with the
# scene extent, 2.5 for the orbit radius used here)
DEFAULT_LR = {
    "means": 1.6e-4 * 2.5,
    "log_scales": 5e-3,
    "quats": 1e-3,
    "opacity_logits": 5e-2,
    "sh_dc": 2.5e-3,
    "sh_rest": 2.5e-3 / 20.0,
}


def adam_step(p, g, m, v, lr, t, b1=BETA1, b2=BETA2, eps=EPS):
    p = np.asarray(p, np.float64)
    g = np.asarray(g, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
