"""Seeded Gaussian parameter draws for the synthetic scenes.

The draws follow the workload recipes: means at isosurface points, log-scales
either constant (log of the grid spacing) or drawn per axis, identity or random
unit quaternions, a constant opacity logit, and SH coefficients either zero
(DC only) or N(0, sigma).  Layout is structure-of-arrays, float32:

    means[3][N], log_scales[3][N], quats[4][N] (w, x, y, z),
    opacity_logits[N], sh[(d+1)^2 * 3][N] with row index j*3 + c.
"""
from __future__ import annotations

import numpy as np


def n_sh_rows(degree: int) -> int:
    return (degree + 1) ** 2 * 3


def synth_params(rng, points, *, sh_degree, log_scale=None, log_scale_range=None,
                 log_scale_jitter=None, random_quats=False, opacity_logit=0.1,
                 opacity_logit_range=None, sh_std=0.0):
    pts = np.asarray(points, np.float64)
    n = pts.shape[0]
    means = pts.T.astype(np.float32).copy()
    if log_scale_range is not None:
        ls = rng.uniform(log_scale_range[0], log_scale_range[1], size=(3, n))
    else:
        ls = np.full((3, n), float(log_scale))
        if log_scale_jitter is not None:
            ls = ls + rng.uniform(-log_scale_jitter, log_scale_jitter, size=(3, n))
    if random_quats:
        q = rng.normal(size=(4, n))
        q /= np.linalg.norm(q, axis=0, keepdims=True)
    else:
        q = np.zeros((4, n))
        q[0] = 1.0
    if opacity_logit_range is not None:
        op = rng.uniform(opacity_logit_range[0], opacity_logit_range[1], size=n)
    else:
        op = np.full(n, float(opacity_logit))
    sh = np.zeros((n_sh_rows(sh_degree), n))
    if sh_std > 0:
        sh = rng.normal(0.0, sh_std, size=sh.shape)
    return {
        "means": means,
        "log_scales": ls.astype(np.float32),
        "quats": q.astype(np.float32),
        "opacity_logits": op.astype(np.float32),
        "sh": sh.astype(np.float32),
        "sh_degree": int(sh_degree),
    }


def subset(params, idx):
    """Gaussians idx of a parameter dict (a smaller scene of the same draw)."""
    out = {k: (v[..., idx].copy() if isinstance(v, np.ndarray) else v) for k, v in params.items()}
    return out
