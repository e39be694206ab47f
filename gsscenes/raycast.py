"""Ray-cast images of a field's isosurface: the training targets.

Rays follow the pinhole camera of the render (x right, y down, z forward,
pixel centres at (x + 0.5, y + 0.5)), march from the entry into [-1, 1]^3 with
a fixed step, refine the first crossing by bisection and shade the hit with a
headlight Lambertian term over a position-dependent albedo.  Misses are black.
Images are planar float32 [3][H][W].
"""
from __future__ import annotations

import numpy as np


def _albedo(p):
    return np.stack([0.85 + 0.0 * p[:, 0],
                     0.45 + 0.25 * p[:, 2],
                     0.30 + 0.25 * (p[:, 0] + 1.0)], 1)


def raycast(field, R, t, fx, fy, cx, cy, W, H, *, step, iso=0.5, chunk=1 << 16):
    R = np.asarray(R, np.float64).reshape(3, 3)
    t = np.asarray(t, np.float64)
    origin = -R.T @ t
    ys, xs = np.mgrid[0:H, 0:W]
    dc = np.stack([(xs.ravel() + 0.5 - cx) / fx, (ys.ravel() + 0.5 - cy) / fy,
                   np.ones(W * H)], 1)
    d = dc @ R                                   # rows: R^T dc
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    img = np.zeros((W * H, 3))
    for s0 in range(0, W * H, chunk):
        dd = d[s0:s0 + chunk]
        with np.errstate(divide="ignore", invalid="ignore"):
            inv = 1.0 / dd
            t0 = (-1.0 - origin) * inv
            t1 = (1.0 - origin) * inv
        tn = np.nanmax(np.minimum(t0, t1), 1)
        tf = np.nanmin(np.maximum(t0, t1), 1)
        tn = np.maximum(tn, 0.0)
        live = tf > tn
        idx = np.nonzero(live)[0]
        if idx.size == 0:
            continue
        tc = tn[idx].copy()
        tend = tf[idx]
        f_prev = field.eval(origin + tc[:, None] * dd[idx]) - iso
        hit_t = np.full(idx.size, np.nan)
        lo = np.zeros(idx.size)
        active = np.ones(idx.size, bool)
        while active.any():
            a = np.nonzero(active)[0]
            tn_a = tc[a] + step
            f = field.eval(origin + tn_a[:, None] * dd[idx[a]]) - iso
            crossed = (f_prev[a] < 0) & (f >= 0)
            out = tn_a > tend[a]
            hc = a[crossed & ~out]
            hit_t[hc] = tn_a[crossed & ~out]
            lo[hc] = tc[hc]
            tc[a] = tn_a
            f_prev[a] = f
            active[a[crossed | out]] = False
        h = np.nonzero(~np.isnan(hit_t))[0]
        a_, b_ = lo[h], hit_t[h]
        ray = dd[idx[h]]
        for _ in range(10):
            mid = 0.5 * (a_ + b_)
            fm = field.eval(origin + mid[:, None] * ray) - iso
            below = fm < 0
            a_ = np.where(below, mid, a_)
            b_ = np.where(below, b_, mid)
        p = origin + (0.5 * (a_ + b_))[:, None] * ray
        n = -field.grad(p)
        n /= np.maximum(np.linalg.norm(n, axis=1, keepdims=True), 1e-30)
        lam = np.abs((n * -ray).sum(1))
        img[s0 + idx[h]] = _albedo(p) * (0.2 + 0.8 * lam)[:, None]
    return np.ascontiguousarray(img.T.reshape(3, H, W).astype(np.float32))
