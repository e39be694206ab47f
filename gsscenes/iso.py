"""Isosurface point sampler: edge crossings of the level set on a G^3 vertex grid.

The grid spans [-1, 1]^3 with spacing h = 2/(G-1).  Every grid edge whose end
values straddle the isovalue yields one point, placed by linear interpolation
(the vertex rule of marching cubes).  Slabs are generated one z-plane at a time
so only two planes are ever resident.  A seeded subset of N points is returned;
when fewer than N crossings exist, seeded copies of crossings are displaced
tangentially (perpendicular to the field gradient) by 0.25 h.
"""
from __future__ import annotations

import numpy as np


def edge_crossings(field, G, iso=0.5, max_points=None, rng=None, progress=None):
    xs = np.linspace(-1.0, 1.0, G)
    h = xs[1] - xs[0]
    pts = []
    prev = None
    k0, k1 = 0, G - 1
    if hasattr(field, "z_support"):
        # planes beyond the support have one sign everywhere and no crossings, nor
        # do the z-edges between two of them; keep one such plane on each side
        lo, hi = field.z_support()
        inside = np.nonzero((xs >= lo) & (xs <= hi))[0]
        if inside.size:
            k0, k1 = max(0, int(inside[0]) - 1), min(G - 1, int(inside[-1]) + 1)
    for k in range(k0, k1 + 1):
        if progress is not None and (k - k0) % 128 == 0:
            progress(f"isosurface: plane {k - k0} of {k1 - k0 + 1}")
        cur = field.slab(xs, xs[k]) - iso                 # (y, x)
        # x-edges inside the plane
        s = cur[:, :-1] * cur[:, 1:] < 0
        j, i = np.nonzero(s)
        t = cur[j, i] / (cur[j, i] - cur[j, i + 1])
        pts.append(np.stack([xs[i] + t * h, xs[j], np.full(i.shape, xs[k])], 1))
        # y-edges inside the plane
        s = cur[:-1, :] * cur[1:, :] < 0
        j, i = np.nonzero(s)
        t = cur[j, i] / (cur[j, i] - cur[j + 1, i])
        pts.append(np.stack([xs[i], xs[j] + t * h, np.full(i.shape, xs[k])], 1))
        # z-edges between the previous plane and this one
        if prev is not None:
            s = prev * cur < 0
            j, i = np.nonzero(s)
            t = prev[j, i] / (prev[j, i] - cur[j, i])
            pts.append(np.stack([xs[i], xs[j], xs[k - 1] + t * h], 1))
        prev = cur
    return np.concatenate(pts, 0), h


def sample_points(field, G, n, rng, iso=0.5, progress=None):
    """n seeded points on the iso level set (float64, shape (n, 3)), and h."""
    cand, h = edge_crossings(field, G, iso, progress=progress)
    m = cand.shape[0]
    if m == 0:
        raise ValueError("field has no crossings of the isovalue on this grid")
    if m >= n:
        idx = rng.choice(m, size=n, replace=False)
        return cand[np.sort(idx)], h
    extra = cand[rng.integers(0, m, size=n - m)]
    nrm = field.grad(extra)
    nrm /= np.maximum(np.linalg.norm(nrm, axis=1, keepdims=True), 1e-30)
    r = rng.normal(size=extra.shape)
    r -= (r * nrm).sum(1, keepdims=True) * nrm
    r /= np.maximum(np.linalg.norm(r, axis=1, keepdims=True), 1e-30)
    return np.concatenate([cand, extra + 0.25 * h * r], 0), h
