"""Isosurface points and ray-cast views of a sampled volume (test infrastructure:
the plain float64 definitions the device extraction and ray-caster are checked
against).

Sec. III (Method Overview) extracts an isosurface from the scientific volume,
initialises Gaussians from its points and renders target views of the surface
on a structured orbit; Sec. V points to doing this in situ.  The paper uses
ParaView for both and states no algorithm; the readings here:

Volume: values v[k][j][i] at the vertices of a regular nx x ny x nz grid over
the box [lo, hi] (vertex (i, j, k) at lo + (i, j, k) * h, h = (hi - lo) / (n - 1)).

Extraction (the vertex rule of marching cubes): every grid edge whose end
values a = v0 - iso, b = v1 - iso have strictly opposite signs yields the point
p0 + t (p1 - p0), t = a / (a - b).  Canonical order: vertices in row-major
(k, j, i) order, and for each vertex its +x, +y, +z edges.  Subsampling keeps
the crossing on edge e = 3 * vertex + axis when the Philox4x32-10 uniform
(x0 >> 8) 2^-24 of counter (e low word, e high word, 3, 0) under the key
(seed low word, seed high word) is below keep_prob.

Ray-cast: the ray of pixel (x, y) leaves the camera centre -R^T t in the
direction R^T ((x + 0.5 - cx) / fx, (y + 0.5 - cy) / fy, 1), normalised.  It is
clipped to the box (slab method; t >= 0), sampled at t_k = t_near + k * step
(k = 0, 1, ...) with the trilinear interpolant of the volume; the first k with
f(t_{k-1}) < iso <= f(t_k), t_k <= t_far, brackets the hit, refined by ten
bisections (the lower end moves while f(mid) < iso); the hit is the bracket's
midpoint.  Shading: albedo(p) (0.2 + 0.8 |n . d|), n the normalised gradient of
the trilinear interpolant at the hit, albedo = (0.85, 0.45 + 0.25 z,
0.30 + 0.25 (x + 1)); misses are 0.
"""
from __future__ import annotations

import numpy as np

from .init import MASK, philox4x32_10, uniform24


def grid_axes(n, lo, hi):
    """Vertex coordinates per axis: lo + i h, h = (hi - lo)/(n - 1)."""
    out = []
    for a in range(3):
        h = (hi[a] - lo[a]) / (n[a] - 1)
        out.append(lo[a] + np.arange(n[a], dtype=np.float64) * h)
    return out


def crossings(vol, lo, hi, iso):
    """All crossing points (3, M) in canonical order, with their edge ids (M,)."""
    v = np.asarray(vol, np.float64) - float(iso)
    nz, ny, nx = v.shape
    ax = grid_axes((nx, ny, nz), lo, hi)
    h = [(hi[a] - lo[a]) / ((nx, ny, nz)[a] - 1) for a in range(3)]
    pts, ids = [], []
    K, J, I = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    vid = (K * ny + J) * nx + I
    for axis in range(3):
        sl0 = [slice(None)] * 3
        sl1 = [slice(None)] * 3
        dim = 2 - axis                       # array axis of x, y, z
        sl0[dim] = slice(0, v.shape[dim] - 1)
        sl1[dim] = slice(1, v.shape[dim])
        a, b = v[tuple(sl0)], v[tuple(sl1)]
        cross = ((a < 0) & (b > 0)) | ((a > 0) & (b < 0))
        k, j, i = np.nonzero(cross)
        t = a[k, j, i] / (a[k, j, i] - b[k, j, i])
        p = np.stack([ax[0][i], ax[1][j], ax[2][k]], 0)
        p[axis] = p[axis] + t * h[axis]
        pts.append(p)
        ids.append(vid[k, j, i].astype(np.int64) * 3 + axis)
    pts = np.concatenate(pts, 1)
    ids = np.concatenate(ids)
    order = np.argsort(ids, kind="stable")
    return pts[:, order], ids[order]


def keep_mask(edge_ids, keep_prob, seed):
    e = np.asarray(edge_ids, np.uint64)
    z = np.zeros(e.shape, np.uint64)
    d = philox4x32_10([e & np.uint64(MASK), e >> np.uint64(32), z + 3, z],
                      (seed & MASK, (seed >> 32) & MASK))
    return uniform24(d[0]) < np.float32(keep_prob)


def extract(vol, lo, hi, iso, keep_prob=1.0, seed=0):
    """Kept crossing points (3, N) in canonical order and the crossing count M."""
    p, ids = crossings(vol, lo, hi, iso)
    k = keep_mask(ids, keep_prob, seed)
    return p[:, k], p.shape[1]


# ---------------------------------------------------------------- ray-cast
def _trilinear(vol, lo, h, p):
    """Values (P,) and gradients (P, 3) of the trilinear interpolant at points p (P, 3)."""
    nz, ny, nx = vol.shape
    n = np.array([nx, ny, nz])
    u = (p - lo) / h
    i0 = np.clip(np.floor(u).astype(np.int64), 0, n - 2)
    f = u - i0
    ix, iy, iz = i0[:, 0], i0[:, 1], i0[:, 2]
    fx, fy, fz = f[:, 0], f[:, 1], f[:, 2]
    c = {}
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                c[dx, dy, dz] = vol[iz + dz, iy + dy, ix + dx].astype(np.float64)
    c00 = c[0, 0, 0] + fx * (c[1, 0, 0] - c[0, 0, 0])
    c10 = c[0, 1, 0] + fx * (c[1, 1, 0] - c[0, 1, 0])
    c01 = c[0, 0, 1] + fx * (c[1, 0, 1] - c[0, 0, 1])
    c11 = c[0, 1, 1] + fx * (c[1, 1, 1] - c[0, 1, 1])
    c0 = c00 + fy * (c10 - c00)
    c1 = c01 + fy * (c11 - c01)
    val = c0 + fz * (c1 - c0)
    # derivative of the interpolant with respect to x, y, z
    dx0 = (c[1, 0, 0] - c[0, 0, 0]) * (1 - fy) + (c[1, 1, 0] - c[0, 1, 0]) * fy
    dx1 = (c[1, 0, 1] - c[0, 0, 1]) * (1 - fy) + (c[1, 1, 1] - c[0, 1, 1]) * fy
    gx = (dx0 * (1 - fz) + dx1 * fz) / h[0]
    gy = ((c10 - c00) * (1 - fz) + (c11 - c01) * fz) / h[1]
    gz = (c1 - c0) / h[2]
    return val, np.stack([gx, gy, gz], 1)


def raycast(vol, lo, hi, iso, cam, step, bisections=10):
    """Planar float64 image (3, H, W) of the isosurface of `vol` seen by `cam`."""
    vol = np.asarray(vol, np.float32)
    nz, ny, nx = vol.shape
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    h = (hi - lo) / (np.array([nx, ny, nz]) - 1)
    R = np.asarray(cam["R"], np.float64).reshape(3, 3)
    t = np.asarray(cam["t"], np.float64)
    W, H = int(cam["width"]), int(cam["height"])
    # camera centre -R^T t and directions R^T dc, as explicit sums of products
    o = -np.array([R[0, a] * t[0] + R[1, a] * t[1] + R[2, a] * t[2] for a in range(3)])
    ys, xs = np.mgrid[0:H, 0:W]
    dc = [(xs.ravel() + 0.5 - float(cam["cx"])) / float(cam["fx"]),
          (ys.ravel() + 0.5 - float(cam["cy"])) / float(cam["fy"]), np.ones(W * H)]
    d = np.stack([dc[0] * R[0, a] + dc[1] * R[1, a] + dc[2] * R[2, a] for a in range(3)], 1)
    d /= np.sqrt(d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2])[:, None]
    img = np.zeros((W * H, 3))
    for pix in range(W * H):
        dd = d[pix]
        tn, tf = 0.0, np.inf
        hit_box = True
        for a in range(3):
            if dd[a] == 0.0:
                if o[a] < lo[a] or o[a] > hi[a]:
                    hit_box = False
                continue
            t0, t1 = (lo[a] - o[a]) / dd[a], (hi[a] - o[a]) / dd[a]
            tn, tf = max(tn, min(t0, t1)), min(tf, max(t0, t1))
        if not hit_box or not tf > tn:
            continue
        f_prev = _trilinear(vol, lo, h, (o + tn * dd)[None])[0][0] - iso
        k = 1
        hit = None
        while True:
            tk = tn + k * step
            if tk > tf:
                break
            f = _trilinear(vol, lo, h, (o + tk * dd)[None])[0][0] - iso
            if f_prev < 0 and f >= 0:
                hit = (tn + (k - 1) * step, tk)
                break
            f_prev = f
            k += 1
        if hit is None:
            continue
        a_, b_ = hit
        for _ in range(bisections):
            mid = 0.5 * (a_ + b_)
            if _trilinear(vol, lo, h, (o + mid * dd)[None])[0][0] - iso < 0:
                a_ = mid
            else:
                b_ = mid
        p = o + 0.5 * (a_ + b_) * dd
        _, g = _trilinear(vol, lo, h, p[None])
        g = g[0]
        gn = np.sqrt((g * g).sum())
        lam = abs((g / gn) @ dd) if gn > 0 else 0.0
        alb = np.array([0.85, 0.45 + 0.25 * p[2], 0.30 + 0.25 * (p[0] + 1.0)])
        img[pix] = alb * (0.2 + 0.8 * lam)
    return img.T.reshape(3, H, W)
