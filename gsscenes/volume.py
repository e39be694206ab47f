"""Sampled volumes of the seeded fields: the stand-in for a simulation's scalar
output already resident on the device (the in-situ setting).  Values at the
vertices of a cubic G^3 grid over [-1, 1]^3, computed slab by slab from the
field's separable form and copied to the device slab by slab."""
from __future__ import annotations

import numpy as np


def sample_volume(field, G, device=None, progress=None):
    """float32 (G, G, G) array indexed [z][y][x] (a torch tensor on `device` if given)."""
    xs = np.linspace(-1.0, 1.0, G)
    if device is None:
        return np.stack([field.slab(xs, z).astype(np.float32) for z in xs], 0)
    import torch
    out = torch.empty((G, G, G), dtype=torch.float32, device=device)
    for k, z in enumerate(xs):
        if progress is not None and k % 256 == 0:
            progress(f"volume: slab {k} of {G}")
        out[k].copy_(torch.from_numpy(field.slab(xs, z).astype(np.float32)))
    return out


def sample_points_grid(field, nx, ny, nz, lo=(-1.0, -1.0, -1.0), hi=(1.0, 1.0, 1.0)):
    """float32 (nz, ny, nx) values of the field at the vertices of a box grid
    (vertex (i, j, k) at lo + (i, j, k) h, h = (hi - lo) / (n - 1)); point by point,
    for small grids."""
    ax = [lo[a] + np.arange(n) * ((hi[a] - lo[a]) / (n - 1)) for a, n in enumerate((nx, ny, nz))]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    p = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    return field.eval(p).reshape(nz, ny, nx).astype(np.float32)
