"""Sampled volumes of the seeded fields: the stand-in for a simulation's scalar
output already resident on the device (the in-situ setting).  Values at the
vertices of a cubic G^3 grid over [-1, 1]^3, computed slab by slab from the
field's separable form and copied to the device slab by slab."""
from __future__ import annotations

import numpy as np


def sample_volume(field, G, device=None, progress=None):
    """float32 (G, G, G) array indexed [z][y][x] (a torch tensor on `device` if given;
    its slabs are then evaluated on the device in float64, the same separable sums)."""
    xs = np.linspace(-1.0, 1.0, G)
    if device is None:
        return np.stack([field.slab(xs, z).astype(np.float32) for z in xs], 0)
    import torch
    out = torch.empty((G, G, G), dtype=torch.float32, device=device)
    slab = _TorchSlab(field, xs, device)
    for k, z in enumerate(xs):
        if progress is not None and k % 512 == 0:
            progress(f"volume: slab {k} of {G}")
        out[k].copy_(slab(float(z)))
    return out


class _TorchSlab:
    """The fields' slab(xs, z) on a torch device (float64): blobs as a product of
    per-axis factors, spectral noise as a complex product, the mixing layer's
    interface height evaluated once per grid."""

    def __init__(self, field, xs, device):
        import torch
        from .fields import BlobField, MixingLayer
        self.t = torch
        self.f = field
        self.dev = device
        self.xs = torch.tensor(xs, dtype=torch.float64, device=device)
        self.kind = "blob" if isinstance(field, BlobField) else (
            "mix" if isinstance(field, MixingLayer) else None)
        if self.kind is None:
            raise TypeError(f"no device slab for {type(field).__name__}")
        if self.kind == "blob":
            c = torch.tensor(field.c, dtype=torch.float64, device=device)
            iw = 1.0 / (2 * torch.tensor(field.w, dtype=torch.float64, device=device) ** 2)
            self.gx = torch.exp(-((self.xs[None, :] - c[:, 0:1]) ** 2) * iw[:, None])
            self.gy = torch.exp(-((self.xs[None, :] - c[:, 1:2]) ** 2) * iw[:, None])
            self.cz, self.iw = c[:, 2], iw
            self.noise = self._noise(field.noise) if field.noise is not None else None
        else:
            k = torch.tensor(field.k, dtype=torch.float64, device=device)
            phi = torch.tensor(field.phi, dtype=torch.float64, device=device)
            a = torch.tensor(field.a, dtype=torch.float64, device=device)
            G = self.xs.shape[0]
            eta = torch.zeros((G, G), dtype=torch.float64, device=device)
            X, Y = self.xs[None, :], self.xs[:, None]
            for m in range(k.shape[0]):
                eta += a[m] * torch.sin(X * k[m, 0] + Y * k[m, 1] + phi[m])
            self.eta = eta
            self.noise = self._noise(field.noise)

    def _noise(self, nz):
        t = self.t
        k = t.tensor(nz.k, dtype=t.float64, device=self.dev)
        return dict(ex=t.exp(1j * t.outer(k[:, 0], self.xs)), ey=t.exp(1j * t.outer(k[:, 1], self.xs)),
                    kz=k[:, 2], a=t.tensor(nz.a, dtype=t.float64, device=self.dev),
                    phi=t.tensor(nz.phi, dtype=t.float64, device=self.dev))

    def _noise_slab(self, z):
        n = self.noise
        ez = n["a"] * self.t.exp(1j * (n["kz"] * z + n["phi"]))
        return ((n["ey"] * ez[:, None]).T @ n["ex"]).real

    def __call__(self, z):
        t = self.t
        if self.kind == "blob":
            gz = t.exp(-((z - self.cz) ** 2) * self.iw)
            out = (self.gy * gz[:, None]).T @ self.gx
            if self.noise is not None:
                out = out + self._noise_slab(z)
        else:
            out = 0.5 + 0.5 * t.tanh((z + self.eta + self._noise_slab(z)) / self.f.delta)
        return out.to(t.float32)


def sample_points_grid(field, nx, ny, nz, lo=(-1.0, -1.0, -1.0), hi=(1.0, 1.0, 1.0)):
    """float32 (nz, ny, nx) values of the field at the vertices of a box grid
    (vertex (i, j, k) at lo + (i, j, k) h, h = (hi - lo) / (n - 1)); point by point,
    for small grids."""
    ax = [lo[a] + np.arange(n) * ((hi[a] - lo[a]) / (n - 1)) for a, n in enumerate((nx, ny, nz))]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    p = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    return field.eval(p).reshape(nz, ny, nx).astype(np.float32)
