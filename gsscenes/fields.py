"""Seeded analytic scalar fields on [-1, 1]^3 whose 0.5 level set stands in for
the scientific volumes (Kingsnake, Miranda) that are not available.

Every field is a sum of terms that factor over x, y and z, so a whole z-slab of
the sampling grid is one small matrix product (``slab``) and the full grid is
never materialised.  Fields also evaluate at arbitrary points with an analytic
gradient (used for tangential jitter and for the target ray-caster).

Three families, matching the synthetic workloads:

* ``BlobField``: sum of isotropic Gaussian blobs (tiny, 1M and 4M scenes);
* ``SpectralNoise``: random-phase Fourier modes with power-law amplitudes
  (spectral-synthesis fBm, Voss/Saupe), added to blobs as surface perturbation;
* ``MixingLayer``: a tanh interface displaced by sinusoidal modes, a stand-in
  for a turbulent mixing layer (18M scene).
"""
from __future__ import annotations

import numpy as np


class BlobField:
    """f(x) = sum_b exp(-|x - c_b|^2 / (2 w_b^2)) (+ optional noise term)."""

    def __init__(self, centers, widths, noise=None):
        self.c = np.asarray(centers, np.float64)      # (B, 3)
        self.w = np.asarray(widths, np.float64)       # (B,)
        self.noise = noise

    # -- point evaluation -------------------------------------------------
    def eval(self, p):
        p = np.asarray(p, np.float64)
        out = np.zeros(p.shape[0])
        for c, w in zip(self.c, self.w):
            d = p - c
            out += np.exp(-(d * d).sum(1) / (2 * w * w))
        if self.noise is not None:
            out += self.noise.eval(p)
        return out

    def grad(self, p):
        p = np.asarray(p, np.float64)
        g = np.zeros_like(p)
        for c, w in zip(self.c, self.w):
            d = p - c
            e = np.exp(-(d * d).sum(1) / (2 * w * w))
            g -= (e / (w * w))[:, None] * d
        if self.noise is not None:
            g += self.noise.grad(p)
        return g

    # -- separable grid evaluation -----------------------------------------
    def slab(self, xs, z):
        """Values on the (y, x) grid xs × xs at height z, shape (G, G)."""
        iw = 1.0 / (2 * self.w * self.w)
        gx = np.exp(-((xs[None, :] - self.c[:, 0:1]) ** 2) * iw[:, None])  # (B, G)
        gy = np.exp(-((xs[None, :] - self.c[:, 1:2]) ** 2) * iw[:, None])
        gz = np.exp(-((z - self.c[:, 2]) ** 2) * iw)                         # (B,)
        out = (gy * gz[:, None]).T @ gx                                      # (G_y, G_x)
        if self.noise is not None:
            out += self.noise.slab(xs, z)
        return out


class SpectralNoise:
    """n(x) = amp * sum_m a_m cos(k_m . x + phi_m), a_m ∝ |k_m|^-beta, sum a_m^2 = 1.

    Wave vectors have log-uniform magnitudes in [kmin, kmax] and uniform
    directions; this is spectral-synthesis fractional Brownian noise.
    """

    def __init__(self, rng, n_modes, kmin, kmax, beta, amp):
        mag = np.exp(rng.uniform(np.log(kmin), np.log(kmax), n_modes))
        d = rng.normal(size=(n_modes, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        self.k = d * mag[:, None]
        self.phi = rng.uniform(0, 2 * np.pi, n_modes)
        a = mag ** (-beta)
        self.a = amp * a / np.sqrt((a * a).sum())

    def eval(self, p):
        return (self.a[None, :] * np.cos(p @ self.k.T + self.phi[None, :])).sum(1)

    def grad(self, p):
        s = -self.a[None, :] * np.sin(p @ self.k.T + self.phi[None, :])     # (P, M)
        return s @ self.k

    def slab(self, xs, z):
        ex = np.exp(1j * np.outer(self.k[:, 0], xs))                          # (M, G)
        ey = np.exp(1j * np.outer(self.k[:, 1], xs))
        ez = self.a * np.exp(1j * (self.k[:, 2] * z + self.phi))              # (M,)
        return ((ey * ez[:, None]).T @ ex).real


class MixingLayer:
    """f(x) = 1/2 + 1/2 tanh((z + eta(x, y)) / delta), eta a sum of 2-D modes plus noise."""

    def __init__(self, rng, n_modes, delta, noise_amp, h):
        mag = np.exp(rng.uniform(np.log(2 * np.pi), np.log(64 * np.pi), n_modes))
        ang = rng.uniform(0, 2 * np.pi, n_modes)
        self.k = np.stack([mag * np.cos(ang), mag * np.sin(ang)], 1)         # (M, 2)
        self.phi = rng.uniform(0, 2 * np.pi, n_modes)
        a = mag ** (-5.0 / 3.0)
        self.a = 0.15 * a / a.sum()
        self.delta = delta
        self.noise = SpectralNoise(rng, 32, 64 * np.pi, 256 * np.pi, 1.0, noise_amp)

    def _eta(self, x, y):
        ph = np.multiply.outer(x, self.k[:, 0]) + np.multiply.outer(y, self.k[:, 1]) + self.phi
        return (self.a * np.sin(ph)).sum(-1)

    def eval(self, p):
        z = p[:, 2] + self._eta(p[:, 0], p[:, 1]) + self.noise.eval(p)
        return 0.5 + 0.5 * np.tanh(z / self.delta)

    def grad(self, p):
        ph = np.multiply.outer(p[:, 0], self.k[:, 0]) + np.multiply.outer(p[:, 1], self.k[:, 1]) + self.phi
        c = self.a * np.cos(ph)
        dz = np.stack([c @ self.k[:, 0], c @ self.k[:, 1], np.ones(p.shape[0])], 1) + self.noise.grad(p)
        z = p[:, 2] + self._eta(p[:, 0], p[:, 1]) + self.noise.eval(p)
        s = 0.5 / self.delta / np.cosh(z / self.delta) ** 2
        return dz * s[:, None]

    def z_support(self):
        """Heights outside which f - 1/2 has one sign on every (x, y): |eta + noise| <= bound."""
        b = float(np.abs(self.a).sum() + np.abs(self.noise.a).sum())
        return -b, b

    def slab(self, xs, z):
        # eta does not depend on z: evaluate it once per grid
        key = (xs.shape[0], float(xs[0]), float(xs[-1]))
        if getattr(self, "_eta_key", None) != key:
            X, Y = np.meshgrid(xs, xs)
            self._eta_grid = self._eta(X, Y)
            self._eta_key = key
        return 0.5 + 0.5 * np.tanh((z + self._eta_grid + self.noise.slab(xs, z)) / self.delta)


def blob_field(rng, n_blobs, center_half, w_lo, w_hi, noise=None):
    c = rng.uniform(-center_half, center_half, size=(n_blobs, 3))
    w = rng.uniform(w_lo, w_hi, size=n_blobs)
    return BlobField(c, w, noise)
