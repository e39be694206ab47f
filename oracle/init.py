"""Gaussians initialised from isosurface points (Sec. III: the extracted point
cloud initialises the Gaussian primitives instead of image-based
reconstruction).

Reading used for the free choices: means are the points; log-scales constant
(plus uniform jitter) or uniform in a range, per axis; quaternions identity or
uniformly random (normalised 4-D normal); constant opacity logit; SH
coefficients N(0, sigma).  Random numbers come from Philox4x32-10 (Salmon,
Moraes, Dror, Shaw: "Parallel random numbers: as easy as 1, 2, 3", SC 2011):
key = (seed low word, seed high word), counter = (Gaussian index, stream,
block, 0); stream 0 gives three uniforms (log-scales), stream 1 four normals
(quaternion), stream 2 block b the SH normals 4b..4b+3.  Uniform:
(x >> 8) 2^-24.  Normals by Box-Muller on a pair (a, b):
r = sqrt(-2 ln(((a >> 8) + 0.5) 2^-24)), theta = 2 pi (b >> 8) 2^-24,
giving (r cos theta, r sin theta).
"""
from __future__ import annotations

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds; ctr (4, n) and key (2,) or (2, n) of uint32."""
    c = [np.asarray(x, np.uint64) & MASK for x in ctr]
    k0 = np.asarray(key[0], np.uint64) & MASK
    k1 = np.asarray(key[1], np.uint64) & MASK
    for r in range(10):
        if r > 0:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = np.uint64(M0) * c[0]
        p1 = np.uint64(M1) * c[2]
        c = [((p1 >> np.uint64(32)) ^ c[1] ^ k0) & MASK, p1 & MASK,
             ((p0 >> np.uint64(32)) ^ c[3] ^ k1) & MASK, p0 & MASK]
    return [x.astype(np.uint32) for x in c]


def uniform24(x):
    return (np.asarray(x, np.uint32) >> 8).astype(np.float64) * 2.0 ** -24


def box_muller(a, b):
    ua = ((np.asarray(a, np.uint32) >> 8).astype(np.float64) + 0.5) * 2.0 ** -24
    r = np.sqrt(-2.0 * np.log(ua))
    th = 2.0 * np.pi * uniform24(b)
    return r * np.cos(th), r * np.sin(th)


def init_from_points(xyz, sh_degree, *, log_scale=0.0, log_scale_jitter=0.0,
                     log_scale_range=None, random_quats=False, opacity_logit=0.1, sh_std=0.0,
                     seed=0):
    xyz = np.asarray(xyz, np.float64)
    n = xyz.shape[1]
    idx = np.arange(n, dtype=np.uint64)
    zero = np.zeros(n, np.uint64)
    key = (seed & MASK, (seed >> 32) & MASK)
    u = philox4x32_10([idx, zero, zero, zero], key)
    U = np.stack([uniform24(u[k]) for k in range(3)], 0)
    if log_scale_range is not None and log_scale_range[0] < log_scale_range[1]:
        lo, hi = log_scale_range
        ls = lo + (hi - lo) * U
    else:
        ls = log_scale + log_scale_jitter * (2.0 * U - 1.0)
    if random_quats:
        d = philox4x32_10([idx, zero + 1, zero, zero], key)
        q0, q1 = box_muller(d[0], d[1])
        q2, q3 = box_muller(d[2], d[3])
        q = np.stack([q0, q1, q2, q3], 0)
        q /= np.sqrt((q * q).sum(0))
    else:
        q = np.zeros((4, n))
        q[0] = 1.0
    rows = (sh_degree + 1) ** 2 * 3
    sh = np.zeros((rows, n))
    if sh_std > 0:
        for b in range((rows + 3) // 4):
            d = philox4x32_10([idx, zero + 2, zero + b, zero], key)
            z = list(box_muller(d[0], d[1])) + list(box_muller(d[2], d[3]))
            for k in range(4):
                if 4 * b + k < rows:
                    sh[4 * b + k] = sh_std * z[k]
    return {"means": xyz.copy(), "log_scales": ls, "quats": q,
            "opacity_logits": np.full(n, float(opacity_logit)), "sh": sh,
            "sh_degree": sh_degree}
