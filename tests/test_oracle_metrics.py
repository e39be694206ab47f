"""Pins of the oracle's image metrics (CPU): closed forms of MSE / PSNR / L1
for constant offsets, brute-force sums on a small random pair, identity
images, and SSIM of constant images against its closed form."""
import math

import numpy as np

from oracle import loss as oloss
from oracle import metrics as M


def test_constant_offset_closed_forms():
    x = np.full((3, 20, 30), 0.25)
    for c in (0.5, 0.1, 1e-3):
        y = x + c
        assert abs(M.mse(x, y) - c * c) < 1e-15
        assert abs(M.psnr(x, y) - (-20.0 * math.log10(c))) < 1e-9
        assert abs(M.l1(x, y) - c) < 1e-15


def test_brute_force_sums():
    rng = np.random.default_rng(0)
    x, y = rng.random((3, 7, 5)), rng.random((3, 7, 5))
    s2 = s1 = 0.0
    for c in range(3):
        for i in range(7):
            for j in range(5):
                d = x[c, i, j] - y[c, i, j]
                s2 += d * d
                s1 += abs(d)
    assert abs(M.mse(x, y) - s2 / 105) < 1e-15
    assert abs(M.l1(x, y) - s1 / 105) < 1e-15
    assert abs(M.psnr(x, y) - 10 * math.log10(105 / s2)) < 1e-9


def test_identity_and_ssim_constants():
    rng = np.random.default_rng(1)
    x = rng.random((3, 16, 16))
    e, p, a, s = M.metrics(x, x)
    assert e == 0 and p == float("inf") and a == 0 and abs(s - 1) < 1e-12
    # SSIM of constant images a, b: (2ab + C1)/(a^2 + b^2 + C1) at pixels at least 5 from
    # the border (zero padding changes the window sums there); the metric is the map's mean
    a0, b0 = 0.3, 0.7
    xa, yb = np.full((3, 40, 40), a0), np.full((3, 40, 40), b0)
    S, _ = oloss.ssim_terms(xa, yb)
    want = (2 * a0 * b0 + 0.01 ** 2) / (a0 * a0 + b0 * b0 + 0.01 ** 2)
    assert np.abs(S[:, 5:35, 5:35] - want).max() < 1e-12
    assert abs(M.metrics(xa, yb)[3] - S.mean()) < 1e-15
