"""Training loss (1 - lambda) L1 + lambda (1 - SSIM) and its image gradient.

The paper trains the cited 3D-GS model and reports PSNR/SSIM/LPIPS (Sec. IV,
Tables II-III) but states no loss.  Reading used: the 3D-GS photometric loss
with lambda = 0.2; SSIM with an 11 x 11 Gaussian window (sigma 1.5, weights
summing to one), C1 = 0.01^2, C2 = 0.03^2, zero padding and same-size output,
averaged over pixels and channels; a batch of views averages the per-view
losses.  The L1 subgradient at zero is zero.

Local statistics: mu = w * x, E[x^2] = w * x^2, E[xy] = w * (x y) with *
the zero-padded correlation.  SSIM = (2 mu_x mu_y + C1)(2 s_xy + C2) /
((mu_x^2 + mu_y^2 + C1)(s_xx + s_yy + C2)), s_xx = E[x^2] - mu_x^2,
s_xy = E[xy] - mu_x mu_y.  Its gradient with respect to x is
w * g1 + 2 x (w * g2) + y (w * g3) with g1 = dS/dmu_x, g2 = dS/dE[x^2],
g3 = dS/dE[xy] (the window is symmetric, so correlation is self-adjoint).
"""
from __future__ import annotations

import numpy as np

C1 = 0.01 ** 2
C2 = 0.03 ** 2
WIN = 11
SIGMA = 1.5
LAMBDA = 0.2


def window1d():
    r = np.arange(WIN) - WIN // 2
    g = np.exp(-(r * r) / (2 * SIGMA * SIGMA))
    return g / g.sum()


def filt(img):
    """Zero-padded 'same' correlation of (..., H, W) with the 2-D window."""
    g = window1d()
    h = WIN // 2
    H, W = img.shape[-2:]
    pad = np.zeros(img.shape[:-2] + (H + 2 * h, W + 2 * h))
    pad[..., h:h + H, h:h + W] = img
    out = np.zeros_like(img, dtype=np.float64)
    for i in range(WIN):
        for j in range(WIN):
            out += g[i] * g[j] * pad[..., i:i + H, j:j + W]
    return out


def ssim_terms(x, y):
    mx, my = filt(x), filt(y)
    exx, eyy, exy = filt(x * x), filt(y * y), filt(x * y)
    sxx, syy, sxy = exx - mx * mx, eyy - my * my, exy - mx * my
    A1, A2 = 2 * mx * my + C1, 2 * sxy + C2
    B1, B2 = mx * mx + my * my + C1, sxx + syy + C2
    S = A1 * A2 / (B1 * B2)
    return S, (mx, my, A1, A2, B1, B2)


def ssim(x, y):
    return ssim_terms(np.asarray(x, np.float64), np.asarray(y, np.float64))[0].mean()


def ssim_grad(x, y):
    """d mean(SSIM) / d x."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    S, (mx, my, A1, A2, B1, B2) = ssim_terms(x, y)
    g1 = S * (2 * my / A1 - 2 * my / A2 - 2 * mx / B1 + 2 * mx / B2)
    g2 = S * (-1.0 / B2)
    g3 = S * (2.0 / A2)
    return (filt(g1) + 2 * x * filt(g2) + y * filt(g3)) / x.size


def view_loss(x, y, lam=LAMBDA):
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    return (1 - lam) * np.abs(x - y).mean() + lam * (1.0 - ssim(x, y))


def view_loss_grad(x, y, lam=LAMBDA):
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    return (1 - lam) * np.sign(x - y) / x.size - lam * ssim_grad(x, y)


def batch_loss(xs, ys, lam=LAMBDA):
    """Mean over views of the per-view loss, and the per-view image gradients."""
    n = len(xs)
    L = sum(view_loss(x, y, lam) for x, y in zip(xs, ys)) / n
    grads = [view_loss_grad(x, y, lam) / n for x, y in zip(xs, ys)]
    return L, grads
