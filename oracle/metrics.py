"""Image-quality metrics of a rendered view against its reference (test
infrastructure: the plain float64 definitions the device metrics are checked
against).  The paper reports PSNR, SSIM and LPIPS of its trained models
(Sec. IV, Tables II and III); LPIPS needs trained network weights and is not
computed.  Values are in [0, 1] (peak 1).

mse  = mean over pixels and channels of (x - y)^2
psnr = 10 log10(1 / mse)        (+inf when mse is 0)
l1   = mean |x - y|
ssim = mean SSIM with the training loss's window and constants
"""
from __future__ import annotations

import numpy as np

from . import loss as _loss


def mse(x, y):
    d = np.asarray(x, np.float64) - np.asarray(y, np.float64)
    return float(np.mean(d * d))


def psnr(x, y):
    e = mse(x, y)
    return float("inf") if e == 0 else float(-10.0 * np.log10(e))


def l1(x, y):
    return float(np.mean(np.abs(np.asarray(x, np.float64) - np.asarray(y, np.float64))))


def metrics(x, y):
    """(mse, psnr, l1, ssim) of one view."""
    return mse(x, y), psnr(x, y), l1(x, y), float(_loss.ssim(x, y))
