"""One training step of the rasterizer, assembled from the oracle's stages.

forward(view):  project -> tile lists (keys, order, ranges) -> composite
loss:           (1 - lambda) L1 + lambda (1 - SSIM), averaged over the views
backward(view): compositing derivative -> chain rule to the parameters,
                summed over the views
step:           Adam on every parameter group

Sec. III of the paper initialises Gaussians from isosurface points and trains
them on orbit views with the 3D-GS pipeline; this module is that pipeline for
one GPU's worth of views.
"""
from __future__ import annotations

import numpy as np

from . import adam as _adam
from . import backward as _bwd
from . import binning as _bin
from . import blend as _blend
from . import loss as _loss
from . import project as _proj


def forward_view(params, cam, tile=16, bg=(0.0, 0.0, 0.0), tile_offset=0):
    W, H = int(cam["width"]), int(cam["height"])
    tx, ty = (W + tile - 1) // tile, (H + tile - 1) // tile
    pr = _proj.project(params, cam, tile)
    lists = _bin.tile_lists(pr, tx, ty, tile_offset)
    img, T, n, flags = _blend.render_view(pr, lists, bg)
    return dict(proj=pr, lists=lists, image=img, T=T, n=n, flags=flags, tiles=(tx, ty))


def backward_view(params, cam, fw, dimg, bg=(0.0, 0.0, 0.0)):
    acc = _blend.backward_view(fw["proj"], fw["lists"], np.asarray(dimg, np.float64), bg)
    return acc, _bwd.param_grads(fw["proj"], params, cam, acc)


def add_grads(a, b):
    if a is None:
        return {k: v.copy() for k, v in b.items()}
    return {k: a[k] + b[k] for k in a}


def train_step_grads(params, cams, targets, tile=16, bg=(0.0, 0.0, 0.0), lam=_loss.LAMBDA):
    """Loss and parameter gradients of one batch of views."""
    fws = [forward_view(params, c, tile, bg) for c in cams]
    L, dimgs = _loss.batch_loss([f["image"] for f in fws], targets, lam)
    total = None
    accs = []
    for c, f, d in zip(cams, fws, dimgs):
        acc, g = backward_view(params, c, f, d, bg)
        accs.append(acc)
        total = add_grads(total, g)
    return L, total, fws, dimgs, accs


def lr_table(sh_degree, lr=None):
    """Per-row learning rates of the sh array: DC rows, then the rest."""
    lr = dict(_adam.DEFAULT_LR if lr is None else lr)
    nrow = (sh_degree + 1) ** 2 * 3
    sh_lr = np.full(nrow, lr["sh_rest"])
    sh_lr[:3] = lr["sh_dc"]
    return lr, sh_lr


def adam_all(params, grads, m, v, t, lr=None):
    """Adam over every group; returns new (params, m, v) dicts in float64."""
    lr, sh_lr = lr_table(params["sh_degree"], lr)
    newp, newm, newv = {"sh_degree": params["sh_degree"]}, {}, {}
    for k in ("means", "log_scales", "quats", "opacity_logits"):
        newp[k], newm[k], newv[k] = _adam.adam_step(params[k], grads[k], m[k], v[k], lr[k], t)
    newp["sh"], newm["sh"], newv["sh"] = _adam.adam_step(
        params["sh"], grads["sh"], m["sh"], v["sh"], sh_lr[:, None], t)
    return newp, newm, newv
