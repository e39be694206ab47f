"""Training loop of the 3D-GS model on orbit views, through the C ABI.

Sec. III (Method Overview) trains the Gaussians initialised from isosurface
points to match synthetic views on a structured orbit; the paper gives no
schedule.  One iteration here: a view from a seeded permutation of the
training views (reshuffled each epoch), forward, the L1 + SSIM image
gradient, backward, one Adam step over every Gaussian; adaptive density
control (statistics, densify, opacity reset) on a schedule.  Every step runs
in the library's kernels; this module only sequences the calls and owns the
device tensors (parameters, moments, statistics, images).

Schedule readings (3D-GS defaults, scaled for short runs by the caller):
statistics from ``densify_from`` (exclusive) to ``densify_until``; densify
every ``densify_interval`` iterations inside that window; opacity reset every
``opacity_reset_interval`` iterations; the screen-size prune (20 px) only
after the first opacity reset; scene extent = the orbit radius.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from . import core
from . import density as dens


@dataclass
class Schedule:
    densify_from: int = 500
    densify_until: int = 15000
    densify_interval: int = 100
    opacity_reset_interval: int = 3000
    screen_prune_px: float = 20.0
    extent: float = 2.5
    seed: int = 0
    density_opts: dict = field(default_factory=dict)


class Trainer:
    """Trains `params` against `targets` (device float32 [3][H][W], one per camera)."""

    def __init__(self, ctx, params, cams, targets, *, lr=None, lam=0.2, tile=16, lds_depth=256,
                 schedule=None, densify=True, seed=0):
        self.ctx = ctx
        self.params = params
        self.cams = list(cams)
        self.targets = [t.contiguous() for t in targets]
        self.lr = lr
        self.lam = lam
        self.tile, self.depth = tile, lds_depth
        self.sched = schedule if schedule is not None else Schedule()
        self.densify_on = densify
        self.m = params.zeros_like()
        self.v = params.zeros_like()
        self.grads = params.zeros_like()
        self.stats = dens.DensityStats.zeros(params.n, params.means.device)
        self.rng = np.random.default_rng(seed)
        self.order = []
        self.it = 0
        self.frame = core.Frame()
        dev = params.means.device
        self.images = {}
        self.dl = {}
        self.loss = torch.zeros(1, device=dev)
        self.history = []

    def _buf(self, d, cam):
        key = (cam.width, cam.height)
        if key not in d:
            d[key] = torch.empty((3, cam.height, cam.width), device=self.params.means.device)
        return d[key]

    def _next_view(self):
        if not self.order:
            self.order = list(self.rng.permutation(len(self.cams)))
        return int(self.order.pop(0))

    def step(self):
        """One iteration; returns (view index, loss tensor on the device)."""
        self.it += 1
        it, sc = self.it, self.sched
        k = self._next_view()
        cam, tgt = self.cams[k], self.targets[k]
        collect = self.densify_on and sc.densify_from < it <= sc.densify_until
        img = self._buf(self.images, cam)
        dl = self._buf(self.dl, cam)
        core.render_fwd(self.ctx, self.params, [cam], [img], tile=self.tile,
                        lds_depth=self.depth, flags=core.RADII if collect else 0,
                        frame=self.frame)
        core.loss_grad_into(self.ctx, [img], [tgt], [cam], self.loss, [dl], self.lam)
        core.render_bwd(self.ctx, self.frame, self.params, [dl], self.grads, keep_screen=collect)
        if collect:
            dens.accumulate(self.ctx, self.frame, self.stats, scale=1.0)
        core.adam_step(self.ctx, self.params, self.grads, self.m, self.v, it, lr=self.lr)
        info = None
        if collect and it % sc.densify_interval == 0:
            info = self.densify(max_screen=sc.screen_prune_px
                                if it > sc.opacity_reset_interval else 0.0)
        if self.densify_on and it <= sc.densify_until and it % sc.opacity_reset_interval == 0:
            dens.opacity_reset(self.ctx, self.params, self.m, self.v, 0.01)
        return k, info

    def densify(self, max_screen=0.0):
        sc = self.sched
        p, m, v, info = dens.densify(self.ctx, self.params, self.m, self.v, self.stats,
                                     sc.extent, seed=sc.seed * 1000003 + self.it,
                                     max_screen=max_screen, **sc.density_opts)
        self.params, self.m, self.v = p, m, v
        self.grads = p.zeros_like()
        self.stats = dens.DensityStats.zeros(p.n, p.means.device)
        # the frame's buffers were sized for the old count; the next forward resizes them
        return info

    def run(self, iters, log_every=10, eval_fn=None, eval_every=None):
        """Runs `iters` iterations; records (iteration, loss, n) every log_every and
        eval_fn(self) every eval_every iterations."""
        for _ in range(iters):
            _, info = self.step()
            rec = None
            if self.it % log_every == 0 or info is not None:
                rec = {"it": self.it, "loss": float(self.loss.item()), "n": self.params.n}
                if info is not None:
                    rec["densify"] = info
            if eval_fn is not None and eval_every and self.it % eval_every == 0:
                rec = rec or {"it": self.it, "loss": float(self.loss.item()),
                              "n": self.params.n}
                rec["eval"] = eval_fn(self)
            if rec is not None:
                self.history.append(rec)
        return self.history

    def evaluate(self, cams, refs):
        """Mean and per-view (mse, psnr, l1, ssim) of renders of `cams` against `refs`."""
        rows = []
        for cam, ref in zip(cams, refs):
            img = self._buf(self.images, cam)
            core.render_fwd(self.ctx, self.params, [cam], [img], tile=self.tile,
                            lds_depth=self.depth, frame=self.frame)
            rows.append(core.image_metrics(self.ctx, [img], [ref], [cam])[0])
        m = torch.stack(rows).cpu().numpy().astype(np.float64)
        return {"mse": float(m[:, 0].mean()), "psnr": float(m[:, 1].mean()),
                "l1": float(m[:, 2].mean()), "ssim": float(m[:, 3].mean()),
                "per_view": m.tolist()}

    def close(self):
        self.frame.release()
