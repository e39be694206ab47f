"""Batched multi-view training step: autotuned render options and a hipGraph.

``autotune`` asks the library to time the tile / LDS-depth / persistent
choices for a scene and view set, and caches the winner in a JSON file keyed
by the Gaussian count, SH degree and view sizes.  ``StepGraph`` captures one
whole step (forward, loss gradient, backward, Adam) for a fixed set of views
and replays it; the library handles record-capacity overflow by growing and
recapturing.
"""
from __future__ import annotations

import ctypes as C
import json
import os

import torch

from . import _lib as L
from .core import DEFAULT_LR, Params, _cam_array, _stream

CACHE = os.environ.get("ISOGS_TUNE_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "isogs_autotune.json"))


def _key(params, cams):
    sizes = ",".join(f"{c.width}x{c.height}" for c in cams)
    return f"n={params.n};deg={params.sh_degree};views={sizes}"


def autotune(ctx, params, cams, reps=2, cache=CACHE, use_cache=True, stream=None):
    """Best render options {tile, lds_depth, flags} and the timing table."""
    key = _key(params, cams)
    if use_cache and cache and os.path.exists(cache):
        try:
            with open(cache) as fh:
                hit = json.load(fh).get(key)
            if hit:
                return hit["best"], hit["table"]
        except (OSError, ValueError):
            pass
    best = L.GsRenderOpts()
    table = (L.GsTuneEntry * 32)()
    n = C.c_int32()
    L.check(L.lib().gs_autotune(ctx.handle, params.abi(), _cam_array(cams), len(cams), reps,
                                C.byref(best), table, 32, C.byref(n), _stream(stream)))
    out = {"tile": best.tile, "lds_depth": best.lds_depth, "flags": best.flags}
    rows = [{"tile": table[i].tile, "lds_depth": table[i].lds_depth, "flags": table[i].flags,
             "ms": round(table[i].ms, 4)} for i in range(n.value)]
    if cache:
        try:
            os.makedirs(os.path.dirname(cache), exist_ok=True)
            data = {}
            if os.path.exists(cache):
                with open(cache) as fh:
                    data = json.load(fh)
            data[key] = {"best": out, "table": rows}
            with open(cache, "w") as fh:
                json.dump(data, fh, indent=1)
        except (OSError, ValueError):
            pass
    return out, rows


class StepGraph:
    """One captured training step over a fixed set of views."""

    def __init__(self, ctx, params, cams, targets, *, grads=None, adam_m=None, adam_v=None,
                 with_adam=True, lr=None, betas=(0.9, 0.999), eps=1e-15, lam=0.2,
                 render=None, first_step=1, capacity_slack=1.25, stream=None):
        self.ctx = ctx
        self.params = params
        self.cams = list(cams)
        dev = params.means.device
        self.grads = grads if grads is not None else params.zeros_like()
        self.m = adam_m if adam_m is not None else params.zeros_like()
        self.v = adam_v if adam_v is not None else params.zeros_like()
        self.targets = [t.contiguous() for t in targets]
        self.images = [torch.empty((3, c.height, c.width), device=dev) for c in self.cams]
        self.dl = [torch.empty_like(i) for i in self.images]
        self.loss = torch.empty(1, device=dev)
        r = dict(tile=16, lds_depth=256, flags=0) if render is None else render
        lr = dict(DEFAULT_LR if lr is None else lr)
        self._cam_arr = _cam_array(self.cams)
        self._img, self._k1 = L.ptr_array([t.data_ptr() for t in self.images])
        self._tgt, self._k2 = L.ptr_array([t.data_ptr() for t in self.targets])
        self._dl, self._k3 = L.ptr_array([t.data_ptr() for t in self.dl])
        d = L.GsStepDesc()
        d.params, d.grads, d.adam_m, d.adam_v = (params.abi(), self.grads.abi(), self.m.abi(),
                                                 self.v.abi())
        d.cams = C.cast(self._cam_arr, C.POINTER(L.GsCamera))
        d.n_views = len(self.cams)
        d.images, d.targets, d.dl_dimg = self._img, self._tgt, self._dl
        d.loss = self.loss.data_ptr()
        d.render.tile, d.render.lds_depth, d.render.flags = r["tile"], r["lds_depth"], r["flags"]
        d.adam = L.GsAdamOpts(lr["means"], lr["log_scales"], lr["quats"], lr["opacity_logits"],
                              lr["sh_dc"], lr["sh_rest"], betas[0], betas[1], eps, 0)
        d.with_adam = 1 if with_adam else 0
        d.lambda_dssim = lam
        d.first_step = first_step
        d.capacity_slack = capacity_slack
        self._desc = d
        self.render = r
        self.handle = C.c_void_p()
        L.check(L.lib().gs_step_graph_create(ctx.handle, C.byref(d), C.byref(self.handle),
                                             _stream(stream)))

    def launch(self, stream=None):
        L.check(L.lib().gs_step_graph_launch(self.handle, _stream(stream)))

    def sync(self, stream=None):
        over, rec = C.c_int32(), C.c_int64()
        L.check(L.lib().gs_step_graph_sync(self.handle, C.byref(over), C.byref(rec),
                                           _stream(stream)))
        return bool(over.value), rec.value

    def run(self, stream=None):
        rec = C.c_int64()
        L.check(L.lib().gs_step_graph_run(self.handle, C.byref(rec), _stream(stream)))
        return rec.value

    def info(self):
        cap, rec, fr = C.c_int64(), C.c_int64(), C.c_void_p()
        L.check(L.lib().gs_step_graph_info(self.handle, C.byref(cap), C.byref(rec),
                                           C.byref(fr)))
        return cap.value, rec.value

    def close(self):
        if getattr(self, "handle", None):
            L.lib().gs_step_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
