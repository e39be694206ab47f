"""Adaptive density control (clone, split, prune, opacity reset) through the C ABI.

``DensityStats`` holds the per-Gaussian statistics on the device;
``accumulate`` adds a frame's views to them (the frame rendered with
``RADII`` and its backward run with ``keep_screen=True``); ``densify`` returns
the new parameter set and Adam moments (sized by a counting call, then
written by the library); ``opacity_reset`` clamps opacities in place.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _lib as L
from .core import Params, _stream

DEFAULTS = dict(grad_threshold=0.0002, percent_dense=0.01, min_opacity=0.005, max_screen=0.0,
                max_world=0.1, split_div=1.6, n_split=2)


@dataclass
class DensityStats:
    grad: torch.Tensor        # float32 (n,)
    count: torch.Tensor       # int32 (n,)
    max_radius: torch.Tensor  # int32 (n,)

    @staticmethod
    def zeros(n, device="cuda"):
        return DensityStats(torch.zeros(n, dtype=torch.float32, device=device),
                            torch.zeros(n, dtype=torch.int32, device=device),
                            torch.zeros(n, dtype=torch.int32, device=device))

    @property
    def n(self):
        return int(self.grad.shape[0])

    def abi(self):
        for t, dt in ((self.grad, torch.float32), (self.count, torch.int32),
                      (self.max_radius, torch.int32)):
            if t.dtype != dt or not t.is_cuda or not t.is_contiguous() or t.shape != (self.n,):
                raise ValueError("statistics: contiguous device tensors of shape (n,), "
                                 "float32 grad and int32 count / max_radius")
        return L.GsDensityStats(self.grad.data_ptr(), self.count.data_ptr(),
                                self.max_radius.data_ptr(), self.n)

    def zero_(self):
        self.grad.zero_()
        self.count.zero_()
        self.max_radius.zero_()


def accumulate(ctx, frame, stats, scale=1.0, stream=None):
    L.check(L.lib().gs_density_accumulate(ctx.handle, frame.handle, stats.abi(), float(scale),
                                          _stream(stream)))


def _opts(extent, seed, **kw):
    d = dict(DEFAULTS)
    unknown = set(kw) - set(d)
    if unknown:
        raise TypeError(f"unknown density options {sorted(unknown)}")
    d.update(kw)
    return L.GsDensityOpts(d["grad_threshold"], d["percent_dense"], d["min_opacity"],
                           d["max_screen"], d["max_world"], float(extent), d["split_div"],
                           int(d["n_split"]), 0, int(seed) & 0xFFFFFFFFFFFFFFFF)


def _info(i):
    return {k: int(getattr(i, k)) for k, _ in L.GsDensityInfo._fields_}


def _empty(n, sh_degree, device):
    rows = (sh_degree + 1) ** 2 * 3
    return Params(torch.empty((3, n), device=device), torch.empty((3, n), device=device),
                  torch.empty((4, n), device=device), torch.empty((n,), device=device),
                  torch.empty((rows, n), device=device), sh_degree)


def count(ctx, params, m, v, stats, extent, *, seed=0, stream=None, **opts):
    """The counts of a densification (nothing is written)."""
    o = _opts(extent, seed, **opts)
    info = L.GsDensityInfo()
    null = L.GsParams()
    L.check(L.lib().gs_densify(ctx.handle, params.abi(), m.abi(), v.abi(), stats.abi(),
                               C.byref(o), null, null, null, None, C.byref(info),
                               _stream(stream)))
    return _info(info)


def densify(ctx, params, m, v, stats, extent, *, seed=0, want_src=False, stream=None, **opts):
    """(params, m, v, info[, src_index]) of the densified set."""
    info = count(ctx, params, m, v, stats, extent, seed=seed, stream=stream, **opts)
    n_out = info["n_out"]
    dev = params.means.device
    po, mo, vo = (_empty(n_out, params.sh_degree, dev) for _ in range(3))
    src = torch.empty(n_out, dtype=torch.int32, device=dev) if want_src else None
    if n_out == 0:                      # everything pruned: nothing to write
        res = (po, mo, vo, info)
        return res + (src,) if want_src else res
    o = _opts(extent, seed, **opts)
    out = L.GsDensityInfo()
    L.check(L.lib().gs_densify(ctx.handle, params.abi(), m.abi(), v.abi(), stats.abi(),
                               C.byref(o), po.abi(), mo.abi(), vo.abi(),
                               C.c_void_p(src.data_ptr()) if src is not None else None,
                               C.byref(out), _stream(stream)))
    res = (po, mo, vo, _info(out))
    return res + (src,) if want_src else res


def opacity_reset(ctx, params, m, v, max_opacity=0.01, stream=None):
    L.check(L.lib().gs_opacity_reset(ctx.handle, params.abi(), m.abi(), v.abi(),
                                     float(max_opacity), _stream(stream)))
