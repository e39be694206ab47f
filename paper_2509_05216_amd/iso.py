"""Isosurface points and ray-cast target views of a device volume, through the C ABI.

``Volume`` wraps a contiguous float32 device tensor (nz, ny, nx) of vertex
values over a box.  ``extract`` returns the kept crossing points as a
(3, n) device tensor (a counting call sizes it); ``raycast`` renders target
views of the isosurface.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _lib as L
from .core import _cam_array, _stream


@dataclass
class Volume:
    values: torch.Tensor            # float32 (nz, ny, nx), contiguous, on the device
    lo: tuple = (-1.0, -1.0, -1.0)
    hi: tuple = (1.0, 1.0, 1.0)

    def abi(self):
        v = self.values
        if v.dim() != 3 or v.dtype != torch.float32 or not v.is_cuda or not v.is_contiguous():
            raise ValueError("volume: contiguous float32 device tensor (nz, ny, nx)")
        nz, ny, nx = v.shape
        return L.GsVolume(v.data_ptr(), nx, ny, nz, (C.c_float * 3)(*self.lo),
                          (C.c_float * 3)(*self.hi))


def extract(ctx, vol, iso=0.5, keep_prob=1.0, seed=0, stream=None):
    """(3, n) float32 device tensor of the kept crossing points."""
    n = C.c_int64()
    va = vol.abi()
    L.check(L.lib().gs_iso_extract(ctx.handle, va, float(iso), float(keep_prob),
                                   C.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), None, 0, C.byref(n),
                                   _stream(stream)))
    cap = max(n.value, 1)
    out = torch.empty((3, cap), dtype=torch.float32, device=vol.values.device)
    L.check(L.lib().gs_iso_extract(ctx.handle, va, float(iso), float(keep_prob),
                                   C.c_uint64(seed & 0xFFFFFFFFFFFFFFFF),
                                   C.c_void_p(out.data_ptr()), cap, C.byref(n),
                                   _stream(stream)))
    return out[:, :n.value]


def count(ctx, vol, iso=0.5, keep_prob=1.0, seed=0, stream=None):
    n = C.c_int64()
    L.check(L.lib().gs_iso_extract(ctx.handle, vol.abi(), float(iso), float(keep_prob),
                                   C.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), None, 0, C.byref(n),
                                   _stream(stream)))
    return n.value


def raycast(ctx, vol, cams, iso=0.5, step=0.01, images=None, stream=None):
    """Target images (list of (3, H, W) float32 device tensors) of the isosurface."""
    dev = vol.values.device
    if images is None:
        images = [torch.empty((3, c.height, c.width), dtype=torch.float32, device=dev)
                  for c in cams]
    pa, keep = L.ptr_array([i.data_ptr() for i in images])
    L.check(L.lib().gs_raycast(ctx.handle, vol.abi(), float(iso), _cam_array(cams), len(cams),
                               float(step), pa, _stream(stream)))
    return images
