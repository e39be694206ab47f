"""Render server front end: resident scenes, request submission, latency stats.

A thin wrapper over the library's server (gs_server_*): the scheduling,
batching, memory admission and statistics all run in the library's worker
threads; this module keeps the scene tensors alive and marshals pointers.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib as L


class Server:
    def __init__(self, ctx, *, n_slots=4, max_batch_views=8, mem_budget=0, tile=16,
                 lds_depth=256, flags=0, bg=(0.0, 0.0, 0.0), max_queue=4096):
        self.ctx = ctx
        o = L.GsServerOpts()
        o.n_slots, o.max_batch_views, o.mem_budget = n_slots, max_batch_views, mem_budget
        o.render.tile, o.render.lds_depth, o.render.flags = tile, lds_depth, flags
        for k in range(3):
            o.render.bg[k] = bg[k]
        o.max_queue = max_queue
        self.handle = C.c_void_p()
        L.check(L.lib().gs_server_create(ctx.handle, C.byref(o), C.byref(self.handle)))
        self._scenes = []

    def add_scene(self, params):
        sid = C.c_int32()
        L.check(L.lib().gs_server_add_scene(self.handle, params.abi(), C.byref(sid)))
        self._scenes.append(params)
        return sid.value

    def submit(self, scene, cam, out=None):
        """Queue a render; returns (ticket, output tensor)."""
        if out is None:
            known = 0 <= scene < len(self._scenes)
            dev = self._scenes[scene].means.device if known else torch.device("cuda")
            out = torch.empty((3, cam.height, cam.width), dtype=torch.float32, device=dev)
        t = C.c_uint64()
        L.check(L.lib().gs_server_submit(self.handle, scene, C.byref(cam),
                                         C.c_void_p(out.data_ptr()), C.byref(t)))
        return t.value, out

    def poll(self, ticket):
        done, lat = C.c_int32(), C.c_double()
        L.check(L.lib().gs_server_poll(self.handle, ticket, C.byref(done), C.byref(lat)))
        return bool(done.value), lat.value

    def wait(self, ticket):
        lat = C.c_double()
        L.check(L.lib().gs_server_wait(self.handle, ticket, C.byref(lat)))
        return lat.value

    def drain(self):
        L.check(L.lib().gs_server_drain(self.handle))

    def stats(self):
        s = L.GsServeStats()
        L.check(L.lib().gs_server_stats(self.handle, C.byref(s)))
        return {f: getattr(s, f) for f, _ in s._fields_}

    def reset_stats(self):
        L.check(L.lib().gs_server_reset_stats(self.handle))

    def close(self):
        if getattr(self, "handle", None):
            L.lib().gs_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
