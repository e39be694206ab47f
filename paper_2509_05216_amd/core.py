"""Python face of the isogs C ABI: torch tensors in, device pointers out.

PyTorch provides device memory and streams only; each function here checks
shapes, gathers pointers and calls one C entry point on the current stream.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L

PARAM_KEYS = ("means", "log_scales", "quats", "opacity_logits", "sh")


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


class Context:
    """A library context on one device (owns the library's device scratch)."""

    def __init__(self, device=0, mem_budget=0):
        self.device = int(device)
        h = C.c_void_p()
        L.check(L.lib().gs_ctx_create(self.device, C.c_size_t(mem_budget), C.byref(h)))
        self.handle = h

    def memory(self):
        a, b = C.c_size_t(), C.c_size_t()
        L.check(L.lib().gs_ctx_memory(self.handle, C.byref(a), C.byref(b)))
        return a.value, b.value

    def set_timing(self, enable=True):
        """Bracket every stage with HIP events (resets the totals)."""
        L.check(L.lib().gs_ctx_set_timing(self.handle, 1 if enable else 0))

    def stage_times(self):
        """{stage name: (total ms, launches)} of the timed stages."""
        out = {}
        i = 0
        while True:
            name = L.lib().gs_stage_name(i)
            if name is None:
                break
            ms, cnt = C.c_double(), C.c_int64()
            L.check(L.lib().gs_ctx_stage_time(self.handle, i, C.byref(ms), C.byref(cnt)))
            out[name.decode()] = (ms.value, cnt.value)
            i += 1
        return out

    def close(self):
        if getattr(self, "handle", None):
            L.lib().gs_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Params:
    """SoA float32 device tensors of one scene (or its gradients / moments)."""
    means: torch.Tensor
    log_scales: torch.Tensor
    quats: torch.Tensor
    opacity_logits: torch.Tensor
    sh: torch.Tensor
    sh_degree: int

    @property
    def n(self):
        return int(self.means.shape[1])

    def tensors(self):
        return [getattr(self, k) for k in PARAM_KEYS]

    def abi(self):
        n = self.n
        shapes = {"means": (3, n), "log_scales": (3, n), "quats": (4, n),
                  "opacity_logits": (n,), "sh": ((self.sh_degree + 1) ** 2 * 3, n)}
        for k in PARAM_KEYS:
            t = getattr(self, k)
            if tuple(t.shape) != shapes[k] or t.dtype != torch.float32 or not t.is_cuda \
                    or not t.is_contiguous():
                raise ValueError(f"{k}: expected contiguous float32 device tensor of shape "
                                 f"{shapes[k]}, got {tuple(t.shape)} {t.dtype} {t.device}")
        return L.GsParams(*(t.data_ptr() for t in self.tensors()), n, self.sh_degree, 0)

    def zeros_like(self):
        return Params(*(torch.zeros_like(t) for t in self.tensors()), self.sh_degree)

    @staticmethod
    def from_numpy(d, device="cuda"):
        return Params(*(torch.as_tensor(np.ascontiguousarray(d[k], np.float32), device=device)
                        for k in PARAM_KEYS), int(d["sh_degree"]))

    def to_numpy(self):
        out = {k: getattr(self, k).detach().cpu().numpy() for k in PARAM_KEYS}
        out["sh_degree"] = self.sh_degree
        return out


def camera(R, t, fx, fy, cx, cy, width, height, z_near=0.2):
    c = L.GsCamera()
    R = np.asarray(R, np.float64).ravel()
    t = np.asarray(t, np.float64).ravel()
    for k in range(9):
        c.R[k] = float(R[k])
    for k in range(3):
        c.t[k] = float(t[k])
    c.fx, c.fy, c.cx, c.cy, c.z_near = float(fx), float(fy), float(cx), float(cy), float(z_near)
    c.width, c.height = int(width), int(height)
    return c


def camera_from_dict(d):
    return camera(d["R"], d["t"], d["fx"], d["fy"], d["cx"], d["cy"], d["width"], d["height"],
                  d.get("z_near", 0.2))


def camera_to_dict(c):
    return dict(R=np.array(list(c.R), np.float64).reshape(3, 3), t=np.array(list(c.t), np.float64),
                fx=float(c.fx), fy=float(c.fy), cx=float(c.cx), cy=float(c.cy),
                width=int(c.width), height=int(c.height), z_near=float(c.z_near))


def orbit_cameras(n_views, radius, fov_y_deg, width, height):
    arr = (L.GsCamera * n_views)()
    L.check(L.lib().gs_orbit_cameras(n_views, radius, fov_y_deg, width, height, arr))
    return list(arr)


def _cam_array(cams):
    arr = (L.GsCamera * len(cams))()
    for i, c in enumerate(cams):
        arr[i] = c
    return arr


class Frame:
    """Forward state kept by the library for the backward pass."""

    def __init__(self):
        self.handle = C.c_void_p()

    def stats(self):
        s = L.GsFrameStats()
        L.check(L.lib().gs_frame_stats_get(self.handle, C.byref(s)))
        return {f: getattr(s, f) for f, _ in s._fields_}

    def export(self, what, view=-1, device="cuda", stream=None):
        st = self.stats()
        code = L.EXPORT[what]
        n = st["n_gaussians"]
        if what == "keys":
            out = torch.empty(max(st["n_records"], 1), dtype=torch.int64, device=device)
            count = st["n_records"]
        elif what == "values":
            out = torch.empty(max(st["n_records"], 1), dtype=torch.int32, device=device)
            count = st["n_records"]
        elif what == "ranges":
            out = torch.empty(st["n_tiles"] * 2, dtype=torch.int32, device=device)
            count = None
        elif what in ("final_T", "n_contrib"):
            out = torch.empty(st["n_pixels"], dtype=torch.float32 if what == "final_T"
                              else torch.int32, device=device)
            count = None
        elif what == "screen_grads":
            out = torch.empty(st["n_views"] * 12 * n, dtype=torch.float32, device=device)
            count = None
        elif what == "splats":
            out = torch.empty(st["n_views"] * n * 12, dtype=torch.float32, device=device)
            count = None
        elif what == "rects":
            out = torch.empty(st["n_views"] * n * 2, dtype=torch.int32, device=device)
            count = None
        elif what == "depths":
            out = torch.empty(st["n_views"] * n, dtype=torch.int32, device=device)
            count = None
        else:
            raise KeyError(what)
        if count == 0:
            return out[:0]
        L.check(L.lib().gs_frame_export(self.handle, code, view, _ptr(out),
                                        out.numel() * out.element_size(), _stream(stream)))
        return out

    def release(self):
        if self.handle:
            L.lib().gs_frame_release(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


PERSISTENT = 1
LONGEST_FIRST = 2
RADII = 4


def _opts(tile, lds_depth, bg, flags=0):
    o = L.GsRenderOpts()
    o.tile, o.lds_depth, o.flags = int(tile), int(lds_depth), int(flags)
    for k in range(3):
        o.bg[k] = float(bg[k])
    return o


def render_fwd(ctx, params, cams, images=None, *, tile=16, lds_depth=256, bg=(0.0, 0.0, 0.0),
               flags=0, frame=None, stream=None):
    """Render len(cams) views; returns (images [list of (3, H, W) tensors], frame)."""
    dev = params.means.device
    if images is None:
        images = [torch.empty((3, c.height, c.width), dtype=torch.float32, device=dev)
                  for c in cams]
    for img, c in zip(images, cams):
        if tuple(img.shape) != (3, c.height, c.width) or not img.is_contiguous() \
                or img.dtype != torch.float32:
            raise ValueError("image tensors must be contiguous float32 (3, H, W)")
    frame = frame if frame is not None else Frame()
    pa, keep = L.ptr_array([i.data_ptr() for i in images])
    o = _opts(tile, lds_depth, bg, flags)
    L.check(L.lib().gs_render_fwd(ctx.handle, params.abi(), _cam_array(cams), len(cams), pa,
                                  C.byref(o), C.byref(frame.handle), _stream(stream)))
    frame.ctx = ctx  # the frame is released before its context is
    return images, frame


def render_fwd_multi(ctx, params_per_view, cams, images=None, *, tile=16, lds_depth=256,
                     bg=(0.0, 0.0, 0.0), flags=0, frame=None, stream=None):
    """Render view v of scene params_per_view[v] (views of several scenes in one
    forward); returns (images, frame).  Forward only."""
    if len(params_per_view) != len(cams):
        raise ValueError("one parameter set per camera")
    dev = params_per_view[0].means.device
    if images is None:
        images = [torch.empty((3, c.height, c.width), dtype=torch.float32, device=dev)
                  for c in cams]
    for img, c in zip(images, cams):
        if tuple(img.shape) != (3, c.height, c.width) or not img.is_contiguous() \
                or img.dtype != torch.float32:
            raise ValueError("image tensors must be contiguous float32 (3, H, W)")
    frame = frame if frame is not None else Frame()
    pa, keep = L.ptr_array([i.data_ptr() for i in images])
    parr = (L.GsParams * len(cams))(*[p.abi() for p in params_per_view])
    o = _opts(tile, lds_depth, bg, flags)
    L.check(L.lib().gs_render_fwd_multi(ctx.handle, parr, _cam_array(cams), len(cams), pa,
                                        C.byref(o), C.byref(frame.handle), _stream(stream)))
    frame.ctx = ctx
    return images, frame


def loss_grad(ctx, rendered, targets, cams, lam=0.2, *, want_grad=True, stream=None):
    """Loss (device scalar tensor) and per-view image gradients."""
    dev = rendered[0].device
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    grads = [torch.empty_like(r) for r in rendered] if want_grad else None
    loss_grad_into(ctx, rendered, [t.contiguous() for t in targets], cams, loss, grads, lam,
                   stream=stream)
    return loss, grads


def loss_grad_into(ctx, rendered, targets, cams, loss, grads, lam=0.2, *, noalloc=False,
                   stream=None):
    """Loss and image gradients into caller tensors (loss: float32 (1,), grads: a list
    like `rendered`, or None).  noalloc=True calls gs_loss_grad_noalloc, whose
    workspace is a fixed device array (views of at most 2^20 pixels)."""
    for t in targets:
        if not t.is_contiguous():
            raise ValueError("target tensors must be contiguous")
    ra, k1 = L.ptr_array([r.data_ptr() for r in rendered])
    ta, k2 = L.ptr_array([t.data_ptr() for t in targets])
    ga, k3 = (L.ptr_array([g.data_ptr() for g in grads]) if grads is not None else (None, None))
    fn = L.lib().gs_loss_grad_noalloc if noalloc else L.lib().gs_loss_grad
    L.check(fn(ctx.handle, ra, ta, _cam_array(cams), len(cams), float(lam),
               _ptr(loss) if loss is not None else None, ga, _stream(stream)))


def image_metrics(ctx, rendered, references, cams, stream=None):
    """Per-view (mse, psnr, l1, ssim) as a float32 device tensor (n_views, 4)."""
    out = torch.empty((len(cams), 4), dtype=torch.float32, device=rendered[0].device)
    refs = [t.contiguous() for t in references]
    ra, k1 = L.ptr_array([r.data_ptr() for r in rendered])
    ta, k2 = L.ptr_array([t.data_ptr() for t in refs])
    L.check(L.lib().gs_image_metrics(ctx.handle, ra, ta, _cam_array(cams), len(cams), _ptr(out),
                                     _stream(stream)))
    return out


BWD_ACCUMULATE = 1
BWD_KEEP_SCREEN = 2


def render_bwd(ctx, frame, params, dl_dimg, grads=None, *, accumulate=False, keep_screen=False,
               stream=None):
    """Parameter gradients of the frame's forward for upstream image gradients.

    keep_screen: leave the screen-space sums in the frame for
    ``frame.export("screen_grads")`` (the next forward clears them)."""
    if grads is None:
        grads = params.zeros_like() if accumulate else Params(
            *(torch.empty_like(t) for t in params.tensors()), params.sh_degree)
    da, keep = L.ptr_array([d.contiguous().data_ptr() for d in dl_dimg])
    flags = (BWD_ACCUMULATE if accumulate else 0) | (BWD_KEEP_SCREEN if keep_screen else 0)
    L.check(L.lib().gs_render_bwd(ctx.handle, frame.handle, params.abi(), da, grads.abi(),
                                  flags, _stream(stream)))
    return grads


DEFAULT_LR = dict(means=1.6e-4 * 2.5, log_scales=5e-3, quats=1e-3, opacity_logits=5e-2,
                  sh_dc=2.5e-3, sh_rest=2.5e-3 / 20.0)


def adam_step(ctx, p, g, m, v, step, *, lr=None, betas=(0.9, 0.999), eps=1e-15,
              zero_grads=False, stream=None):
    lr = dict(DEFAULT_LR if lr is None else lr)
    o = L.GsAdamOpts(lr["means"], lr["log_scales"], lr["quats"], lr["opacity_logits"],
                     lr["sh_dc"], lr["sh_rest"], betas[0], betas[1], eps, 1 if zero_grads else 0)
    L.check(L.lib().gs_adam_step(ctx.handle, p.abi(), g.abi(), m.abi(), v.abi(), C.byref(o),
                                 int(step), _stream(stream)))


def init_from_points(ctx, xyz, sh_degree, *, log_scale=0.0, log_scale_jitter=0.0,
                     log_scale_range=None, random_quats=False, opacity_logit=0.1, sh_std=0.0,
                     seed=0, stream=None):
    """Gaussians from (3, n) points: a device tensor, or host data (a CPU tensor or a
    numpy array, copied by the library); returns Params on the context's device."""
    if isinstance(xyz, np.ndarray) or not xyz.is_cuda:
        host = np.ascontiguousarray(xyz.numpy() if torch.is_tensor(xyz) else xyz, np.float32)
        n = int(host.shape[1])
        dev = torch.device("cuda", ctx.device)
        ptr = host.ctypes.data_as(C.c_void_p)
    else:
        xyz = xyz.contiguous()
        n = int(xyz.shape[1])
        dev = xyz.device
        ptr = _ptr(xyz)
    p = Params(torch.empty((3, n), device=dev), torch.empty((3, n), device=dev),
               torch.empty((4, n), device=dev), torch.empty((n,), device=dev),
               torch.empty(((sh_degree + 1) ** 2 * 3, n), device=dev), sh_degree)
    lo, hi = (log_scale_range if log_scale_range is not None else (0.0, 0.0))
    o = L.GsInitOpts(log_scale, log_scale_jitter, lo, hi, 1 if random_quats else 0,
                     opacity_logit, sh_std, 0)
    L.check(L.lib().gs_init_from_points(ctx.handle, ptr, n, C.byref(o),
                                        C.c_uint64(seed), p.abi(), _stream(stream)))
    return p


def bw_probe(ctx, src, dst, stream=None):
    """Copy src -> dst (same-size contiguous device tensors) with the probe kernel."""
    nbytes = src.numel() * src.element_size()
    L.check(L.lib().gs_bw_probe(ctx.handle, _ptr(src), _ptr(dst), nbytes, _stream(stream)))
