"""isogs: MI355X-native differentiable tile rasterizer of 3-D Gaussians for
isosurface visualization (hot path of 3D-GS training: EWA projection, SH
colour, tile binning and sort, alpha compositing, its backward, the loss
gradient and Adam), behind the C ABI of include/isogs.h."""
from ._lib import IsogsError, lib  # noqa: F401
from .core import (Context, Frame, Params, adam_step, bw_probe, camera, camera_from_dict,  # noqa: F401
                   camera_to_dict, init_from_points, loss_grad, loss_grad_into, orbit_cameras, render_bwd, render_fwd_multi,
                   render_fwd)
from .autograd import RasterizeFn, rasterize  # noqa: F401
from .batched import StepGraph, autotune  # noqa: F401
from .serve import Server  # noqa: F401
from .train import Schedule, Trainer  # noqa: F401
from . import density  # noqa: F401
from .core import LONGEST_FIRST, PERSISTENT  # noqa: F401

__all__ = ["Context", "Frame", "Params", "IsogsError", "adam_step", "camera",
           "camera_from_dict", "camera_to_dict", "init_from_points", "loss_grad", "loss_grad_into", "lib",
           "orbit_cameras", "render_bwd", "render_fwd", "RasterizeFn", "rasterize"]
