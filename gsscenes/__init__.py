"""Seeded synthetic inputs: analytic fields, isosurface points, parameter draws
and ray-cast target images.  Shared by the tests, the oracle runs and the
benchmark; it contains none of the rasterizer's arithmetic."""
from .configs import PRESETS, Scene, ViewSet, arrival_times, make_field, make_scene
from .params import n_sh_rows, subset, synth_params
from .raycast import raycast
from .volume import sample_points_grid, sample_volume
