"""Named synthetic workloads: tiny (10k), iso1m (1M), kingsnake4m (4M),
miranda18m (18M) and the serving mix.

Each preset fixes the field recipe, the grid size G, the Gaussian count, the
parameter draw and the view set (count, orbit radius, field of view, sizes).
Seeds: ``SeedSequence(1000 + index)`` spawns independent child streams for the
field, the points, the parameters and the request arrivals, so each part can
be regenerated on its own.  ``n`` and ``G`` may be overridden to get a smaller
scene of the same recipe (tests, CPU baselines).
"""
from __future__ import annotations

from dataclasses import dataclass, field as dfield

import numpy as np

from .fields import BlobField, MixingLayer, SpectralNoise, blob_field
from .iso import sample_points
from .params import synth_params

PRESETS = ("tiny", "iso1m", "kingsnake4m", "miranda18m", "serve")


@dataclass
class ViewSet:
    n_views: int
    radius: float
    fov_deg: float
    sizes: list                       # [(W, H), ...] cycled over views


@dataclass
class Scene:
    name: str
    field: object
    points: np.ndarray                # (N, 3) float64
    h: float
    params: dict
    views: ViewSet
    tile: int = 16
    extra: dict = dfield(default_factory=dict)


def _streams(index):
    ss = np.random.SeedSequence(1000 + index)
    return [np.random.default_rng(s) for s in ss.spawn(5)]


def make_field(name):
    idx = PRESETS.index(name)
    r_field = _streams(idx)[0]
    if name in ("tiny", "serve"):
        return blob_field(r_field, 8, 0.5, 0.15, 0.35), 64
    if name == "iso1m":
        noise = SpectralNoise(r_field, 48, 4 * np.pi, 16 * np.pi, 1.0, 0.1)
        return blob_field(r_field, 64, 0.6, 0.05, 0.2, noise), 512
    if name == "kingsnake4m":
        noise = SpectralNoise(r_field, 64, 4 * np.pi, 32 * np.pi, 1.0, 0.15)
        return blob_field(r_field, 128, 0.6, 0.03, 0.15, noise), 1024
    if name == "miranda18m":
        return MixingLayer(r_field, 64, 2.0 * 2.0 / 2047, 0.02, 2.0 / 2047), 2048
    raise KeyError(name)


def make_scene(name, n=None, G=None, progress=None):
    idx = PRESETS.index(name)
    _, r_pts, r_par, _, _ = _streams(idx)
    fld, G0 = make_field(name)
    G = G0 if G is None else G
    if name == "tiny":
        n = 10_000 if n is None else n
        pts, h = sample_points(fld, G, n, r_pts, progress=progress)
        params = synth_params(r_par, pts, sh_degree=0, log_scale=np.log(h),
                              opacity_logit=0.1)
        views = ViewSet(8, 2.5, 60.0, [(256, 256)])
    elif name == "iso1m":
        n = 1_000_000 if n is None else n
        pts, h = sample_points(fld, G, n, r_pts, progress=progress)
        params = synth_params(r_par, pts, sh_degree=3, log_scale_range=(-5.0, -3.0),
                              random_quats=True, opacity_logit=0.1, sh_std=0.1)
        views = ViewSet(128, 2.5, 60.0, [(1024, 1024)])
    elif name == "kingsnake4m":
        n = 4_000_000 if n is None else n
        pts, h = sample_points(fld, G, n, r_pts, progress=progress)
        params = synth_params(r_par, pts, sh_degree=3, log_scale=np.log(h),
                              log_scale_jitter=0.5, random_quats=True,
                              opacity_logit=0.1, sh_std=0.1)
        views = ViewSet(4, 2.5, 60.0, [(2048, 2048), (2048, 2048), (1536, 1536), (1536, 1536)])
    elif name == "miranda18m":
        n = 18_000_000 if n is None else n
        pts, h = sample_points(fld, G, n, r_pts, progress=progress)
        params = synth_params(r_par, pts, sh_degree=3, log_scale=np.log(h),
                              log_scale_jitter=0.5, random_quats=True,
                              opacity_logit=0.1, sh_std=0.1)
        views = ViewSet(2, 2.5, 60.0, [(4096, 4096)])
    elif name == "serve":
        n = 100_000 if n is None else n
        pts, h = sample_points(fld, G, n, r_pts, progress=progress)
        params = synth_params(r_par, pts, sh_degree=3, log_scale=np.log(h),
                              log_scale_jitter=0.5, random_quats=True,
                              opacity_logit_range=(0.0, 4.0), sh_std=0.1)
        views = ViewSet(1, 2.5, 60.0, [(512, 512), (1024, 1024), (2048, 2048)])
    else:
        raise KeyError(name)
    return Scene(name, fld, pts, h, params, views)


def arrival_times(rate_hz, n, seed_index=PRESETS.index("serve")):
    """Poisson arrival times (seconds) and uniform draws for scene/resolution."""
    rng = _streams(seed_index)[4]
    gaps = rng.exponential(1.0 / rate_hz, size=n)
    return np.cumsum(gaps), rng.random(n), rng.random(n)
