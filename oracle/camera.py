"""Pinhole cameras and the structured orbit of training views.

The paper generates "a set of synthetic camera views in a structured orbit"
around the volume (Sec. III) and uses 448 of them per dataset (Sec. IV); it
fixes no layout.  Reading used here: views on a Fibonacci sphere of the given
radius, each looking at the origin.

Conventions: world->camera rotation R (rows = camera x right, y down, z
forward) and translation t, so p_cam = R p + t; focal lengths in pixels from
the vertical field of view with square pixels; principal point at the image
centre; pixel (x, y) is sampled at (x + 0.5, y + 0.5).
"""
from __future__ import annotations

import math

import numpy as np

Z_NEAR = 0.2


def intrinsics(width, height, fov_y_deg):
    fy = height / (2.0 * math.tan(math.radians(fov_y_deg) / 2.0))
    return fy, fy, width / 2.0, height / 2.0


def look_at(center, target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0)):
    c = np.asarray(center, np.float64)
    f = np.asarray(target, np.float64) - c
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, np.float64))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f], 0)
    return R, -R @ c


def orbit_cameras(n_views, radius, fov_y_deg, width, height):
    """List of camera dicts (float64 values) on a Fibonacci sphere.

    View i of n sits at radius * (sqrt(1-y^2) cos(phi), y, sqrt(1-y^2) sin(phi))
    with y = 1 - 2 (i + 0.5) / n and phi = i * pi * (3 - sqrt(5)); world up is +y
    unless |y| > 0.99, where +z is used.
    """
    fx, fy, cx, cy = intrinsics(width, height, fov_y_deg)
    cams = []
    golden = math.pi * (3.0 - math.sqrt(5.0))
    for i in range(n_views):
        y = 1.0 - 2.0 * (i + 0.5) / n_views
        rxz = math.sqrt(max(0.0, 1.0 - y * y))
        phi = i * golden
        d = np.array([rxz * math.cos(phi), y, rxz * math.sin(phi)])
        up = (0.0, 0.0, 1.0) if abs(y) > 0.99 else (0.0, 1.0, 0.0)
        R, t = look_at(radius * d, up=up)
        cams.append(dict(R=R, t=t, fx=fx, fy=fy, cx=cx, cy=cy,
                         width=int(width), height=int(height), z_near=Z_NEAR))
    return cams


def to_float32(cam):
    """The camera as the float32 values a device consumes, widened back to float64."""
    out = dict(cam)
    for k in ("R", "t"):
        out[k] = np.asarray(cam[k], np.float32).astype(np.float64)
    for k in ("fx", "fy", "cx", "cy", "z_near"):
        out[k] = float(np.float32(cam[k]))
    return out


def center(cam):
    """Camera position in world space: -R^T t."""
    return -np.asarray(cam["R"]).T @ np.asarray(cam["t"])
