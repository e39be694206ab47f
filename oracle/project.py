"""EWA projection of anisotropic 3-D Gaussians, tile rectangles and SH colour.

The paper initialises 3D-GS primitives from isosurface points and trains the
cited 3D-GS model on orbit views (Sec. III); the projection is that model's
elliptical-weighted-average splat.  Readings used (each a choice where the
paper is silent):

* camera-space centre t = R mu + t_cam, culled when t_z <= z_near (0.2);
* Sigma3 = M M^T with M = R(q / |q|) diag(exp(log_scale));
* Jacobian of the perspective map at t, with t_x / t_z and t_y / t_z clamped to
  +-1.3 tan(fov/2) (guard band; the clamp has zero derivative);
* Sigma2 = J R Sigma3 R^T J^T + 0.3 I (low-pass), culled when det <= 0;
* conic = Sigma2^-1; radius r = ceil(3 sqrt(lambda_max(Sigma2)));
* mean2D = (fx t_x / t_z + cx, fy t_y / t_z + cy); depth = t_z;
* pixel rectangle: centres within [m - r, m + r] per axis, clamped to the
  image; tile rectangle floor(lo / T)..floor(hi / T);
* opacity = sigmoid(logit); rgb = max(0, sum_j sh_j Y_j(d) + 0.5) with d the
  unit vector from the camera centre to mu.

Scalar expressions are written element by element in a fixed order so that the
integer decisions (cull, radius, rectangle) and the float32 depth used in sort
keys are reproducible by any IEEE float64 evaluation of the same formulas.
"""
from __future__ import annotations

import numpy as np

from . import sh as _sh
from .camera import center

LOWPASS = 0.3
GUARD = 1.3


def quat_to_rot(qn):
    """Rotation matrices (3, 3, N) of unit quaternions qn = (w, x, y, z) (4, N)."""
    w, x, y, z = qn
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def project(params, cam, tile):
    """Per-Gaussian screen-space state for one camera.

    Returns a dict of float64 arrays over the N Gaussians:
    ``tz, visible, m (2,N), conic (3,N), cov2 (3,N), radius (int), rect (4,N:
    tile x0,y0,x1,y1 inclusive), tiles (int), opacity, rgb (3,N), clamped
    (3,N bool), depth32 (float32)`` plus intermediates for the backward pass.
    """
    mu = np.asarray(params["means"], np.float64)
    ls = np.asarray(params["log_scales"], np.float64)
    q = np.asarray(params["quats"], np.float64)
    logit = np.asarray(params["opacity_logits"], np.float64)
    shc = np.asarray(params["sh"], np.float64)
    deg = int(params["sh_degree"])
    R = np.asarray(cam["R"], np.float64)
    tc = np.asarray(cam["t"], np.float64)
    fx, fy, cx, cy = cam["fx"], cam["fy"], cam["cx"], cam["cy"]
    W, H = int(cam["width"]), int(cam["height"])
    n = mu.shape[1]

    # camera-space centre, one product-sum per row in a fixed order
    t = np.empty((3, n))
    for r in range(3):
        t[r] = R[r, 0] * mu[0] + R[r, 1] * mu[1] + R[r, 2] * mu[2] + tc[r]
    tx, ty, tz = t
    visible = tz > cam["z_near"]
    tzs = np.where(visible, tz, 1.0)

    # 3-D covariance from rotation and scale
    s = np.exp(ls)
    qnorm = np.sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3])
    qn = q / qnorm
    Rq = quat_to_rot(qn)
    M = Rq * s[None, :, :]
    Sig = np.einsum("ikn,jkn->ijn", M, M)

    # perspective Jacobian with guard band
    limx = GUARD * (0.5 * W / fx)
    limy = GUARD * (0.5 * H / fy)
    xz = tx / tzs
    yz = ty / tzs
    u = np.clip(xz, -limx, limx)
    v = np.clip(yz, -limy, limy)
    J = np.zeros((2, 3, n))
    J[0, 0] = fx / tzs
    J[0, 2] = -fx * u / tzs
    J[1, 1] = fy / tzs
    J[1, 2] = -fy * v / tzs
    T = np.einsum("ikn,kj->ijn", J, R)
    cov = np.einsum("ikn,kln,jln->ijn", T, Sig, T)
    a = cov[0, 0] + LOWPASS
    b = cov[0, 1]
    c = cov[1, 1] + LOWPASS
    det = a * c - b * b
    ok = visible & (det > 0)
    dets = np.where(ok, det, 1.0)
    conic = np.stack([c / dets, -b / dets, a / dets], 0)
    half = 0.5 * (a - c)
    lmax = 0.5 * (a + c) + np.sqrt(half * half + b * b)
    radius = np.where(ok, np.ceil(3.0 * np.sqrt(np.maximum(lmax, 0.0))), 0.0)

    mx = fx * xz + cx
    my = fy * yz + cy
    # pixel rectangle: centres inside [m - r, m + r], clamped to the image
    lox = np.ceil(mx - 0.5 - radius)
    hix = np.floor(mx - 0.5 + radius)
    loy = np.ceil(my - 0.5 - radius)
    hiy = np.floor(my - 0.5 + radius)
    lox, loy = np.maximum(lox, 0), np.maximum(loy, 0)
    hix, hiy = np.minimum(hix, W - 1), np.minimum(hiy, H - 1)
    touched = ok & (radius > 0) & (lox <= hix) & (loy <= hiy)
    rect = np.zeros((4, n), np.int64)
    rect[0] = np.where(touched, np.floor(lox / tile), 0)
    rect[1] = np.where(touched, np.floor(loy / tile), 0)
    rect[2] = np.where(touched, np.floor(hix / tile), -1)
    rect[3] = np.where(touched, np.floor(hiy / tile), -1)
    tiles = np.where(touched, (rect[2] - rect[0] + 1) * (rect[3] - rect[1] + 1), 0)

    opacity = 1.0 / (1.0 + np.exp(-logit))

    # view-dependent colour
    cpos = center(cam)
    dirv = mu - cpos[:, None]
    dlen = np.sqrt(dirv[0] ** 2 + dirv[1] ** 2 + dirv[2] ** 2)
    dhat = dirv / dlen
    Y = _sh.basis(dhat, deg)
    nb = (deg + 1) ** 2
    raw = np.stack([(shc[c::3][:nb] * Y).sum(0) for c in range(3)], 0) + 0.5
    clamped = raw < 0
    rgb = np.maximum(raw, 0.0)

    return dict(
        t=t, tz=tz, visible=visible, ok=ok, touched=touched, m=np.stack([mx, my], 0),
        conic=conic, cov2=np.stack([a, b, c], 0), det=det, radius=radius.astype(np.int64),
        rect=rect, tiles=tiles.astype(np.int64), opacity=opacity, rgb=rgb, clamped=clamped,
        depth32=tz.astype(np.float32), s=s, q=q, qnorm=qnorm, qn=qn, Rq=Rq, M=M, Sig=Sig,
        J=J, T=T, u=u, v=v, xz=xz, yz=yz, limx=limx, limy=limy, dirv=dirv, dlen=dlen,
        dhat=dhat, Y=Y, sh_degree=deg, W=W, H=H, tile=tile,
    )
