"""Pins of the oracle's cameras, projection, rectangles and SH against closed
forms, brute force and an independent library (scipy)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import camera, project, sh
from tests._util import identity_camera, make_params

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


# ---------------------------------------------------------------- cameras
def test_orbit_cameras_look_at_origin():
    cams = camera.orbit_cameras(16, 2.5, 60.0, 256, 256)
    ys = []
    for c in cams:
        R = c["R"]
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-12)
        assert abs(np.linalg.det(R) - 1) < 1e-12
        C = camera.center(c)
        assert abs(np.linalg.norm(C) - 2.5) < 1e-12
        o = R @ np.zeros(3) + c["t"]                 # origin in camera space
        assert abs(o[0]) < 1e-12 and abs(o[1]) < 1e-12 and abs(o[2] - 2.5) < 1e-12
        ys.append(C[1] / 2.5)
    # Fibonacci lattice: heights evenly spaced, azimuth steps by the golden angle
    assert np.allclose(np.diff(ys), -2.0 / 16, atol=1e-12)
    c0, c1 = camera.center(cams[0]), camera.center(cams[1])
    dphi = math.atan2(c1[2], c1[0]) - math.atan2(c0[2], c0[0])
    assert abs((dphi - math.pi * (3 - math.sqrt(5))) % (2 * math.pi)) < 1e-12


def test_image_axes_follow_world_up():
    # a camera on +z looking at the origin: world +x is image right, world +y is image up
    R, t = camera.look_at((0, 0, 2.5))
    assert np.allclose(R @ np.array([1, 0, 0.0]), [-1, 0, 0]) or np.allclose(R @ np.array([1, 0, 0.0]), [1, 0, 0])
    assert (R @ np.array([0, 1, 0.0]))[1] < 0          # world up -> image y decreasing


def test_intrinsics_from_fov():
    fx, fy, cx, cy = camera.intrinsics(256, 256, 60.0)
    assert abs(fx - GOLD["on_axis_tiny"]["fx"]) < 1e-9 and fx == fy and cx == 128 and cy == 128


# ---------------------------------------------------------------- projection
def test_isotropic_on_axis_closed_form():
    g = GOLD["on_axis_tiny"]
    cam = dict(camera.orbit_cameras(1, 2.5, 60.0, 256, 256)[0])
    cam["R"], cam["t"] = np.eye(3), np.array([0, 0, 2.5])
    p = make_params([[0, 0, 0]], log_scales=np.full(3, np.log(2 / 63)))
    pr = project.project(p, cam, 16)
    s32 = float(np.float32(np.log(2 / 63)))
    sig = cam["fx"] * math.exp(s32) / 2.5
    assert abs(pr["cov2"][0, 0] - (sig * sig + 0.3)) < 1e-9
    assert abs(pr["cov2"][2, 0] - (sig * sig + 0.3)) < 1e-9
    assert abs(pr["cov2"][1, 0]) < 1e-12
    assert abs(sig - g["sigma_px"]) < 1e-5
    assert pr["radius"][0] == g["radius"]
    assert tuple(pr["rect"][:, 0]) == (g["tile_lo"], g["tile_lo"], g["tile_hi"], g["tile_hi"])
    assert pr["tiles"][0] == g["tiles_touched"]
    lam = sig * sig + 0.3
    assert np.allclose(pr["conic"][:, 0], [1 / lam, 0, 1 / lam], rtol=1e-12)
    assert np.allclose(pr["m"][:, 0], [128, 128])


def test_isotropic_off_axis_closed_form():
    # Sigma2 = s^2 J J^T + 0.3 I for an isotropic Gaussian, any camera rotation
    rng = np.random.default_rng(0)
    cams = camera.orbit_cameras(5, 2.5, 60.0, 320, 240)
    for c in cams:
        mu = rng.uniform(-0.4, 0.4, 3)
        s = 0.03
        p = make_params([mu], log_scales=np.full(3, np.log(s)))
        pr = project.project(p, c, 16)
        t = c["R"] @ p["means"][:, 0].astype(np.float64) + c["t"]
        sc = math.exp(float(p["log_scales"][0, 0]))
        J = np.array([[c["fx"] / t[2], 0, -c["fx"] * t[0] / t[2] ** 2],
                      [0, c["fy"] / t[2], -c["fy"] * t[1] / t[2] ** 2]])
        cov = sc * sc * J @ J.T + 0.3 * np.eye(2)
        assert np.allclose(pr["cov2"][:, 0], [cov[0, 0], cov[0, 1], cov[1, 1]], rtol=1e-10)
        assert np.allclose(pr["m"][:, 0], [c["fx"] * t[0] / t[2] + c["cx"], c["fy"] * t[1] / t[2] + c["cy"]])
        assert abs(pr["tz"][0] - t[2]) < 1e-12


def test_anisotropic_rotation_about_view_axis():
    # scales (a, b) rotated by theta about the optical axis: Sigma2 = R2 diag R2^T + 0.3 I
    cam = identity_camera(256, 256, 200.0)
    z, sa, sb = 3.0, 0.05, 0.02
    for theta in (0.3, -1.1, 2.0):
        q = [math.cos(theta / 2), 0, 0, math.sin(theta / 2)]
        p = make_params([[0, 0, z]], log_scales=np.log([sa, sb, 0.01]), quats=q)
        pr = project.project(p, cam, 16)
        e = np.exp(p["log_scales"][:, 0].astype(np.float64))
        qq = p["quats"][:, 0].astype(np.float64)
        th = 2 * math.atan2(qq[3], qq[0])
        R2 = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
        D = np.diag([(200 * e[0] / z) ** 2, (200 * e[1] / z) ** 2])
        cov = R2 @ D @ R2.T + 0.3 * np.eye(2)
        assert np.allclose(pr["cov2"][:, 0], [cov[0, 0], cov[0, 1], cov[1, 1]], rtol=1e-6)


def test_guard_band_clamps_jacobian():
    cam = identity_camera(200, 200, 100.0)
    lim = 1.3 * 100 / 100.0                       # 1.3 tan(fov/2) with tan = (W/2)/fx = 1
    mu = [4.0, 0.0, 2.0]                          # x/z = 2 > 1.3
    p = make_params([mu], log_scales=np.full(3, np.log(0.05)))
    pr = project.project(p, cam, 16)
    s = math.exp(float(p["log_scales"][0, 0]))
    J = np.array([[100 / 2.0, 0, -100 * lim / 2.0], [0, 100 / 2.0, 0]])
    cov = s * s * J @ J.T + 0.3 * np.eye(2)
    assert np.allclose(pr["cov2"][:, 0], [cov[0, 0], cov[0, 1], cov[1, 1]], rtol=1e-10)


def test_near_plane_and_degenerate_cull():
    cam = identity_camera()
    p = make_params([[0, 0, 0.1], [0, 0, 0.19], [0, 0, 0.21], [0, 0, -3]])
    pr = project.project(p, cam, 16)
    assert list(pr["touched"]) == [False, False, True, False]
    assert list(pr["tiles"][[0, 1, 3]]) == [0, 0, 0]


def test_rect_matches_pixel_brute_force():
    rng = np.random.default_rng(1)
    cam = camera.orbit_cameras(3, 2.5, 60.0, 100, 70)[1]
    n = 400
    p = make_params(rng.uniform(-1.2, 1.2, (n, 3)), log_scales=rng.uniform(-5, -2, (3, n)),
                    quats=rng.normal(size=(4, n)))
    for tile in (8, 16, 32):
        pr = project.project(p, cam, tile)
        xs = np.arange(100) + 0.5
        ys = np.arange(70) + 0.5
        for g in range(n):
            if not pr["ok"][g]:
                assert pr["tiles"][g] == 0
                continue
            r = pr["radius"][g]
            inx = np.nonzero((xs >= pr["m"][0, g] - r) & (xs <= pr["m"][0, g] + r))[0]
            iny = np.nonzero((ys >= pr["m"][1, g] - r) & (ys <= pr["m"][1, g] + r))[0]
            if inx.size == 0 or iny.size == 0:
                assert pr["tiles"][g] == 0
                continue
            want = (inx[0] // tile, iny[0] // tile, inx[-1] // tile, iny[-1] // tile)
            assert tuple(pr["rect"][:, g]) == want
            assert pr["tiles"][g] == (want[2] - want[0] + 1) * (want[3] - want[1] + 1)


def test_radius_is_three_sigma_of_major_axis():
    rng = np.random.default_rng(2)
    cam = camera.orbit_cameras(2, 2.5, 60.0, 256, 256)[0]
    n = 200
    p = make_params(rng.uniform(-0.5, 0.5, (n, 3)), log_scales=rng.uniform(-5, -2.5, (3, n)),
                    quats=rng.normal(size=(4, n)))
    pr = project.project(p, cam, 16)
    for g in np.nonzero(pr["ok"])[0]:
        a, b, c = pr["cov2"][:, g]
        lmax = np.linalg.eigvalsh(np.array([[a, b], [b, c]]))[-1]
        assert pr["radius"][g] == math.ceil(3 * math.sqrt(lmax) - 1e-12) or \
            abs(3 * math.sqrt(lmax) - round(3 * math.sqrt(lmax))) < 1e-9


def test_opacity_is_sigmoid():
    p = make_params([[0, 0, 3]] * 3, logits=[-2.0, 0.1, 4.0])
    pr = project.project(p, identity_camera(), 16)
    x = p["opacity_logits"].astype(np.float64)
    assert np.allclose(pr["opacity"], 1 / (1 + np.exp(-x)), rtol=1e-15)


# ---------------------------------------------------------------- SH
def _sphere_quadrature(nt=40, nphi=80):
    xg, wg = np.polynomial.legendre.leggauss(nt)      # cos(theta) nodes
    phi = (np.arange(nphi) + 0.5) * 2 * np.pi / nphi
    ct, ph = np.meshgrid(xg, phi, indexing="ij")
    st = np.sqrt(1 - ct * ct)
    d = np.stack([st * np.cos(ph), st * np.sin(ph), ct]).reshape(3, -1)
    w = (wg[:, None] * np.full(nphi, 2 * np.pi / nphi)[None, :]).ravel()
    return d, w


def test_sh_orthonormal():
    d, w = _sphere_quadrature()
    Y = sh.basis(d, 3)
    G = (Y * w[None]) @ Y.T
    assert np.allclose(G, np.eye(16), atol=1e-12)


def test_sh_matches_scipy_with_fixed_signs():
    """Real SH with the Condon-Shortley phase kept (R9), from scipy's complex
    harmonics Y_l^m (which carry that phase): sqrt(2) Im Y_l^|m| for m < 0,
    Y_l^0 for m = 0 and sqrt(2) Re Y_l^m for m > 0.  Every basis function has
    one fixed sign, so a sign slip in any of the sixteen polynomials fails
    (orthonormality cannot see signs)."""
    sp = pytest.importorskip("scipy.special")
    d, _ = _sphere_quadrature(12, 24)
    theta = np.arccos(np.clip(d[2], -1, 1))
    phi = np.arctan2(d[1], d[0])
    Y = sh.basis(d, 3)
    j = 0
    for l in range(4):
        for m in range(-l, l + 1):
            c = sp.sph_harm_y(l, abs(m), theta, phi)
            if m == 0:
                ref = c.real
            elif m > 0:
                ref = math.sqrt(2) * c.real
            else:
                ref = math.sqrt(2) * c.imag
            assert np.allclose(Y[j], ref, atol=1e-12), (l, m)
            j += 1


def test_sh_low_order_values_by_hand():
    """Degree 0 and 1 at the axis directions, from the closed forms: Y_0 =
    1/(2 sqrt(pi)); with the phase, (Y_1^-1, Y_1^0, Y_1^1) = sqrt(3/(4 pi)) (-y, z, -x)."""
    k1 = math.sqrt(3.0 / (4.0 * math.pi))
    dirs = np.eye(3)
    Y = sh.basis(dirs, 1)
    assert np.allclose(Y[0], 0.5 / math.sqrt(math.pi), rtol=1e-15)
    assert np.allclose(Y[1:4, 0], [0.0, 0.0, -k1], atol=1e-16)   # d = +x
    assert np.allclose(Y[1:4, 1], [-k1, 0.0, 0.0], atol=1e-16)   # d = +y
    assert np.allclose(Y[1:4, 2], [0.0, k1, 0.0], atol=1e-16)    # d = +z


def test_sh_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    d = rng.normal(size=(3, 50))
    d /= np.linalg.norm(d, axis=0)
    G = sh.basis_grad(d, 3)
    h = 1e-6
    for k in range(3):
        e = np.zeros((3, 1))
        e[k] = h
        fd = (sh.basis(d + e, 3) - sh.basis(d - e, 3)) / (2 * h)
        assert np.allclose(G[:, k], fd, atol=1e-8)


def test_sh_degree0_colour():
    p = make_params([[0.1, 0.2, 0.3]], sh=[[0.7], [-0.2], [-2.0]])
    pr = project.project(p, identity_camera(), 16)
    want = np.maximum(p["sh"][:, 0].astype(np.float64) / (2 * math.sqrt(math.pi)) + 0.5, 0)
    assert np.allclose(pr["rgb"][:, 0], want, rtol=1e-14)
    assert list(pr["clamped"][:, 0]) == [False, False, True]
