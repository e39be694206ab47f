"""Pins of the oracle's isosurface extraction and ray-caster (CPU): a linear
field (exact for the vertex rule and for the trilinear interpolant) with its
closed-form crossings, hit points and shading; brute-force extraction by
Python loops in the canonical order; the Philox keep rule's rate and
determinism; a sphere's silhouette."""
import numpy as np

from oracle import iso as I
from oracle.init import philox4x32_10


def _grid(n, lo=-1.0, hi=1.0):
    return lo + np.arange(n) * ((hi - lo) / (n - 1))


def test_plane_crossings_closed_form():
    nx, ny, nz = 9, 5, 4
    x = _grid(nx)
    vol = np.broadcast_to(x[None, None, :], (nz, ny, nx)).astype(np.float32)
    c = 0.3
    p, ids = I.crossings(vol, (-1, -1, -1), (1, 1, 1), c)
    assert p.shape[1] == ny * nz                  # one x-edge per grid row
    assert np.abs(p[0] - np.float32(c)).max() < 1e-7 * 4
    assert np.all(ids % 3 == 0)
    assert np.all(np.diff(ids) > 0)


def test_brute_force_canonical_order():
    rng = np.random.default_rng(0)
    nz, ny, nx = 4, 5, 6
    vol = rng.random((nz, ny, nx)).astype(np.float32)
    lo, hi, iso = (-1.0, -0.5, 0.0), (1.0, 0.5, 2.0), 0.5
    h = [(hi[a] - lo[a]) / ((nx, ny, nz)[a] - 1) for a in range(3)]
    want = []
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                a = float(vol[k, j, i]) - iso
                for axis, (di, dj, dk) in enumerate(((1, 0, 0), (0, 1, 0), (0, 0, 1))):
                    if i + di >= nx or j + dj >= ny or k + dk >= nz:
                        continue
                    b = float(vol[k + dk, j + dj, i + di]) - iso
                    if (a < 0 < b) or (b < 0 < a):
                        t = a / (a - b)
                        q = [lo[0] + i * h[0], lo[1] + j * h[1], lo[2] + k * h[2]]
                        q[axis] += t * h[axis]
                        want.append(q)
    p, _ = I.crossings(vol, lo, hi, iso)
    assert p.shape[1] == len(want)
    assert np.abs(p.T - np.array(want)).max() < 1e-15


def test_keep_rule():
    ids = np.arange(200000, dtype=np.int64) * 3 + 1
    k = I.keep_mask(ids, 0.25, 77)
    rate = k.mean()
    assert abs(rate - 0.25) < 5 * np.sqrt(0.25 * 0.75 / ids.size)
    assert np.array_equal(k, I.keep_mask(ids, 0.25, 77))
    assert not np.array_equal(k, I.keep_mask(ids, 0.25, 78))
    assert I.keep_mask(ids, 1.0, 5).all() and not I.keep_mask(ids, 0.0, 5).any()
    # the uniform is the generator's first word, (x >> 8) 2^-24
    e = np.uint64(3 * 12345 + 2)
    d = philox4x32_10([np.array([e]), np.array([0], np.uint64), np.array([3], np.uint64),
                       np.array([0], np.uint64)], (77, 0))
    u = (int(d[0][0]) >> 8) * 2.0 ** -24
    assert I.keep_mask(np.array([e], np.int64), np.float32(u + 1e-7), 77)[0]
    assert not I.keep_mask(np.array([e], np.int64), np.float32(u), 77)[0]


def _look_along_x(C, W=24, H=20, f=30.0):
    R = np.array([[0.0, 1.0, 0.0], [0.0, 0.0, 1.0], [1.0, 0.0, 0.0]])
    return dict(R=R, t=-R @ np.asarray(C, np.float64), fx=f, fy=f, cx=W / 2, cy=H / 2,
                width=W, height=H, z_near=0.2)


def test_raycast_plane_closed_form():
    n = 17
    x = _grid(n)
    vol = np.broadcast_to(x[None, None, :], (n, n, n)).astype(np.float32)
    c, step = 0.25, 0.01
    cam = _look_along_x((-3.0, 0.1, -0.2))
    img = I.raycast(vol, (-1, -1, -1), (1, 1, 1), c, cam, step)
    W, H = cam["width"], cam["height"]
    o = np.array([-3.0, 0.1, -0.2])
    for y in range(H):
        for xx in range(W):
            dc = np.array([(xx + 0.5 - W / 2) / 30.0, (y + 0.5 - H / 2) / 30.0, 1.0])
            d = cam["R"].T @ dc
            d /= np.linalg.norm(d)
            t = (c - o[0]) / d[0]
            p = o + t * d
            inside = np.all(np.abs(p) <= 1.0)
            got = img[:, y, xx]
            if not inside:
                # rays that leave the box before reaching the plane miss
                if np.all(np.abs(o + (-1 - o[0]) / d[0] * d)[1:] > 1.0):
                    assert np.all(got == 0)
                continue
            lam = abs(d[0])
            want = np.array([0.85, 0.45 + 0.25 * p[2], 0.30 + 0.25 * (p[0] + 1)]) * (0.2 + 0.8 * lam)
            assert np.abs(got - want).max() < 1e-5, (xx, y, got, want)


def test_raycast_sphere_silhouette():
    n = 33
    g = _grid(n)
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    vol = (1.0 - (X * X + Y * Y + Z * Z) / 0.49).astype(np.float32)   # iso 0: radius 0.7
    cam = _look_along_x((-3.0, 0.0, 0.0), W=20, H=20, f=20.0)
    img = I.raycast(vol, (-1, -1, -1), (1, 1, 1), 0.0, cam, 0.01)
    o = np.array([-3.0, 0.0, 0.0])
    for y in range(20):
        for xx in range(20):
            dc = np.array([(xx + 0.5 - 10) / 20.0, (y + 0.5 - 10) / 20.0, 1.0])
            d = cam["R"].T @ dc
            d /= np.linalg.norm(d)
            dist = np.linalg.norm(np.cross(d, -o))          # ray's distance from the centre
            if dist < 0.7 - 0.03:
                assert img[:, y, xx].max() > 0
            elif dist > 0.7 + 0.03:
                assert img[:, y, xx].max() == 0
