"""Pins of the oracle's binning and compositing: a global key sort, brute force
without tiles, and the closed-form transmittance of stacked Gaussians."""
import json
import os

import numpy as np

from oracle import binning, blend, camera, pipeline, project
from tests._util import identity_camera, make_params

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def _cams(n=8, W=256, H=256):
    return [camera.to_float32(c) for c in camera.orbit_cameras(n, 2.5, 60.0, W, H)]


def test_tile_lists_equal_global_key_sort(tiny_scene):
    cam = _cams()[3]
    for tile in (8, 16, 32):
        pr = project.project(tiny_scene.params, cam, tile)
        tx, ty = (256 + tile - 1) // tile, (256 + tile - 1) // tile
        keys, gids, ranges = binning.tile_lists(pr, tx, ty, tile_offset=5)
        ek, eg = binning.emitted_records(pr, tx, tile_offset=5)
        order = np.lexsort((eg, ek))                  # by key, then index
        assert np.array_equal(keys, ek[order])
        assert np.array_equal(gids, eg[order])
        tiles = (keys >> np.uint64(32)).astype(np.int64) - 5
        for t in range(tx * ty):
            lo = np.searchsorted(tiles, t, "left")
            hi = np.searchsorted(tiles, t, "right")
            want = (lo, hi) if hi > lo else (0, 0)
            assert tuple(ranges[t]) == want
        assert keys.size == pr["tiles"].sum()


def test_tile_lists_python_sorted_brute_force():
    rng = np.random.default_rng(5)
    n = 60
    p = make_params(rng.uniform(-0.3, 0.3, (n, 3)), log_scales=rng.uniform(-4, -2.5, (3, n)))
    # duplicate depths to exercise the index tie-break
    p["means"][:, 10:20] = p["means"][:, 0:1]
    cam = _cams(2, 64, 48)[0]
    pr = project.project(p, cam, 8)
    keys, gids, ranges = binning.tile_lists(pr, 8, 6)
    recs = []
    for g in range(n):
        if not pr["touched"][g]:
            continue
        d = float(np.float32(pr["tz"][g]))
        for y in range(pr["rect"][1, g], pr["rect"][3, g] + 1):
            for x in range(pr["rect"][0, g], pr["rect"][2, g] + 1):
                recs.append((y * 8 + x, d, g))
    recs.sort()
    assert [r[2] for r in recs] == list(gids)
    assert [r[0] for r in recs] == list((keys >> np.uint64(32)).astype(int))


def test_stacked_transmittance_closed_form():
    g = GOLD["stacked_tiny"]
    cam = identity_camera(32, 32, 100.0)
    for N in (5, 12, 13, 30):
        # identical Gaussians centred on pixel (16, 16); same depth -> index order
        mu = np.array([16.5 - 16, 16.5 - 16, 100.0]) / 100.0 * 3.0
        mu[2] = 3.0
        p = make_params([mu] * N, logits=[0.1] * N, sh=np.repeat([[1.0], [0.5], [-0.5]], N, 1))
        pr = project.project(p, cam, 16)
        assert np.allclose(pr["m"][:, 0], [16.5, 16.5])
        lists = binning.tile_lists(pr, 2, 2)
        img, T, nc, _ = blend.render_view(pr, lists, bg=(0.1, 0.2, 0.3))
        a = pr["opacity"][0]
        assert abs(a - g["alpha"]) < 1e-8
        n_exp = min(N, g["n_contrib"])
        T_exp = (1 - a) ** n_exp
        assert nc[16, 16] == n_exp
        assert abs(T[16, 16] - T_exp) < 1e-15
        if N >= 13:
            assert abs(T[16, 16] - g["T_final"]) < 1e-9
        rgb = pr["rgb"][:, 0]
        want = rgb * (1 - T_exp) + np.array([0.1, 0.2, 0.3]) * T_exp
        assert np.allclose(img[:, 16, 16], want, atol=1e-14)
        out, Tl, last = blend.pixel_loop(pr, 16, 16, bg=(0.1, 0.2, 0.3), tile=16)
        assert np.allclose(out, want, atol=1e-14) and last == n_exp - 1


def test_tiled_equals_brute_force_per_pixel(tiny_scene):
    cam = _cams()[1]
    fw = pipeline.forward_view(tiny_scene.params, cam, 16, bg=(0.05, 0.1, 0.2))
    pr = fw["proj"]
    rng = np.random.default_rng(7)
    bits = pr["depth32"].view(np.uint32)
    ids = np.nonzero(pr["touched"])[0]
    order = ids[np.argsort(bits[ids], kind="stable")]
    ys, xs = np.nonzero(fw["image"].sum(0) > 0.06)
    pick = rng.choice(xs.size, 150, replace=False)
    for x, y in zip(xs[pick], ys[pick]):
        out, T, last = blend.pixel_loop(pr, x, y, bg=(0.05, 0.1, 0.2), tile=16, order=order)
        assert np.allclose(out, fw["image"][:, y, x], atol=1e-13)
        assert abs(T - fw["T"][y, x]) < 1e-13


def test_low_opacity_needs_no_tile_predicate():
    # o <= e^{4.5}/255: outside 3 sigma alpha < 1/255, so tiles change nothing
    rng = np.random.default_rng(8)
    n = 300
    p = make_params(rng.uniform(-0.5, 0.5, (n, 3)), log_scales=rng.uniform(-4, -2.5, (3, n)),
                    quats=rng.normal(size=(4, n)), logits=np.full(n, -0.7),
                    sh=rng.normal(0, 0.3, (3, n)))
    cam = _cams(3, 96, 80)[2]
    fw = pipeline.forward_view(p, cam, 16)
    pr = fw["proj"]
    assert pr["opacity"].max() <= np.exp(4.5) / 255
    for y in range(0, 80, 7):
        for x in range(0, 96, 5):
            out, T, _ = blend.pixel_loop(pr, x, y)
            assert np.allclose(out, fw["image"][:, y, x], atol=1e-13)


def test_empty_tiles_and_empty_scene():
    cam = identity_camera(40, 24, 50.0)
    p = make_params([[0, 0, -5.0]])                  # behind the camera
    fw = pipeline.forward_view(p, cam, 16, bg=(0.3, 0.2, 0.1))
    assert fw["lists"][0].size == 0
    assert np.all(fw["lists"][2] == 0)
    assert np.allclose(fw["image"], np.array([0.3, 0.2, 0.1])[:, None, None])
    assert np.all(fw["T"] == 1) and np.all(fw["n"] == 0)
