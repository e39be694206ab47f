"""Pins of the oracle's initialisation: Philox4x32-10 known-answer vectors and
distribution checks of the derived uniforms and normals."""
import json
import os

import numpy as np

from oracle import init

KAT = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "philox_kat.json")))


def test_philox_known_answers():
    for v in KAT["vectors"]:
        ctr = [np.array([int(x, 16)], np.uint64) for x in v["ctr"]]
        key = tuple(int(x, 16) for x in v["key"])
        out = init.philox4x32_10(ctr, key)
        assert ["%08x" % int(o[0]) for o in out] == v["out"]


def test_uniform_and_normal_moments():
    n = 200_000
    idx = np.arange(n, dtype=np.uint64)
    z = np.zeros(n, np.uint64)
    u = init.philox4x32_10([idx, z, z, z], (12345, 678))
    U = init.uniform24(u[0])
    assert U.min() >= 0 and U.max() < 1
    assert abs(U.mean() - 0.5) < 3e-3 and abs(U.var() - 1 / 12) < 2e-3
    a, b = init.box_muller(u[1], u[2])
    for x in (a, b):
        assert abs(x.mean()) < 1e-2 and abs(x.var() - 1) < 1.5e-2
        assert abs((x ** 4).mean() - 3) < 0.1
    assert abs((a * b).mean()) < 1e-2


def test_init_rules():
    rng = np.random.default_rng(0)
    xyz = rng.uniform(-1, 1, (3, 1000))
    p = init.init_from_points(xyz, 3, log_scale=-4.0, log_scale_jitter=0.5, random_quats=True,
                              opacity_logit=0.1, sh_std=0.1, seed=77)
    assert np.array_equal(p["means"], xyz)
    assert p["log_scales"].min() >= -4.5 and p["log_scales"].max() <= -3.5
    assert np.allclose((p["quats"] ** 2).sum(0), 1.0)
    assert np.all(p["opacity_logits"] == 0.1)
    assert p["sh"].shape == (48, 1000) and abs(p["sh"].std() - 0.1) < 5e-3
    q = init.init_from_points(xyz, 0, log_scale_range=(-5, -3), seed=77)
    assert q["log_scales"].min() >= -5 and q["log_scales"].max() < -3
    assert np.all(q["quats"][0] == 1) and np.all(q["sh"] == 0)
