"""Pins of the oracle's initialisation: Philox4x32-10 known-answer vectors and
distribution checks of the derived uniforms and normals (moments, and
Kolmogorov-Smirnov tests against the uniform, normal, exponential and
Rayleigh-angle laws the Box-Muller transform is defined to produce)."""
import json
import os

import numpy as np
import pytest

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


def test_uniform_and_box_muller_distributions_ks():
    """Kolmogorov-Smirnov against the exact laws: u = (x >> 8) 2^-24 is uniform
    on [0, 1); a Box-Muller pair (z0, z1) is two independent standard normals,
    so z0^2 + z1^2 is exponential with mean 2 and atan2(z1, z0) is uniform on
    (-pi, pi].  A wrong constant (2 pi, the factor -2, a swapped sine and
    cosine with a sign, the 2^-24 scale) shifts one of these laws."""
    stats = pytest.importorskip("scipy.stats")
    n = 200_000
    idx = np.arange(n, dtype=np.uint64)
    z = np.zeros(n, np.uint64)
    u = init.philox4x32_10([idx, z + 3, z, z], (12345, 678))
    U = init.uniform24(u[0])
    assert stats.kstest(U, "uniform").pvalue > 1e-3
    a, b = init.box_muller(u[1], u[2])
    for x in (a, b):
        assert stats.kstest(x, "norm").pvalue > 1e-3
    r2 = a * a + b * b
    assert stats.kstest(r2, "expon", args=(0, 2.0)).pvalue > 1e-3
    ang = np.arctan2(b, a)
    assert stats.kstest(ang, "uniform", args=(-np.pi, 2 * np.pi)).pvalue > 1e-3
    # independence of the pair: correlation of the two normals and of their squares
    assert abs(np.corrcoef(a, b)[0, 1]) < 0.02
    assert abs(np.corrcoef(a * a, b * b)[0, 1]) < 0.02


def test_random_quaternions_uniform_on_the_sphere():
    """Normalised 4-D normals are uniform on S^3: each coordinate q_k satisfies
    q_k^2 ~ Beta(1/2, 3/2)."""
    stats = pytest.importorskip("scipy.stats")
    xyz = np.zeros((3, 50_000))
    p = init.init_from_points(xyz, 0, random_quats=True, seed=99)
    for k in range(4):
        assert stats.kstest(p["quats"][k] ** 2, "beta", args=(0.5, 1.5)).pvalue > 1e-3, k
