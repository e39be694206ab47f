"""Pins of the oracle's adaptive density control (CPU): hand-worked cases of
clone / split / prune and the output order, the split children's distribution
against the closed-form covariance R S^2 R^T, the statistics' NDC scaling,
and the opacity reset."""
import numpy as np

from oracle import density as D
from oracle.init import philox4x32_10, box_muller
from tests._util import make_params

EXT = 2.5


def _moments(p):
    z = {k: (np.zeros_like(np.asarray(v, np.float64)) if isinstance(v, np.ndarray) else v)
         for k, v in p.items()}
    return z, {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in z.items()}


def _f64(p):
    return {k: (np.asarray(v, np.float64) if isinstance(v, np.ndarray) else v)
            for k, v in p.items()}


def _case():
    """Seven Gaussians with hand-chosen statistics (threshold 0.0002, clone/split
    boundary 0.01 * 2.5 = 0.025, world limit 0.25, screen limit 20 px)."""
    ls = np.log(np.array([
        [0.010, 0.012, 0.011],   # 0: grad 0.0003, small  -> clone
        [0.050, 0.030, 0.020],   # 1: grad 0.0004, large  -> split
        [0.010, 0.010, 0.010],   # 2: grad 0.0001         -> kept
        [0.010, 0.010, 0.010],   # 3: opacity 0.001       -> pruned
        [0.020, 0.020, 0.020],   # 4: never seen          -> kept
        [0.010, 0.010, 0.010],   # 5: radius 25 px        -> pruned when the size test is on
        [0.300, 0.010, 0.010],   # 6: scale 0.3 > 0.25    -> split; pruned (and its children
    ])).T                        #    kept) when the size test is on
    logits = np.array([0.5, 1.0, -1.0, np.log(0.001 / 0.999), 2.0, 0.0, 0.3])
    rng = np.random.default_rng(3)
    p = _f64(make_params(rng.uniform(-1, 1, (7, 3)), log_scales=ls,
                         quats=rng.normal(size=(4, 7)), logits=logits,
                         sh=rng.normal(size=(3, 7)), sh_degree=0))
    p["log_scales"] = ls
    p["opacity_logits"] = logits
    stats = dict(grad=np.array([0.0006, 0.0012, 0.0002, 0.01, 0.0, 0.0, 0.001]),
                 count=np.array([2, 3, 2, 1, 0, 1, 2]),
                 max_radius=np.array([3, 5, 2, 4, 0, 25, 9]))
    return p, stats


def test_clone_split_prune_by_hand():
    p, stats = _case()
    m, v = _moments(p)
    m["means"][:] = 1.0      # nonzero moments: copied for originals, zero for new ones
    v["sh"][:] = 2.0
    out, om, ov, info = D.densify(p, m, v, stats, EXT, seed=7)
    # originals kept: 0, 2, 4, 5 (0 is also cloned; 1 and 6 split; 3 pruned)
    # then the clone of 0, then children of 1 (two) and of 6 (two)
    assert (info["kept"], info["cloned"], info["split"], info["children"]) == (4, 1, 2, 4)
    assert out["means"].shape == (3, 9)
    order = [0, 2, 4, 5, 0]
    assert np.array_equal(out["means"][:, :5], p["means"][:, order])
    assert np.array_equal(out["sh"][:, :5], p["sh"][:, order])
    assert np.array_equal(om["means"][:, :4], m["means"][:, [0, 2, 4, 5]])
    assert np.all(om["means"][:, 4:] == 0) and np.all(ov["sh"][:, 4:] == 0)
    assert np.all(ov["sh"][:, :4] == 2.0)
    # children: log-scales less ln 1.6, parent's rotation, opacity, colour
    for k, src in enumerate([1, 1, 6, 6]):
        j = 5 + k
        assert np.allclose(out["log_scales"][:, j], p["log_scales"][:, src] - np.log(1.6))
        assert np.array_equal(out["quats"][:, j], p["quats"][:, src])
        assert out["opacity_logits"][j] == p["opacity_logits"][src]
        assert np.array_equal(out["sh"][:, j], p["sh"][:, src])
    # the two children of a source differ, and lie within a few sigma of it
    assert not np.allclose(out["means"][:, 5], out["means"][:, 6])
    d = out["means"][:, 5] - p["means"][:, 1]
    assert np.linalg.norm(d) < 5 * 0.05


def test_size_prune_after_reset():
    p, stats = _case()
    m, v = _moments(p)
    out, _, _, info = D.densify(p, m, v, stats, EXT, max_screen=20.0, seed=7)
    # 5 (radius 25) goes; 6 was split (its children, scale 0.3 / 1.6 = 0.1875 <= 0.25,
    # stay); 3 pruned as before
    assert (info["kept"], info["cloned"], info["children"]) == (3, 1, 4)
    assert np.array_equal(out["means"][:, :4], p["means"][:, [0, 2, 4, 0]])
    # a larger split source whose children exceed the world limit loses them
    p2 = dict(p)
    p2["log_scales"] = p["log_scales"].copy()
    p2["log_scales"][0, 6] = np.log(0.5)       # child scale 0.3125 > 0.25
    out2, _, _, info2 = D.densify(p2, m, v, stats, EXT, max_screen=20.0, seed=7)
    assert info2["children"] == 2 and out2["means"].shape[1] == 6


def test_threshold_ties_and_unseen():
    p, stats = _case()
    m, v = _moments(p)
    # mean gradient exactly at the threshold is selected (>=), count 0 never is
    stats = dict(stats, grad=np.array([0.0004, 0.0, 0.0, 0.0, 5.0, 0.0, 0.0]),
                 count=np.array([2, 1, 1, 1, 0, 1, 1]))
    _, _, _, info = D.densify(p, m, v, stats, EXT)
    assert info["clone_mask"][0] and not info["clone_mask"][4] and not info["split_mask"][4]


def test_split_children_follow_the_gaussian_covariance():
    """Children of one anisotropic, rotated Gaussian over many seeds: their
    sample covariance approaches R diag(s^2) R^T (closed form), their mean mu."""
    q = np.array([0.8, 0.3, -0.4, 0.2])
    s = np.array([0.3, 0.1, 0.05])
    n = 4000
    p = _f64(make_params(np.tile([0.2, -0.1, 0.4], (n, 1)),
                         log_scales=np.tile(np.log(s)[:, None], (1, n)),
                         quats=np.tile(q[:, None], (1, n)), logits=np.full(n, 1.0)))
    m, v = _moments(p)
    stats = dict(grad=np.full(n, 1.0), count=np.ones(n, int), max_radius=np.zeros(n, int))
    out, _, _, info = D.densify(p, m, v, stats, EXT, seed=11)
    # the stored (float32-rounded) parameters define the closed form
    qn = p["quats"][:, 0] / np.linalg.norm(p["quats"][:, 0])
    w, x, y, z = qn
    R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                  [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                  [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
    s = np.exp(p["log_scales"][:, 0])
    mu = p["means"][:, 0]
    assert info["children"] == 2 * n and out["means"].shape[1] == 2 * n
    d = out["means"] - mu[:, None]
    cov = d @ d.T / d.shape[1]
    want = R @ np.diag(s * s) @ R.T
    assert np.abs(d.mean(1)).max() < 4 * 0.3 / np.sqrt(2 * n)
    assert np.abs(cov - want).max() < 0.06 * s[0] ** 2
    # the local coordinates R^T d / s are the generator's normals, child by child
    zloc = (R.T @ d) / s[:, None]
    for c in range(2):
        idx = np.arange(n, dtype=np.uint64)
        zero = np.zeros(n, np.uint64)
        dd = philox4x32_10([idx, zero + 16 + c, zero, zero], (11, 0))
        a0, a1 = box_muller(dd[0], dd[1])
        a2, _ = box_muller(dd[2], dd[3])
        assert np.allclose(zloc[:, c::2], np.stack([a0, a1, a2]), atol=1e-9)


def test_accumulate_ndc_scaling():
    n = 3
    stats = dict(grad=np.zeros(n), count=np.zeros(n, int), max_radius=np.zeros(n, int))
    g = np.zeros((2, 2, n))
    g[0, :, 0] = (3e-6, 4e-6)         # view 0: 200 x 100 px
    g[1, :, 0] = (1e-6, 0.0)          # view 1: 50 x 80 px
    g[0, :, 1] = (1e-6, 1e-6)
    touched = np.array([[1, 1, 0], [1, 0, 0]], bool)
    radius = np.array([[4, 7, 0], [9, 3, 0]])
    D.accumulate(stats, g, touched, radius, [200, 50], [100, 80], scale=2.0)
    want0 = 2.0 * (np.hypot(3e-6 * 100, 4e-6 * 50) + np.hypot(1e-6 * 25, 0.0))
    want1 = 2.0 * np.hypot(1e-6 * 100, 1e-6 * 50)
    assert np.allclose(stats["grad"], [want0, want1, 0.0], rtol=1e-14)
    assert list(stats["count"]) == [2, 1, 0]
    assert list(stats["max_radius"]) == [9, 7, 0]   # untouched view 1 of Gaussian 1 ignored


def test_opacity_reset_closed_form():
    p = {"opacity_logits": np.array([-6.0, -4.0, 0.0, 5.0])}
    m = {"opacity_logits": np.ones(4)}
    v = {"opacity_logits": np.ones(4)}
    out, om, ov = D.opacity_reset(p, m, v, 0.01)
    op = 1 / (1 + np.exp(-out["opacity_logits"]))
    assert np.allclose(op, [1 / (1 + np.exp(6.0)), 0.01, 0.01, 0.01], rtol=1e-12)
    assert np.all(om["opacity_logits"] == 0) and np.all(ov["opacity_logits"] == 0)
