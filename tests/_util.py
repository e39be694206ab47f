"""Small helpers shared by the tests (no rasterizer arithmetic)."""
import numpy as np


def make_params(means, log_scales=None, quats=None, logits=None, sh=None, sh_degree=0):
    means = np.asarray(means, np.float64).reshape(-1, 3).T
    n = means.shape[1]
    if log_scales is None:
        log_scales = np.full((3, n), np.log(0.05))
    if quats is None:
        quats = np.zeros((4, n))
        quats[0] = 1
    if logits is None:
        logits = np.zeros(n)
    if sh is None:
        sh = np.zeros(((sh_degree + 1) ** 2 * 3, n))
    return {
        "means": np.asarray(means, np.float32),
        "log_scales": np.asarray(log_scales, np.float32).reshape(3, n),
        "quats": np.asarray(quats, np.float32).reshape(4, n),
        "opacity_logits": np.asarray(logits, np.float32).reshape(n),
        "sh": np.asarray(sh, np.float32).reshape(-1, n),
        "sh_degree": sh_degree,
    }


def identity_camera(W=256, H=256, f=200.0):
    return dict(R=np.eye(3), t=np.zeros(3), fx=f, fy=f, cx=W / 2, cy=H / 2,
                width=W, height=H, z_near=0.2)


def rel_l2(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def density_inputs(n, sh_degree, seed, *, extent=2.5, tau=2e-4, percent_dense=0.01,
                   min_opacity=0.005, max_world=0.1):
    """Seeded parameters, Adam moments and density statistics whose decisions
    (mean gradient vs tau, largest scale vs the clone and world limits, a
    child's largest scale vs the world limit, opacity vs min_opacity) all lie
    at least 6% away from their thresholds (children's scales are the
    parent's / 1.6), plus exact ties of the gradient
    test at its first entries (grad / count == float32(tau) exactly, for the
    threshold tau = float32(tau)).  Returns params, m, v (float32 dicts) and
    stats (grad float32, count int32, max_radius int32)."""
    rng = np.random.default_rng(seed)

    def bands(lo_hi, size):
        pick = rng.integers(0, len(lo_hi), size)
        lo = np.array([b[0] for b in lo_hi])[pick]
        hi = np.array([b[1] for b in lo_hi])[pick]
        return lo * np.exp(rng.uniform(0, 1, size) * np.log(hi / lo))

    clone_lim = percent_dense * extent
    world = max_world * extent
    count = rng.integers(0, 6, n).astype(np.int32)
    ratio = bands([(0.1, 0.9), (1.1, 4.0)], n)
    grad = np.where(count > 0, ratio * tau * count, rng.uniform(0, 1e-3, n)).astype(np.float32)
    # exact ties: g = float32(tau) with count 1 and 2
    t32 = np.float32(tau)
    k = min(n, 4)
    count[:k] = [1, 2, 1, 2][:k]
    grad[:k] = [t32, t32 * np.float32(2), t32, t32 * np.float32(2)][:k]
    smax = bands([(0.3 * clone_lim, 0.9 * clone_lim), (1.1 * clone_lim, 0.9 * world),
                  (1.1 * world, 1.5 * world), (1.7 * world, 3.0 * world)], n)
    ls = np.log(smax)[None, :] - rng.uniform(0.0, 1.5, (3, n)) * (rng.random((3, n)) < 0.67)
    for i in range(n):                  # the largest axis keeps smax exactly
        ls[rng.integers(0, 3), i] = np.log(smax[i])
    op = np.minimum(bands([(0.2 * min_opacity, 0.9 * min_opacity),
                           (1.1 * min_opacity, 150 * min_opacity)], n), 0.98)
    logits = np.log(op / (1 - op))
    params = make_params(rng.uniform(-1, 1, (n, 3)), log_scales=ls,
                         quats=rng.normal(size=(4, n)), logits=logits,
                         sh=rng.normal(0, 0.3, ((sh_degree + 1) ** 2 * 3, n)),
                         sh_degree=sh_degree)
    moments = []
    for _ in range(2):
        moments.append({key: rng.normal(size=np.shape(val)).astype(np.float32)
                        for key, val in params.items() if key != "sh_degree"})
        moments[-1]["sh_degree"] = sh_degree
    stats = dict(grad=grad, count=count,
                 max_radius=rng.integers(0, 41, n).astype(np.int32))
    return params, moments[0], moments[1], stats
