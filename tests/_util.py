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
