"""Pins of the oracle's hand-derived backward: central finite differences of
the oracle forward, and torch.autograd on an independent float64 torch
transcription of the same forward (fixed per-pixel contributor sets)."""
import math

import numpy as np
import pytest

from oracle import binning, blend, camera, pipeline, project
from tests._util import make_params, rel_l2

GROUPS = ("means", "log_scales", "quats", "opacity_logits", "sh")


def _scene(n=120, W=64, H=56, deg=3, seed=11, logit_hi=1.5, logit_lo=-2.0):
    rng = np.random.default_rng(seed)
    p = make_params(rng.uniform(-0.35, 0.35, (n, 3)), log_scales=rng.uniform(-3.6, -2.6, (3, n)),
                    quats=rng.normal(size=(4, n)), logits=rng.uniform(logit_lo, logit_hi, n),
                    sh=rng.normal(0, 0.25, ((deg + 1) ** 2 * 3, n)), sh_degree=deg)
    p64 = {k: (v.astype(np.float64) if isinstance(v, np.ndarray) else v) for k, v in p.items()}
    cam = camera.to_float32(camera.orbit_cameras(5, 2.5, 60.0, W, H)[2])
    w = rng.normal(size=(3, H, W))
    return p64, cam, w


def _loss(p, cam, w, tile=16):
    fw = pipeline.forward_view(p, cam, tile)
    return float((fw["image"] * w).sum())


def test_param_grads_match_central_differences():
    p, cam, w = _scene()
    fw = pipeline.forward_view(p, cam, 16)
    _, g = pipeline.backward_view(p, cam, fw, w)
    rng = np.random.default_rng(0)
    checked = 0
    for k in GROUPS:
        rows = p[k].shape[0] if p[k].ndim == 2 else 1
        for _ in range(24):
            i = int(rng.integers(0, p[k].shape[-1]))
            r = int(rng.integers(0, rows))
            x0 = p[k][r, i] if p[k].ndim == 2 else p[k][i]
            vals = []
            for h in (1e-6 * max(1, abs(x0)), 2e-6 * max(1, abs(x0))):
                out = []
                for sgn in (1, -1):
                    q = {kk: (vv.copy() if isinstance(vv, np.ndarray) else vv) for kk, vv in p.items()}
                    if q[k].ndim == 2:
                        q[k][r, i] += sgn * h
                    else:
                        q[k][i] += sgn * h
                    out.append(_loss(q, cam, w))
                vals.append((out[0] - out[1]) / (2 * h))
            if abs(vals[0] - vals[1]) > 1e-2 * max(abs(vals[0]), 1e-8):
                continue                                 # a threshold was crossed
            an = g[k][r, i] if g[k].ndim == 2 else g[k][i]
            assert abs(an - vals[0]) <= 1e-5 * max(abs(vals[0]), 1e-3), (k, r, i, an, vals[0])
            checked += 1
    assert checked >= 100


def test_directional_derivatives():
    p, cam, w = _scene(seed=12)
    fw = pipeline.forward_view(p, cam, 16)
    _, g = pipeline.backward_view(p, cam, fw, w)
    rng = np.random.default_rng(1)
    good = 0
    for _ in range(8):
        v = {k: rng.normal(size=p[k].shape) for k in GROUPS}
        an = sum((g[k] * v[k]).sum() for k in GROUPS)
        fds = []
        for h in (1e-7, 2e-7):
            q1 = dict(p, **{k: p[k] + h * v[k] for k in GROUPS})
            q2 = dict(p, **{k: p[k] - h * v[k] for k in GROUPS})
            fds.append((_loss(q1, cam, w) - _loss(q2, cam, w)) / (2 * h))
        if abs(fds[0] - fds[1]) > 1e-2 * abs(fds[0]):
            continue
        assert abs(an - fds[0]) <= 1e-4 * abs(fds[0]), (an, fds)
        good += 1
    assert good >= 6


def test_screen_space_grads_match_central_differences():
    p, cam, w = _scene(seed=13)
    fw = pipeline.forward_view(p, cam, 16)
    acc, _ = pipeline.backward_view(p, cam, fw, w)
    pr = fw["proj"]

    def L(pr2):
        img, *_ = blend.render_view(pr2, fw["lists"])
        return float((img * w).sum())

    rng = np.random.default_rng(2)
    ids = np.nonzero(pr["touched"])[0]
    for key, rows in (("m", 2), ("conic", 3), ("opacity", 1), ("rgb", 3)):
        for _ in range(10):
            i = int(rng.choice(ids))
            r = int(rng.integers(0, rows))
            fds = []
            for h in (1e-5, 2e-5):
                vals = []
                for sgn in (1, -1):
                    q = dict(pr)
                    q[key] = pr[key].copy()
                    if q[key].ndim == 2:
                        q[key][r, i] += sgn * h
                    else:
                        q[key][i] += sgn * h
                    vals.append(L(q))
                fds.append((vals[0] - vals[1]) / (2 * h))
            fd = fds[0]
            if abs(fds[0] - fds[1]) > 1e-2 * max(abs(fd), 1e-8):
                continue                                 # a threshold was crossed
            an = acc[key][r, i] if acc[key].ndim == 2 else acc[key][i]
            assert abs(an - fd) <= 1e-5 * max(abs(fd), 1e-4), (key, r, i, an, fd)


# ----------------------------------------------------- torch transcription
def _torch_forward(torch, P, cam, fw, tile, bg):
    """Independent float64 transcription of projection + compositing with the
    contributor sets of ``fw`` held fixed."""
    pr = fw["proj"]
    R = torch.tensor(cam["R"], dtype=torch.float64)
    tcam = torch.tensor(cam["t"], dtype=torch.float64)
    fx, fy, cx, cy = cam["fx"], cam["fy"], cam["cx"], cam["cy"]
    W, H = cam["width"], cam["height"]
    mu = P["means"]
    t = R @ mu + tcam[:, None]
    tz = t[2]
    s = torch.exp(P["log_scales"])
    q = P["quats"] / torch.linalg.norm(P["quats"], dim=0, keepdim=True)
    w_, x_, y_, z_ = q
    Rq = torch.stack([
        torch.stack([1 - 2 * (y_ ** 2 + z_ ** 2), 2 * (x_ * y_ - w_ * z_), 2 * (x_ * z_ + w_ * y_)]),
        torch.stack([2 * (x_ * y_ + w_ * z_), 1 - 2 * (x_ ** 2 + z_ ** 2), 2 * (y_ * z_ - w_ * x_)]),
        torch.stack([2 * (x_ * z_ - w_ * y_), 2 * (y_ * z_ + w_ * x_), 1 - 2 * (x_ ** 2 + y_ ** 2)]),
    ])                                                  # (3, 3, N)
    M = Rq * s[None]
    Sig = torch.einsum("ikn,jkn->ijn", M, M)
    limx, limy = 1.3 * 0.5 * W / fx, 1.3 * 0.5 * H / fy
    u = torch.clamp(t[0] / tz, -limx, limx)
    v = torch.clamp(t[1] / tz, -limy, limy)
    zero = torch.zeros_like(tz)
    J = torch.stack([torch.stack([fx / tz, zero, -fx * u / tz]),
                     torch.stack([zero, fy / tz, -fy * v / tz])])
    T = torch.einsum("ikn,kj->ijn", J, R)
    cov = torch.einsum("ikn,kln,jln->ijn", T, Sig, T)
    a, b, c = cov[0, 0] + 0.3, cov[0, 1], cov[1, 1] + 0.3
    D = a * c - b * b
    con = torch.stack([c / D, -b / D, a / D])
    m = torch.stack([fx * t[0] / tz + cx, fy * t[1] / tz + cy])
    o = torch.sigmoid(P["opacity_logits"])
    cpos = -R.T @ tcam
    d = mu - cpos[:, None]
    d = d / torch.linalg.norm(d, dim=0, keepdim=True)
    from oracle import sh as _sh_np
    dx_, dy_, dz_ = d
    ks = [_sh_np.K0, _sh_np.K1, _sh_np.K2, _sh_np.K3, _sh_np.A3, _sh_np.B3, _sh_np.C3, _sh_np.E3]
    K0, K1, K2, K3, A3, B3, C3, E3 = ks
    Y = [K0 + 0 * dx_, -K1 * dy_, K1 * dz_, -K1 * dx_,
         K2 * dx_ * dy_, -K2 * dy_ * dz_, K3 * (2 * dz_ ** 2 - dx_ ** 2 - dy_ ** 2), -K2 * dx_ * dz_,
         0.5 * K2 * (dx_ ** 2 - dy_ ** 2),
         -A3 * dy_ * (3 * dx_ ** 2 - dy_ ** 2), B3 * dx_ * dy_ * dz_,
         -C3 * dy_ * (4 * dz_ ** 2 - dx_ ** 2 - dy_ ** 2), E3 * dz_ * (2 * dz_ ** 2 - 3 * dx_ ** 2 - 3 * dy_ ** 2),
         -C3 * dx_ * (4 * dz_ ** 2 - dx_ ** 2 - dy_ ** 2), 0.5 * B3 * dz_ * (dx_ ** 2 - dy_ ** 2),
         -A3 * dx_ * (dx_ ** 2 - 3 * dy_ ** 2)]
    nb = P["sh"].shape[0] // 3
    Y = torch.stack(Y[:nb])
    rgb = torch.stack([(P["sh"][ch::3] * Y).sum(0) + 0.5 for ch in range(3)])
    rgb = torch.clamp(rgb, min=0.0)

    keys, gids, ranges = fw["lists"]
    tiles_x = (W + tile - 1) // tile
    img = torch.zeros(3, H, W, dtype=torch.float64)
    bgt = torch.tensor(bg, dtype=torch.float64)
    for tt in range(ranges.shape[0]):
        g = gids[ranges[tt, 0]:ranges[tt, 1]]
        X, Yp = blend.tile_pixels(tt % tiles_x, tt // tiles_x, tile, W, H)
        if g.size == 0:
            img[:, Yp, X] = bgt[:, None].expand(3, X.size)
            continue
        ref = blend.composite_tile(pr, g, X + 0.5, Yp + 0.5, bg)
        mask = torch.tensor(ref["contrib"])
        gi = torch.tensor(g)
        ddx = torch.tensor(X + 0.5)[:, None] - m[0][gi][None]
        ddy = torch.tensor(Yp + 0.5)[:, None] - m[1][gi][None]
        cg = con[:, gi]
        power = -0.5 * (cg[0] * ddx ** 2 + cg[2] * ddy ** 2) - cg[1] * ddx * ddy
        alpha = torch.clamp(o[gi][None] * torch.exp(power), max=0.99)
        ae = torch.where(mask, alpha, torch.zeros_like(alpha))
        one = torch.ones(ae.shape[0], 1, dtype=torch.float64)
        Tex = torch.cumprod(torch.cat([one, 1 - ae[:, :-1]], 1), 1)
        Tfin = torch.prod(1 - ae, 1)
        out = (ae * Tex) @ rgb[:, gi].T + Tfin[:, None] * bgt[None]
        img[:, Yp, X] = out.T
    return img


def test_param_grads_match_torch_autograd():
    torch = pytest.importorskip("torch")
    for seed, deg, tile in ((21, 3, 16), (22, 1, 8), (23, 0, 32)):
        p, cam, w = _scene(n=90, seed=seed, deg=deg)
        bg = (0.1, 0.3, 0.2)
        fw = pipeline.forward_view(p, cam, tile, bg)
        _, g = pipeline.backward_view(p, cam, fw, w, bg)
        P = {k: torch.tensor(p[k], dtype=torch.float64, requires_grad=True) for k in GROUPS}
        img = _torch_forward(torch, P, cam, fw, tile, bg)
        assert np.allclose(img.detach().numpy(), fw["image"], atol=1e-12)
        (img * torch.tensor(w)).sum().backward()
        for k in GROUPS:
            assert rel_l2(g[k], P[k].grad.numpy()) < 1e-9, (seed, k)


def clamp_scene(seed, deg, n=20, W=96, H=80):
    """Few large splats spread over the image with logits U(3, 7) (opacity
    0.953 .. 0.999).  alpha = o G passes 0.99 only within about 0.14 sigma of a
    centre, so the splats are large (sigma 10 .. 25 px) and few enough for
    their centres to be seen: every seed yields tens of clamped pairs that
    contribute."""
    from tests._util import identity_camera
    rng = np.random.default_rng(seed)
    xyz = np.hstack([rng.uniform(-0.9, 0.9, (n, 2)), rng.uniform(2.2, 2.8, (n, 1))])
    p = make_params(xyz, log_scales=rng.uniform(-1.5, -1.1, (3, n)), quats=rng.normal(size=(4, n)),
                    logits=rng.uniform(3.0, 7.0, n), sh=rng.normal(0, 0.25, ((deg + 1) ** 2 * 3, n)),
                    sh_degree=deg)
    p64 = {k: (v.astype(np.float64) if isinstance(v, np.ndarray) else v) for k, v in p.items()}
    return p64, identity_camera(W, H, 80.0), rng.normal(size=(3, H, W))


def test_alpha_clamp_branch_matches_torch_autograd():
    """R14: where opacity * G exceeds 0.99 the forward clamps alpha, so alpha has
    zero derivative there.  With opacities up to 0.999 the clamped branch is
    taken by contributing pairs, and the oracle's hand-written backward must
    still equal autograd of the transcription (whose clamp, like the forward,
    passes no gradient above 0.99)."""
    torch = pytest.importorskip("torch")
    for seed, deg, tile in ((31, 3, 16), (32, 1, 8), (33, 0, 32)):
        p, cam, w = clamp_scene(seed, deg)
        bg = (0.2, 0.1, 0.3)
        fw = pipeline.forward_view(p, cam, tile, bg)
        _, g = pipeline.backward_view(p, cam, fw, w, bg)
        # the clamped branch is exercised: count contributing pairs with o G > 0.99
        pr = fw["proj"]
        keys, gids, ranges = fw["lists"]
        W, H = cam["width"], cam["height"]
        tx = (W + tile - 1) // tile
        clamped = live = 0
        for t in range(ranges.shape[0]):
            gg = gids[ranges[t, 0]:ranges[t, 1]]
            X, Y = blend.tile_pixels(t % tx, t // tx, tile, W, H)
            r = blend.composite_tile(pr, gg, X + 0.5, Y + 0.5, bg)
            if gg.size:
                clamped += int((r["contrib"] & (r["a_raw"] > 0.99)).sum())
                live += int(r["contrib"].sum())
        assert clamped >= 20, (seed, clamped, live)
        P = {k: torch.tensor(p[k], dtype=torch.float64, requires_grad=True) for k in GROUPS}
        img = _torch_forward(torch, P, cam, fw, tile, bg)
        assert np.allclose(img.detach().numpy(), fw["image"], atol=1e-12)
        (img * torch.tensor(w)).sum().backward()
        for k in GROUPS:
            assert rel_l2(g[k], P[k].grad.numpy()) < 1e-9, (seed, k)


def test_alpha_clamp_opacity_derivative_by_finite_differences():
    """R14 by central differences: a Gaussian whose every contributing pair is
    clamped at 0.99 has exactly zero opacity-logit gradient, and one with no
    clamped pair has the FD derivative."""
    from tests._util import identity_camera
    cam = identity_camera(32, 32, 60.0)
    # two Gaussians stacked on the optical axis: the front one very opaque
    # (every pixel it reaches within one sigma is clamped), the back one not
    p = make_params([[0.0, 0.0, 2.0], [0.01, 0.0, 2.5]],
                    log_scales=np.full((3, 2), np.log(0.02)), logits=[8.0, 0.0],
                    sh=[[0.6, 0.2], [0.3, 0.5], [0.1, 0.7]])
    p = {k: (v.astype(np.float64) if isinstance(v, np.ndarray) else v) for k, v in p.items()}
    w = np.random.default_rng(4).normal(size=(3, 32, 32))
    fw = pipeline.forward_view(p, cam, 16)
    _, g = pipeline.backward_view(p, cam, fw, w)

    def L(logit0, logit1):
        q = dict(p, opacity_logits=np.array([logit0, logit1]))
        return float((pipeline.forward_view(q, cam, 16)["image"] * w).sum())

    h = 1e-6
    fd1 = (L(8.0, h) - L(8.0, -h)) / (2 * h)
    assert abs(g["opacity_logits"][1] - fd1) <= 1e-6 * max(abs(fd1), 1e-3)
    assert abs(fd1) > 1e-4
    # front Gaussian: pixels with o G > 0.99 contribute nothing; the others do, so
    # compare with FD (which sees the same clamp)
    fd0 = (L(8.0 + h, 0.0) - L(8.0 - h, 0.0)) / (2 * h)
    assert abs(g["opacity_logits"][0] - fd0) <= 1e-6 * max(abs(fd0), 1e-6)


def test_underflowed_opacity_gets_zero_gradient():
    """A logit so negative that the opacity is 0 in float32 (sigmoid(-120))
    makes the Gaussian invisible: its every gradient is exactly zero, and the
    other Gaussians' gradients are those of the scene without it."""
    p, cam, w = _scene(n=40, seed=41)
    p["opacity_logits"][7] = -120.0
    fw = pipeline.forward_view(p, cam, 16)
    _, g = pipeline.backward_view(p, cam, fw, w)
    for k in GROUPS:
        col = g[k][..., 7]
        assert np.all(np.isfinite(g[k])) and np.all(col == 0), k
    keep = np.array([i for i in range(40) if i != 7])
    q = {k: (v[..., keep] if isinstance(v, np.ndarray) else v) for k, v in p.items()}
    fq = pipeline.forward_view(q, cam, 16)
    _, gq = pipeline.backward_view(q, cam, fq, w)
    assert np.allclose(fw["image"], fq["image"], atol=1e-15)
    for k in GROUPS:
        assert np.allclose(g[k][..., keep], gq[k], rtol=1e-12, atol=1e-15), k
