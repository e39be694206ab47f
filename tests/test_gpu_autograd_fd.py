"""The autograd form against central finite differences of the FP64 oracle.

A seeded 1,000-Gaussian subset of the 1M-Gaussian scene (SH degree 3,
anisotropic log-scales U(-5, -3), random rotations) is rendered through
``rasterize`` (the torch.autograd.Function over the C ABI) and the scalar
L = sum(w * image) is differentiated by autograd.  The reference is the
central difference of the oracle's forward (float64) at step h and 2h for a
seeded sample of parameter coordinates of Gaussians the view touches;
coordinates whose two estimates disagree by more than 1% (a threshold crossed
between them) are skipped.  Bar: 1e-3 relative L2 over the checked set.
"""
import numpy as np
import pytest
import torch

import gsscenes
from oracle import camera as ocam
from oracle import pipeline, project
from tests._parity import rel_l2

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]

GROUPS = ("means", "log_scales", "quats", "opacity_logits", "sh")
W = H = 192
PER_GROUP = 12


def subset_scene():
    scene = gsscenes.make_scene("iso1m")
    rng = np.random.default_rng(7)
    idx = np.sort(rng.choice(scene.params["means"].shape[1], 1000, replace=False))
    p = gsscenes.subset(scene.params, idx)
    c = ocam.orbit_cameras(128, 2.5, 60.0, 1024, 1024)[0]
    c.update(fx=c["fx"] * W / 1024, fy=c["fy"] * H / 1024, cx=W / 2, cy=H / 2, width=W, height=H)
    return p, ocam.to_float32(c)


def oracle_loss(p64, cam, w):
    return float((pipeline.forward_view(p64, cam, 16)["image"] * w).sum())


def central_differences(p, cam, w, seed=3):
    """[(group, row, col, fd)] for a seeded sample of coordinates of touched Gaussians."""
    p64 = {k: (v.astype(np.float64) if isinstance(v, np.ndarray) else v) for k, v in p.items()}
    touched = np.nonzero(project.project(p64, cam, 16)["touched"])[0]
    rng = np.random.default_rng(seed)
    out = []
    for k in GROUPS:
        rows = p64[k].shape[0] if p64[k].ndim == 2 else 1
        for _ in range(PER_GROUP):
            i = int(rng.choice(touched))
            r = int(rng.integers(0, rows))
            x0 = p64[k][r, i] if p64[k].ndim == 2 else p64[k][i]
            est = []
            for h in (1e-6 * max(1.0, abs(x0)), 2e-6 * max(1.0, abs(x0))):
                vals = []
                for sgn in (1, -1):
                    q = dict(p64)
                    q[k] = p64[k].copy()
                    if q[k].ndim == 2:
                        q[k][r, i] += sgn * h
                    else:
                        q[k][i] += sgn * h
                    vals.append(oracle_loss(q, cam, w))
                est.append((vals[0] - vals[1]) / (2 * h))
            if abs(est[0] - est[1]) > 1e-2 * max(abs(est[0]), 1e-8):
                continue  # a threshold was crossed between the two steps
            out.append((k, r, i, est[0]))
    return out


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2509_05216_amd as P
    return P


def test_autograd_matches_central_differences(P):
    ctx = P.Context(0)
    p, cam = subset_scene()
    w = np.random.default_rng(11).normal(size=(3, H, W))
    tensors = [torch.tensor(p[k], dtype=torch.float32, device="cuda", requires_grad=True)
               for k in GROUPS]
    img = P.rasterize(ctx, tensors, p["sh_degree"], [P.camera_from_dict(cam)])
    loss = (img[0] * torch.tensor(w, dtype=torch.float32, device="cuda")).sum()
    loss.backward()
    torch.cuda.synchronize()
    g = {k: t.grad.cpu().numpy().astype(np.float64) for k, t in zip(GROUPS, tensors)}
    fd = central_differences(p, cam, w)
    assert len(fd) >= 40, len(fd)
    got = np.array([g[k][r, i] if g[k].ndim == 2 else g[k][i] for k, r, i, _ in fd])
    want = np.array([v for *_, v in fd])
    e = rel_l2(got, want)
    print(f"autograd vs central differences: rel L2 {e:.2e} over {len(fd)} coordinates")
    assert e < 1e-3, e
    for k in GROUPS:
        sel = [j for j, (kk, *_r) in enumerate(fd) if kk == k]
        if sel:
            print(f"  {k}: rel L2 {rel_l2(got[sel], want[sel]):.2e} ({len(sel)})")
