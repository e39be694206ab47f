"""Pins of the oracle's loss (SSIM identities, constant-image closed form,
torch conv2d autograd, finite differences) and Adam (torch.optim.Adam)."""
import numpy as np
import pytest

from oracle import adam, loss, pipeline


def _imgs(seed=0, H=24, W=30):
    rng = np.random.default_rng(seed)
    return rng.random((3, H, W)), rng.random((3, H, W))


def test_ssim_of_identical_images_is_one_with_zero_gradient():
    x, _ = _imgs()
    assert abs(loss.ssim(x, x) - 1.0) < 1e-12
    assert np.abs(loss.ssim_grad(x, x)).max() < 1e-15


def test_ssim_constant_images_closed_form():
    a, b = 0.3, 0.7
    x = np.full((3, 20, 20), a)
    y = np.full((3, 20, 20), b)
    S, _ = loss.ssim_terms(x, y)
    want = (2 * a * b + loss.C1) / (a * a + b * b + loss.C1)
    assert np.allclose(S[:, 5:-5, 5:-5], want, rtol=1e-12)


def test_window_is_normalised_gaussian():
    g = loss.window1d()
    assert abs(g.sum() - 1) < 1e-15 and g.size == 11
    assert abs(g[5] / g[6] - np.exp(1 / (2 * 1.5 ** 2))) < 1e-12


def test_l1_gradient_is_sign_over_count():
    x, y = _imgs(1)
    g = loss.view_loss_grad(x, y, lam=0.0)
    assert np.allclose(g, np.sign(x - y) / x.size)
    z = x.copy()
    assert np.all(loss.view_loss_grad(z, z, lam=0.0) == 0)


def test_ssim_grad_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    import torch.nn.functional as F
    x, y = _imgs(2)
    g1 = loss.window1d()
    win = torch.tensor(np.outer(g1, g1))[None, None].repeat(3, 1, 1, 1)
    X = torch.tensor(x[None], requires_grad=True)
    Y = torch.tensor(y[None])

    def f(t):
        return F.conv2d(t, win, padding=5, groups=3)

    mx, my = f(X), f(Y)
    sxx, syy, sxy = f(X * X) - mx ** 2, f(Y * Y) - my ** 2, f(X * Y) - mx * my
    S = ((2 * mx * my + loss.C1) * (2 * sxy + loss.C2)) / ((mx ** 2 + my ** 2 + loss.C1) * (sxx + syy + loss.C2))
    L = 0.8 * (X - Y).abs().mean() + 0.2 * (1 - S.mean())
    L.backward()
    assert abs(L.item() - loss.view_loss(x, y)) < 1e-13
    assert np.allclose(loss.view_loss_grad(x, y), X.grad.numpy()[0], rtol=1e-10, atol=1e-14)


def test_loss_grad_matches_central_differences():
    x, y = _imgs(3, 14, 16)
    g = loss.view_loss_grad(x, y)
    rng = np.random.default_rng(4)
    for _ in range(30):
        idx = tuple(int(rng.integers(0, s)) for s in x.shape)
        h = 1e-7
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (loss.view_loss(xp, y) - loss.view_loss(xm, y)) / (2 * h)
        assert abs(fd - g[idx]) < 1e-7 * max(1.0, abs(g[idx]) * 1e3)


def test_batch_loss_averages_views():
    a, b = _imgs(5)
    c, d = _imgs(6)
    L, gr = loss.batch_loss([a, c], [b, d])
    assert abs(L - 0.5 * (loss.view_loss(a, b) + loss.view_loss(c, d))) < 1e-15
    assert np.allclose(gr[0], 0.5 * loss.view_loss_grad(a, b))


def test_adam_matches_torch_optim():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(7)
    p0 = rng.normal(size=50)
    grads = [rng.normal(size=50) * 10 ** rng.uniform(-6, 1) for _ in range(6)]
    P = torch.tensor(p0, requires_grad=True)
    opt = torch.optim.Adam([P], lr=3e-3, betas=(0.9, 0.999), eps=1e-15)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for t, g in enumerate(grads, 1):
        P.grad = torch.tensor(g)
        opt.step()
        p, m, v = adam.adam_step(p, g, m, v, 3e-3, t)
        assert np.allclose(p, P.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_adam_all_groups_use_their_rates():
    rng = np.random.default_rng(8)
    n = 5
    params = {"means": rng.normal(size=(3, n)), "log_scales": rng.normal(size=(3, n)),
              "quats": rng.normal(size=(4, n)), "opacity_logits": rng.normal(size=n),
              "sh": rng.normal(size=(48, n)), "sh_degree": 3}
    grads = {k: np.ones_like(v) for k, v in params.items() if k != "sh_degree"}
    zeros = {k: np.zeros_like(v) for k, v in grads.items()}
    newp, _, _ = pipeline.adam_all(params, grads, zeros, zeros, 1)
    # first step with a constant gradient moves every coordinate by lr (eps negligible)
    lr = adam.DEFAULT_LR
    assert np.allclose(params["means"] - newp["means"], lr["means"])
    assert np.allclose(params["sh"][:3] - newp["sh"][:3], lr["sh_dc"])
    assert np.allclose(params["sh"][3:] - newp["sh"][3:], lr["sh_rest"])
    assert np.allclose(params["opacity_logits"] - newp["opacity_logits"], lr["opacity_logits"])
