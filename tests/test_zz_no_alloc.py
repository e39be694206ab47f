"""gs_loss_grad_noalloc (the loss gradient on a fixed device workspace, for
callers that cannot allocate) against gs_loss_grad, through the C ABI: two
calls in a row, the second on smaller views, bit-identical loss and image
gradients; no library allocation on a fresh context; views beyond the fixed
workspace rejected before any launch."""
import numpy as np
import pytest
import torch

from oracle import loss as oloss

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2509_05216_amd as P
    return P


def _views(P, sizes, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    cams, xs, ys = [], [], []
    for W, H in sizes:
        cams.append(P.camera(np.eye(3), np.zeros(3), 200.0, 200.0, W / 2, H / 2, W, H))
        y = torch.rand((3, H, W), generator=g)
        x = (y + 0.2 * torch.randn((3, H, W), generator=g)).clamp_(0, 1)
        xs.append(x.cuda())
        ys.append(y.cuda())
    return cams, xs, ys


def _run(P, ctx, cams, xs, ys, noalloc):
    loss = torch.full((1,), float("nan"), device="cuda")
    grads = [torch.full_like(x, float("nan")) for x in xs]
    P.loss_grad_into(ctx, xs, ys, cams, loss, grads, 0.2, noalloc=noalloc)
    return loss, grads


def test_noalloc_matches_allocating_call_twice(P):
    ctx = P.Context(0)
    # first call: views up to the workspace's 2^20-pixel limit (square, ragged, and a
    # 16384 x 64 strip); second call: smaller views
    big = _views(P, [(1024, 1024), (640, 480), (333, 517), (16384, 64)], 11)
    small = _views(P, [(200, 150), (97, 61)], 12)
    out_big = _run(P, ctx, *big, noalloc=True)
    out_small = _run(P, ctx, *small, noalloc=True)
    torch.cuda.synchronize()
    assert ctx.memory() == (0, 0), "the allocation-free call allocated library memory"
    ref_big = _run(P, ctx, *big, noalloc=False)
    ref_small = _run(P, ctx, *small, noalloc=False)
    torch.cuda.synchronize()
    for (l, g), (rl, rg) in ((out_big, ref_big), (out_small, ref_small)):
        assert torch.equal(l, rl), (l.item(), rl.item())
        for a, b in zip(g, rg):
            assert torch.equal(a, b)
    # and the smaller call against the oracle's loss and gradient (float64)
    cams, xs, ys = small
    xn = [x.cpu().double().numpy() for x in xs]
    yn = [y.cpu().double().numpy() for y in ys]
    L, G = oloss.batch_loss(xn, yn)
    assert abs(out_small[0].item() - L) < 1e-5 * max(1.0, abs(L))
    for v in range(len(xs)):
        gv = out_small[1][v].cpu().double().numpy()
        e = np.linalg.norm(gv - G[v]) / np.linalg.norm(G[v])
        assert e < 1e-4, e
    ctx.close()


def test_noalloc_sixteen_views_at_the_limit(P):
    ctx = P.Context(0)
    views = _views(P, [(1024, 1024)] * 16, 13)
    out = _run(P, ctx, *views, noalloc=True)
    ref = _run(P, ctx, *views, noalloc=False)
    torch.cuda.synchronize()
    assert torch.equal(out[0], ref[0])
    for a, b in zip(out[1], ref[1]):
        assert torch.equal(a, b)
    ctx.close()


def test_noalloc_rejects_views_beyond_the_workspace(P):
    ctx = P.Context(0)
    for sizes in ([(1025, 1024)], [(64, 64), (2048, 1024)]):
        cams, xs, ys = _views(P, sizes, 14)
        loss = torch.full((1,), 7.0, device="cuda")
        with pytest.raises(P.IsogsError) as e:
            P.loss_grad_into(ctx, xs, ys, cams, loss, None, 0.2, noalloc=True)
        assert e.value.status == -4 and "1048576 pixels per view" in str(e.value)
        torch.cuda.synchronize()
        assert loss.item() == 7.0
    assert ctx.memory() == (0, 0)
    ctx.close()
