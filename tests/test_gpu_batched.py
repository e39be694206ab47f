"""The batched form: persistent work-queue compositing, the hipGraph-captured
step and the autotuner, each checked against the plain eager path (and the
oracle) on the same seeded inputs."""
import numpy as np
import pytest
import torch

import gsscenes
from oracle import camera as ocam
from oracle import pipeline
from tests._parity import assert_image, rel_l2

pytestmark = pytest.mark.gpu
GROUPS = ("means", "log_scales", "quats", "opacity_logits", "sh")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2509_05216_amd as P
    return P


@pytest.fixture(scope="module")
def ctx(P):
    return P.Context(0)


def _mixed_views(P):
    sizes = [(192, 160), (128, 128), (96, 72)]
    cams = [ocam.to_float32(ocam.orbit_cameras(6, 2.5, 60.0, W, H)[i])
            for i, (W, H) in enumerate(sizes)]
    return cams, [P.camera_from_dict(c) for c in cams]


@pytest.fixture(scope="module")
def scene():
    return gsscenes.make_scene("iso1m", n=5000, G=96)


@pytest.mark.parametrize("tile,depth", [(16, 256), (32, 64), (8, 64)])
def test_persistent_longest_first_matches_grid_and_oracle(P, ctx, scene, tile, depth):
    cams_d, cams = _mixed_views(P)
    params = P.Params.from_numpy(scene.params)
    flags = P.PERSISTENT | P.LONGEST_FIRST
    img0, f0 = P.render_fwd(ctx, params, cams, tile=tile, lds_depth=depth)
    img1, f1 = P.render_fwd(ctx, params, cams, tile=tile, lds_depth=depth, flags=flags)
    torch.cuda.synchronize()
    for a, b in zip(img0, img1):
        assert torch.equal(a, b)
    assert torch.equal(f0.export("keys"), f1.export("keys"))
    assert torch.equal(f0.export("n_contrib"), f1.export("n_contrib"))
    rng = np.random.default_rng(3)
    dl = [torch.tensor(rng.normal(size=(3, c.height, c.width)), dtype=torch.float32,
                       device="cuda") for c in cams]
    g0 = P.render_bwd(ctx, f0, params, dl)
    g1 = P.render_bwd(ctx, f1, params, dl)
    torch.cuda.synchronize()
    for a, b in zip(g0.tensors(), g1.tensors()):
        assert rel_l2(b.cpu().numpy(), a.cpu().numpy()) < 1e-5
    # and against the oracle
    off = 0
    for v, c in enumerate(cams_d):
        fw = pipeline.forward_view(scene.params, c, tile, tile_offset=off)
        off += fw["tiles"][0] * fw["tiles"][1]
        assert_image(fw, img1[v].cpu().numpy())


def _eager_step(P, ctx, params, cams, targets, grads):
    imgs, frame = P.render_fwd(ctx, params, cams)
    loss, dl = P.loss_grad(ctx, imgs, targets, cams)
    P.render_bwd(ctx, frame, params, dl, grads)
    return imgs, loss, dl


def test_capture_entry_point_matches_create(P, ctx, scene):
    """gs_step_graph_capture (measuring pass on the null stream) builds the same
    step as gs_step_graph_create on the same description."""
    import ctypes as C
    from paper_2509_05216_amd import _lib as L
    cams_d, cams = _mixed_views(P)
    params = P.Params.from_numpy(scene.params)
    rng = np.random.default_rng(6)
    targets = [torch.tensor(rng.random((3, c.height, c.width)), dtype=torch.float32,
                            device="cuda") for c in cams]
    g = P.StepGraph(ctx, params, cams, targets, with_adam=False,
                    render=dict(tile=16, lds_depth=128, flags=P.PERSISTENT | P.LONGEST_FIRST))
    g.run()
    torch.cuda.synchronize()
    imgs = [t.clone() for t in g.images]
    grads = [t.clone() for t in g.grads.tensors()]
    loss = g.loss.item()
    h = C.c_void_p()
    L.check(L.lib().gs_step_graph_capture(ctx.handle, C.byref(g._desc), C.byref(h)))
    try:
        rec = C.c_int64()
        for _ in range(2):
            L.check(L.lib().gs_step_graph_run(h, C.byref(rec), P.core._stream(None)))
            torch.cuda.synchronize()
            for a, b in zip(g.images, imgs):
                assert torch.equal(a, b)
            assert abs(g.loss.item() - loss) < 1e-6
            for a, b in zip(g.grads.tensors(), grads):
                assert rel_l2(a.cpu().numpy(), b.cpu().numpy()) < 1e-5
    finally:
        L.lib().gs_step_graph_destroy(h)


@pytest.mark.parametrize("nviews", [3, 1])
def test_graph_replays_match_eager(P, ctx, scene, nviews):
    # one view takes the same side-stream fork and join in the captured
    # projection backward as several
    cams_d, cams = _mixed_views(P)
    cams = cams[:nviews]
    params = P.Params.from_numpy(scene.params)
    rng = np.random.default_rng(4)
    targets = [torch.tensor(rng.random((3, c.height, c.width)), dtype=torch.float32,
                            device="cuda") for c in cams]
    g = P.StepGraph(ctx, params, cams, targets, with_adam=False,
                    render=dict(tile=16, lds_depth=128, flags=P.PERSISTENT | P.LONGEST_FIRST))
    ref_grads = params.zeros_like()
    ref_imgs, ref_loss, ref_dl = _eager_step(P, ctx, params, cams, targets, ref_grads)
    torch.cuda.synchronize()
    for rep in range(3):
        rec = g.run()
        torch.cuda.synchronize()
        # eager work between replays
        junk = torch.randn(1000, device="cuda").sum().item()
        assert np.isfinite(junk)
        for a, b in zip(g.images, ref_imgs):
            assert torch.equal(a, b), rep
        assert abs(g.loss.item() - ref_loss.item()) < 1e-6
        for a, b in zip(g.grads.tensors(), ref_grads.tensors()):
            assert rel_l2(a.cpu().numpy(), b.cpu().numpy()) < 1e-5, rep
        cap, rec2 = g.info()
        assert rec == rec2 and 0 < rec <= cap
    g.close()


def test_graph_adam_steps_match_eager(P, ctx, scene):
    cams_d, cams = _mixed_views(P)
    rng = np.random.default_rng(5)
    targets = [torch.tensor(rng.random((3, c.height, c.width)), dtype=torch.float32,
                            device="cuda") for c in cams]
    pg = P.Params.from_numpy(scene.params)
    pe = P.Params.from_numpy(scene.params)
    p0 = [t.clone() for t in pe.tensors()]
    g = P.StepGraph(ctx, pg, cams, targets, with_adam=True, first_step=1)
    ge = pe.zeros_like()
    me, ve = pe.zeros_like(), pe.zeros_like()
    for t in range(1, 4):
        g.run()
        _eager_step(P, ctx, pe, cams, targets, ge)
        P.adam_step(ctx, pe, ge, me, ve, t)
        torch.cuda.synchronize()
        # parameter changes agree (gradient sums differ only in atomic order)
        for a, b, z in zip(pg.tensors(), pe.tensors(), p0):
            assert rel_l2((a - z).cpu().numpy(), (b - z).cpu().numpy()) < 1e-3, t
    g.close()


def test_graph_record_overflow_regrows(P, ctx):
    scene = gsscenes.make_scene("tiny", n=20000)
    cams_d = [ocam.to_float32(c) for c in ocam.orbit_cameras(2, 2.5, 60.0, 160, 160)]
    cams = [P.camera_from_dict(c) for c in cams_d]
    params = P.Params.from_numpy(scene.params)
    targets = [torch.zeros((3, 160, 160), device="cuda") for _ in cams]
    g = P.StepGraph(ctx, params, cams, targets, with_adam=False, capacity_slack=1.05)
    cap0, rec0 = g.info()
    # grow every Gaussian: the records outgrow the captured capacity
    params.log_scales.add_(1.2)
    torch.cuda.synchronize()
    g.launch()
    over, rec = g.sync()
    assert over and rec > cap0
    cap1, _ = g.info()
    assert cap1 >= rec
    rec_run = g.run()
    ref_grads = params.zeros_like()
    ref_imgs, ref_loss, _ = _eager_step(P, ctx, params, cams, targets, ref_grads)
    torch.cuda.synchronize()
    assert rec_run == rec
    for a, b in zip(g.images, ref_imgs):
        assert torch.equal(a, b)
    g.close()


def test_autotune_returns_a_valid_option(P, ctx, scene, tmp_path):
    cams_d, cams = _mixed_views(P)
    params = P.Params.from_numpy(scene.params)
    best, table = P.autotune(ctx, params, cams, reps=1, cache=str(tmp_path / "tune.json"))
    assert best["tile"] in (8, 16, 32) and best["lds_depth"] in (32, 64, 128, 256)
    assert len(table) == 17 and all(r["ms"] > 0 for r in table)
    assert min(r["ms"] for r in table) == min(r["ms"] for r in table
                                              if (r["tile"], r["lds_depth"], r["flags"]) ==
                                              (best["tile"], best["lds_depth"], best["flags"]))
    best2, _ = P.autotune(ctx, params, cams, reps=1, cache=str(tmp_path / "tune.json"))
    assert best2 == best
