"""Object lifetimes across the C ABI: a context destroyed while a frame it
created is alive stays usable by that frame, and is freed by the frame's
release; a later context on the device works normally."""
import ctypes as C

import numpy as np
import pytest
import torch

import gsscenes
from oracle import camera as ocam

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2509_05216_amd as P
    return P


def _render_raw(P, ctx_handle, params, cam, img, frame_handle):
    from paper_2509_05216_amd import _lib as L
    from paper_2509_05216_amd.core import _cam_array, _opts
    pa, keep = L.ptr_array([img.data_ptr()])
    o = _opts(16, 256, (0.0, 0.0, 0.0), 0)
    return L.lib().gs_render_fwd(ctx_handle, params.abi(), _cam_array([cam]), 1, pa, C.byref(o),
                                 C.byref(frame_handle), None)


def test_frame_outlives_destroyed_context(P):
    from paper_2509_05216_amd import _lib as L
    lib = L.lib()
    scene = gsscenes.make_scene("tiny", n=2000)
    params = P.Params.from_numpy(scene.params)
    cam = P.camera_from_dict(ocam.to_float32(ocam.orbit_cameras(4, 2.5, 60.0, 96, 80)[1]))
    ref, _ = P.render_fwd(P.Context(0), params, [cam])
    torch.cuda.synchronize()

    h = C.c_void_p()
    assert lib.gs_ctx_create(0, C.c_size_t(0), C.byref(h)) == 0
    img = torch.empty((3, 80, 96), device="cuda")
    fr = C.c_void_p()
    assert _render_raw(P, h, params, cam, img, fr) == 0
    torch.cuda.synchronize()
    lib.gs_ctx_destroy(h)                      # the frame still holds the context
    st = L.GsFrameStats()
    assert lib.gs_frame_stats_get(fr, C.byref(st)) == 0
    assert st.n_gaussians == 2000 and st.n_records > 0
    out = torch.empty(st.n_pixels, dtype=torch.int32, device="cuda")
    assert lib.gs_frame_export(fr, L.EXPORT["n_contrib"], -1, C.c_void_p(out.data_ptr()),
                               C.c_size_t(out.numel() * 4), None) == 0
    torch.cuda.synchronize()
    lib.gs_frame_release(fr)                   # frees the context too
    assert torch.equal(img, ref[0])

    # a new context on the same device is unaffected
    imgs, frame = P.render_fwd(P.Context(0), params, [cam])
    torch.cuda.synchronize()
    assert torch.equal(imgs[0], ref[0])
    frame.release()


def _views(P, sizes, start=0):
    return [P.camera_from_dict(ocam.to_float32(ocam.orbit_cameras(8, 2.5, 60.0, W, H)[start + i]))
            for i, (W, H) in enumerate(sizes)]


def test_graph_keeps_its_loss_workspace(P):
    """A captured step owns its loss workspace: a second graph on larger views and
    eager loss calls on a larger image (which grow the context's own workspace)
    must not disturb the replays of the first graph, which stay equal to the
    eager step on its views."""
    ctx = P.Context(0)
    scene = gsscenes.make_scene("tiny", n=3000)
    params = P.Params.from_numpy(scene.params)
    rng = np.random.default_rng(12)
    small = _views(P, [(96, 80), (64, 64)])
    tgt = [torch.tensor(rng.random((3, c.height, c.width)), dtype=torch.float32, device="cuda")
           for c in small]
    ga = P.StepGraph(ctx, params, small, tgt, with_adam=False)
    big = _views(P, [(320, 288), (256, 256)], start=2)
    tgt_b = [torch.tensor(rng.random((3, c.height, c.width)), dtype=torch.float32,
                          device="cuda") for c in big]
    gb = P.StepGraph(ctx, params, big, tgt_b, with_adam=False)
    # eager reference of graph A's step
    grads = params.zeros_like()
    imgs, frame = P.render_fwd(ctx, params, small)
    loss, dl = P.loss_grad(ctx, imgs, tgt, small)
    P.render_bwd(ctx, frame, params, dl, grads)
    torch.cuda.synchronize()
    ref_dl = [d.clone() for d in dl]
    huge = _views(P, [(640, 600)], start=5)
    x = torch.rand((3, 600, 640), device="cuda")
    for rep in range(3):
        gb.run()
        # an eager loss on a larger image than any graph's: the context workspace grows
        P.loss_grad(ctx, [x], [x * 0.5], huge)
        ga.run()
        torch.cuda.synchronize()
        for a, b in zip(ga.images, imgs):
            assert torch.equal(a, b), rep
        assert ga.loss.item() == loss.item(), rep
        for a, b in zip(ga.dl, ref_dl):
            assert torch.equal(a, b), rep
        for a, b in zip(ga.grads.tensors(), grads.tensors()):
            d = (a - b).abs().max().item()
            assert d <= 1e-5 * max(b.abs().max().item(), 1e-6), rep
    ga.close()
    gb.close()
    frame.release()


def test_server_first_batches_on_fresh_slots(P):
    """Each slot's first batch runs on a fresh frame (its device words cleared on
    the slot's own stream): a burst of requests that reaches every slot at once
    gives the images of eager rendering."""
    ctx = P.Context(0)
    a = gsscenes.make_scene("tiny", n=4000)
    b = gsscenes.make_scene("iso1m", n=3000, G=96)
    params = [P.Params.from_numpy(a.params), P.Params.from_numpy(b.params)]
    sizes = [(128, 96), (96, 96), (160, 128), (80, 64), (112, 112), (64, 48)]
    reqs = [(i % 2, c) for i, c in enumerate(_views(P, sizes))]
    refs = []
    for sid, cam in reqs:
        imgs, fr = P.render_fwd(ctx, params[sid], [cam])
        refs.append(imgs[0])
        fr.release()
    torch.cuda.synchronize()
    for trial in range(2):
        srv = P.Server(ctx, n_slots=6, max_batch_views=1)
        ids = [srv.add_scene(p) for p in params]
        tickets = [srv.submit(ids[sid], cam) for sid, cam in reqs]
        srv.drain()
        torch.cuda.synchronize()
        for (t, out), ref in zip(tickets, refs):
            assert torch.equal(out, ref), trial
        srv.close()


def test_entry_limit_is_checked_before_any_launch(P):
    """views x Gaussians past the frame's entry limit (2^32 - 2^20) is rejected with
    GS_ERR_CAPACITY on the host, before the parameters are touched (the count is set
    in the ABI struct; the arrays hold one Gaussian)."""
    from paper_2509_05216_amd import _lib as L
    from paper_2509_05216_amd.core import _cam_array, _opts
    ctx = P.Context(0)
    small = P.Params.from_numpy(gsscenes.make_scene("tiny", n=1000).params)
    ab = small.abi()
    ab.n = 1 << 28                           # 16 views x 2^28 = 2^32 > the limit
    cams = [P.camera_from_dict(c) for c in
            [ocam.to_float32(x) for x in ocam.orbit_cameras(16, 2.5, 60.0, 64, 64)]]
    imgs = [torch.empty((3, 64, 64), device="cuda") for _ in cams]
    pa, keep = L.ptr_array([t.data_ptr() for t in imgs])
    o = _opts(16, 256, (0.0, 0.0, 0.0), 0)
    fr = C.c_void_p()
    st = L.lib().gs_render_fwd(ctx.handle, ab, _cam_array(cams), 16, pa, C.byref(o),
                               C.byref(fr), None)
    assert st == -4, L.lib().gs_last_error()
    assert b"exceeds" in L.lib().gs_last_error()
    assert not fr.value
    ctx.close()
