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
