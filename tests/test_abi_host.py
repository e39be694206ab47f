"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol that include/isogs.h declares, validates arguments, and its host
camera generator matches the oracle."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "isogs.h")).read()
    return sorted(set(re.findall(r"\b(gs_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import paper_2509_05216_amd._lib as L
    lib = L.lib()
    names = _declared()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    assert lib.gs_version().startswith(b"isogs")


def test_orbit_cameras_match_oracle():
    import paper_2509_05216_amd as P
    from oracle import camera
    for n, W, H in ((8, 256, 256), (7, 320, 200), (448, 512, 512)):
        ours = P.orbit_cameras(n, 2.5, 60.0, W, H)
        ref = camera.orbit_cameras(n, 2.5, 60.0, W, H)
        for a, b in zip(ours, ref):
            d = P.camera_to_dict(a)
            assert np.allclose(d["R"], b["R"], atol=2e-7)
            assert np.allclose(d["t"], b["t"], atol=1e-6)
            assert abs(d["fx"] - b["fx"]) < 1e-4 and d["cx"] == b["cx"] and d["cy"] == b["cy"]
            assert d["width"] == W and d["height"] == H and abs(d["z_near"] - 0.2) < 1e-7


def test_invalid_arguments_are_rejected():
    import ctypes as C
    import paper_2509_05216_amd._lib as L
    lib = L.lib()
    arr = (L.GsCamera * 2)()
    assert lib.gs_orbit_cameras(0, 2.5, 60.0, 64, 64, arr) == -1
    assert b"invalid" in lib.gs_last_error()
    assert lib.gs_orbit_cameras(2, 2.5, 60.0, 0, 64, arr) == -1
    assert lib.gs_orbit_cameras(2, 2.5, 60.0, 64, 20000, arr) == -1
    h = C.c_void_p()
    assert lib.gs_ctx_create(0, 0, None) == -1
    # null context / frame pointers
    assert lib.gs_render_fwd(None, L.GsParams(), arr, 1, None, None, None, None) == -1
    assert lib.gs_render_bwd(None, None, L.GsParams(), None, L.GsParams(), 0, None) == -1
    assert lib.gs_adam_step(None, L.GsParams(), L.GsParams(), L.GsParams(), L.GsParams(),
                            None, 1, None) == -1
    st = L.GsFrameStats()
    assert lib.gs_frame_stats_get(None, C.byref(st)) == -1
    lib.gs_frame_release(None)
    lib.gs_ctx_destroy(None)
