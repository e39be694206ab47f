"""On-GPU isosurface extraction and target ray-casting (through the C ABI)
against the float64 oracle, on seeded volumes of the blob + noise field.

* extraction: every crossing point and the order bit-exact (within one
  float32 ulp), counts exact; odd grid sizes (not multiples of the
  4096-vertex block), subsampling by the Philox keep rule, an iso level with no
  crossing, a non-cubic box;
* ray-cast: images against the oracle's float64 ray-caster (same decisions:
  max abs error 1e-5), several views of different sizes in one launch;
* the in-situ chain: volume -> points -> Gaussians -> render.
"""
import numpy as np
import pytest
import torch

import gsscenes
from oracle import camera as ocam
from oracle import iso as OI

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2509_05216_amd as P
    return P


@pytest.fixture(scope="module")
def ctx(P):
    return P.Context(0)


@pytest.fixture(scope="module")
def field():
    return gsscenes.make_field("iso1m")[0]


def _check_points(got, want):
    assert got.shape == want.shape, (got.shape, want.shape)
    ulp = np.spacing(np.abs(want).astype(np.float32)).astype(np.float64)
    err = np.abs(got.astype(np.float64) - want)
    assert np.all(err <= ulp), err.max()


@pytest.mark.parametrize("shape,lo,hi,keep,seed", [
    ((61, 47, 53), (-1, -1, -1), (1, 1, 1), 1.0, 0),
    ((64, 64, 64), (-1, -1, -1), (1, 1, 1), 0.3, 11),
    ((17, 130, 33), (-1.0, -0.5, -1.0), (0.5, 1.0, 1.0), 1.0, 0),
    ((2, 2, 2), (-1, -1, -1), (1, 1, 1), 1.0, 0)])
def test_extraction_matches_oracle(P, ctx, field, shape, lo, hi, keep, seed):
    from paper_2509_05216_amd import iso
    nx, ny, nz = shape
    vol = gsscenes.sample_points_grid(field, nx, ny, nz, lo, hi)
    V = iso.Volume(torch.tensor(vol, device="cuda"), lo, hi)
    pts = iso.extract(ctx, V, 0.5, keep, seed).cpu().numpy()
    want, m = OI.extract(vol, lo, hi, 0.5, keep, seed)
    print(f"{shape}: {pts.shape[1]} of {m} crossings")
    if want.shape[1]:
        _check_points(pts, want)
    else:
        assert pts.shape[1] == 0
    assert iso.count(ctx, V, 0.5, keep, seed) == want.shape[1]
    # an iso level above every value: nothing
    assert iso.count(ctx, V, float(vol.max()) + 1.0) == 0


def test_extraction_capacity_error(P, ctx, field):
    import ctypes as C
    from paper_2509_05216_amd import _lib as L
    from paper_2509_05216_amd import iso
    vol = gsscenes.sample_points_grid(field, 40, 40, 40)
    V = iso.Volume(torch.tensor(vol, device="cuda"))
    n = iso.count(ctx, V)
    out = torch.full((3, n - 1), -7.0, device="cuda")
    k = C.c_int64()
    r = L.lib().gs_iso_extract(ctx.handle, V.abi(), 0.5, 1.0, 0, C.c_void_p(out.data_ptr()),
                               n - 1, C.byref(k), None)
    assert r == -4 and k.value == n
    torch.cuda.synchronize()
    assert float(out.max()) == -7.0 and float(out.min()) == -7.0


def test_raycast_matches_oracle(P, ctx, field):
    from paper_2509_05216_amd import iso
    vol = gsscenes.sample_points_grid(field, 48, 48, 48)
    V = iso.Volume(torch.tensor(vol, device="cuda"))
    cams = [ocam.to_float32(c) for c in ocam.orbit_cameras(5, 2.5, 60.0, 40, 32)][:2]
    cams.append(ocam.to_float32(ocam.orbit_cameras(5, 2.5, 60.0, 24, 36)[3]))
    step = float(np.float32(0.02))              # the float32 step the library receives
    imgs = iso.raycast(ctx, V, [P.camera_from_dict(c) for c in cams], 0.5, step)
    torch.cuda.synchronize()
    for img, c in zip(imgs, cams):
        want = OI.raycast(vol, (-1, -1, -1), (1, 1, 1), 0.5, c, step)
        got = img.cpu().numpy().astype(np.float64)
        err = np.abs(got - want).max()
        print(f"{c['width']}x{c['height']}: max abs {err:.2e}, hit pixels "
              f"{int((want.max(0) > 0).sum())}")
        assert err < 1e-5
        assert (want.max(0) > 0).sum() > 0.2 * c["width"] * c["height"]


def test_raycast_rejects_bad_steps(P, ctx, field):
    from paper_2509_05216_amd import iso
    vol = gsscenes.sample_points_grid(field, 8, 8, 8)
    V = iso.Volume(torch.tensor(vol, device="cuda"))
    cam = P.camera_from_dict(ocam.to_float32(ocam.orbit_cameras(1, 2.5, 60.0, 8, 8)[0]))
    for step in (0.0, -1.0, 1e-7):
        with pytest.raises(P.IsogsError):
            iso.raycast(ctx, V, [cam], 0.5, step)


def test_volume_to_gaussians_to_render(P, ctx, field):
    """The in-situ chain on the device: sampled volume, isosurface points,
    Gaussians initialised from them, a render that covers the ray-cast target."""
    from paper_2509_05216_amd import iso
    G = 128
    vol = gsscenes.sample_volume(field, G, device="cuda")
    V = iso.Volume(vol)
    m = iso.count(ctx, V)
    pts = iso.extract(ctx, V, 0.5, min(1.0, 50000 / m), 3)
    assert 0.8 * 50000 < pts.shape[1] < 1.2 * 50000
    h = 2.0 / (G - 1)
    params = P.init_from_points(ctx, pts.contiguous(), 0, log_scale=float(np.log(h)),
                                opacity_logit=2.0, seed=5)
    cams = [P.camera_from_dict(c) for c in
            [ocam.to_float32(c) for c in ocam.orbit_cameras(3, 2.5, 60.0, 96, 96)]]
    tgt = iso.raycast(ctx, V, cams, 0.5, 0.01)
    img, frame = P.render_fwd(ctx, params, cams)
    torch.cuda.synchronize()
    for a, t in zip(img, tgt):
        cover_t = (t.max(0).values > 0)
        cover_r = (a.max(0).values > 0.05)
        inter = (cover_t & cover_r).sum().item() / max(cover_t.sum().item(), 1)
        print(f"target coverage {cover_t.float().mean().item():.3f}, overlap {inter:.3f}")
        assert inter > 0.9
    frame.release()
