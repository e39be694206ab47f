"""Adaptive density control on the GPU (through the C ABI) against the FP64 oracle.

* statistics: a batched forward with GS_RENDER_RADII, the L1+SSIM loss
  gradient and a backward that keeps its screen-space sums, accumulated twice;
  counts and largest radii bit-exact, the NDC gradient sums within 1e-4
  relative L2 (float32 screen gradients against float64);
* densify: seeded parameters, moments and statistics whose decisions lie away
  from their thresholds, plus exact ties of the gradient test; counts, the
  source index of every output and every copied parameter / moment bit-exact,
  the children's drawn means and reduced log-scales within a float32 ulp of
  the float64 oracle, new moments zero; degrees 0 and 3, with and without the
  size prune, 1-3 children, ragged sizes (not multiples of the 1024-Gaussian
  block), nothing selected, everything pruned;
* the densified set renders like the oracle's densified set;
* opacity reset bit-exact.
"""
import numpy as np
import pytest
import torch

import gsscenes
from oracle import camera as ocam
from oracle import density as OD
from oracle import loss as oloss
from oracle import pipeline
from tests._parity import assert_image
from tests._util import density_inputs, rel_l2

pytestmark = pytest.mark.gpu

KEYS = ("means", "log_scales", "quats", "opacity_logits", "sh")
EXT = 2.5
TAU = float(np.float32(2e-4))


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2509_05216_amd as P
    return P


@pytest.fixture(scope="module")
def D(P):
    from paper_2509_05216_amd import density as D
    return D


@pytest.fixture(scope="module")
def ctx(P):
    return P.Context(0)


def _cams(n, W, H):
    return [ocam.to_float32(c) for c in ocam.orbit_cameras(n, 2.5, 60.0, W, H)]


def _stats_dev(D, s):
    return D.DensityStats(torch.tensor(s["grad"], device="cuda"),
                          torch.tensor(s["count"], device="cuda"),
                          torch.tensor(s["max_radius"], device="cuda"))


def test_statistics_match_oracle(P, D, ctx):
    scene = gsscenes.make_scene("iso1m", n=3000, G=96)
    n = 3000
    cams = _cams(5, 128, 112)[:3]
    cams[2] = ocam.to_float32(ocam.orbit_cameras(5, 2.5, 60.0, 96, 144)[2])
    gcams = [P.camera_from_dict(c) for c in cams]
    rng = np.random.default_rng(21)
    params = P.Params.from_numpy(scene.params)
    stats = D.DensityStats.zeros(n)
    ostats = dict(grad=np.zeros(n), count=np.zeros(n), max_radius=np.zeros(n))
    for it in range(2):
        targets = [rng.random((3, c["height"], c["width"])).astype(np.float32) for c in cams]
        imgs, frame = P.render_fwd(ctx, params, gcams, flags=P.core.RADII)
        loss, dl = P.loss_grad(ctx, imgs, [torch.tensor(t, device="cuda") for t in targets],
                               gcams)
        P.render_bwd(ctx, frame, params, dl, keep_screen=True)
        D.accumulate(ctx, frame, stats, scale=len(cams))
        torch.cuda.synchronize()
        frame.release()
        # the oracle: forward, loss gradient, compositing derivative per view
        fws = [pipeline.forward_view(scene.params, c, 16) for c in cams]
        L, dimgs = oloss.batch_loss([f["image"] for f in fws], targets)
        sg, touched, radius = [], [], []
        for c, f, d in zip(cams, fws, dimgs):
            acc, _ = pipeline.backward_view(scene.params, c, f, d)
            sg.append(acc["m"])
            touched.append(f["proj"]["touched"])
            radius.append(f["proj"]["radius"])
        OD.accumulate(ostats, sg, touched, radius, [c["width"] for c in cams],
                      [c["height"] for c in cams], scale=len(cams))
        assert np.array_equal(stats.count.cpu().numpy(), ostats["count"].astype(np.int32))
        assert np.array_equal(stats.max_radius.cpu().numpy(),
                              ostats["max_radius"].astype(np.int32))
        e = rel_l2(stats.grad.cpu().numpy(), ostats["grad"])
        print(f"iteration {it}: grad sums rel L2 {e:.2e}, seen {int((ostats['count'] > 0).sum())}")
        assert e < 1e-4, e
    assert ostats["count"].max() == 6


def test_statistics_need_radii_and_kept_sums(P, D, ctx):
    scene = gsscenes.make_scene("tiny", n=500)
    params = P.Params.from_numpy(scene.params)
    gcams = [P.camera_from_dict(c) for c in _cams(2, 64, 64)]
    stats = D.DensityStats.zeros(500)
    dl = [torch.ones((3, 64, 64), device="cuda") * 1e-3 for _ in gcams]
    for radii, keep in ((False, True), (True, False)):
        _, frame = P.render_fwd(ctx, params, gcams, flags=P.core.RADII if radii else 0)
        P.render_bwd(ctx, frame, params, dl, keep_screen=keep)
        with pytest.raises(P.IsogsError):
            D.accumulate(ctx, frame, stats)
        frame.release()
    _, frame = P.render_fwd(ctx, params, gcams, flags=P.core.RADII)
    P.render_bwd(ctx, frame, params, dl, keep_screen=True)
    with pytest.raises(P.IsogsError):       # wrong size
        D.accumulate(ctx, frame, D.DensityStats.zeros(499))
    frame.release()


def _oracle_src(info, n_split):
    kc = info["split_src"][info["keep_child"]]
    return np.concatenate([np.nonzero(info["keep_orig"])[0], np.nonzero(info["keep_clone"])[0],
                           np.repeat(kc, n_split)]).astype(np.int64)


def _check_densify(P, D, ctx, n, deg, seed, max_screen, n_split, tau=TAU):
    p, m, v, s = density_inputs(n, deg, seed)
    opts = dict(grad_threshold=tau, max_screen=max_screen, n_split=n_split)
    po, mo, vo, info, src = D.densify(ctx, P.Params.from_numpy(p), P.Params.from_numpy(m),
                                      P.Params.from_numpy(v), _stats_dev(D, s), EXT, seed=seed,
                                      want_src=True, **opts)
    torch.cuda.synchronize()
    rp, rm, rv, ri = OD.densify(p, m, v, s, EXT, tau=tau, max_screen=max_screen,
                                n_split=n_split, seed=seed)
    for k in ("n_in", "n_out", "kept", "cloned", "split", "children", "pruned"):
        assert info[k] == ri[k], (k, info[k], ri[k])
    n_out = ri["n_out"]
    if n_out == 0:
        return ri
    want_src = _oracle_src(ri, n_split)
    assert np.array_equal(src.cpu().numpy().astype(np.int64), want_src)
    first_child = ri["kept"] + ri["cloned"]
    gp, gm, gv = po.to_numpy(), mo.to_numpy(), vo.to_numpy()
    for k in KEYS:
        got = np.asarray(gp[k]).reshape(-1, n_out)
        ref = np.asarray(rp[k], np.float64).reshape(-1, n_out)
        if k in ("means", "log_scales"):
            # copies exact; children within one float32 ulp of the float64 value
            assert np.array_equal(got[:, :first_child], ref[:, :first_child].astype(np.float32))
            c, r = got[:, first_child:].astype(np.float64), ref[:, first_child:]
            ulp = np.spacing(np.abs(r).astype(np.float32)).astype(np.float64)
            assert np.all(np.abs(c - r) <= ulp), (k, np.abs(c - r).max())
        else:
            assert np.array_equal(got, ref.astype(np.float32)), k
        for dev, orc in ((gm, rm), (gv, rv)):
            a = np.asarray(dev[k]).reshape(-1, n_out)
            b = np.asarray(orc[k], np.float64).reshape(-1, n_out).astype(np.float32)
            assert np.array_equal(a, b), k
            assert np.all(a[:, ri["kept"]:] == 0)
    return ri


@pytest.mark.parametrize("n,deg,seed,max_screen,n_split", [
    (3000, 3, 1, 0.0, 2), (3000, 3, 2, 20.0, 2), (1, 0, 3, 0.0, 2), (1023, 0, 4, 20.0, 1),
    (1025, 1, 5, 0.0, 3), (4096, 2, 6, 20.0, 2), (70001, 3, 7, 20.0, 2)])
def test_densify_matches_oracle(P, D, ctx, n, deg, seed, max_screen, n_split):
    ri = _check_densify(P, D, ctx, n, deg, seed, max_screen, n_split)
    print(f"n={n}: kept {ri['kept']} cloned {ri['cloned']} split {ri['split']} "
          f"children {ri['children']} pruned {ri['pruned']}")
    if n >= 3000:
        assert ri["cloned"] > 0 and ri["split"] > 0 and ri["pruned"] > 0 and ri["children"] > 0


def test_densify_nothing_selected_and_everything_pruned(P, D, ctx):
    # a threshold above every mean gradient: kept originals only (low opacities pruned)
    ri = _check_densify(P, D, ctx, 2000, 3, 8, 0.0, 2, tau=1.0)
    assert ri["cloned"] == ri["split"] == 0
    p, m, v, s = density_inputs(2000, 3, 8)
    # min_opacity 1 prunes every original and every new Gaussian
    po, mo, vo, info = D.densify(ctx, P.Params.from_numpy(p), P.Params.from_numpy(m),
                                 P.Params.from_numpy(v), _stats_dev(D, s), EXT, min_opacity=1.0)
    rp, _, _, r2 = OD.densify(p, m, v, s, EXT, min_opacity=1.0)
    assert info["n_out"] == 0 == r2["n_out"] and po.n == 0
    assert ri["n_out"] == 2000 - ri["pruned"]


def test_densify_rejects_bad_outputs(P, D, ctx):
    from paper_2509_05216_amd import _lib as L
    import ctypes as C
    p, m, v, s = density_inputs(500, 0, 9)
    pp, mm, vv = (P.Params.from_numpy(x) for x in (p, m, v))
    st = _stats_dev(D, s)
    o = D._opts(EXT, 1)
    info = L.GsDensityInfo()
    n_out = D.count(ctx, pp, mm, vv, st, EXT, seed=1)["n_out"]
    for size, code in ((n_out - 1, -4), (n_out + 1, -1)):
        outs = [D._empty(size, 0, "cuda") for _ in range(3)]
        r = L.lib().gs_densify(ctx.handle, pp.abi(), mm.abi(), vv.abi(), st.abi(), C.byref(o),
                               outs[0].abi(), outs[1].abi(), outs[2].abi(), None,
                               C.byref(info), None)
        assert r == code, (size, r)
    # output aliasing an input
    r = L.lib().gs_densify(ctx.handle, pp.abi(), mm.abi(), vv.abi(), st.abi(), C.byref(o),
                           pp.abi(), mm.abi(), vv.abi(), None, C.byref(info), None)
    assert r == -1


def test_densified_scene_renders_like_the_oracle(P, D, ctx):
    """Densify a small scene with the GPU and with the oracle from the same
    inputs, then render both sets: images within 1e-4."""
    scene = gsscenes.make_scene("iso1m", n=2500, G=96)
    base = dict(scene.params)
    rng = np.random.default_rng(31)
    n = 2500
    stats = dict(grad=(rng.uniform(0.2, 3.0, n) * TAU * 2).astype(np.float32),
                 count=np.full(n, 2, np.int32), max_radius=rng.integers(0, 30, n).astype(np.int32))
    zeros = {k: np.zeros_like(v) for k, v in base.items() if k != "sh_degree"}
    zeros["sh_degree"] = base["sh_degree"]
    po, _, _, info = D.densify(ctx, P.Params.from_numpy(base), P.Params.from_numpy(zeros),
                               P.Params.from_numpy(zeros), _stats_dev(D, stats), EXT, seed=77,
                               grad_threshold=TAU, max_screen=20.0)
    rp, _, _, ri = OD.densify(base, zeros, zeros, stats, EXT, tau=TAU, max_screen=20.0, seed=77)
    assert info["n_out"] == ri["n_out"] and ri["split"] > 0 and ri["cloned"] > 0
    rp32 = {k: (np.asarray(rp[k], np.float32) if k != "sh_degree" else rp[k]) for k in rp}
    cams = _cams(4, 128, 128)[:2]
    imgs, frame = P.render_fwd(ctx, po, [P.camera_from_dict(c) for c in cams])
    torch.cuda.synchronize()
    for img, c in zip(imgs, cams):
        f = pipeline.forward_view(rp32, c, 16)
        assert_image(f, img.cpu().numpy())
    frame.release()


def test_opacity_reset_matches_oracle(P, D, ctx):
    p, m, v, _ = density_inputs(3001, 1, 10)
    p["opacity_logits"][:5] = [np.inf, -np.inf, 0.0, -4.59511985, 20.0]
    pp, mm, vv = (P.Params.from_numpy(x) for x in (p, m, v))
    D.opacity_reset(ctx, pp, mm, vv, 0.01)
    torch.cuda.synchronize()
    rp, rm, rv = OD.opacity_reset(p, m, v, 0.01)
    assert np.array_equal(pp.opacity_logits.cpu().numpy(),
                          np.asarray(rp["opacity_logits"], np.float64).astype(np.float32))
    assert np.all(mm.opacity_logits.cpu().numpy() == 0)
    assert np.all(vv.opacity_logits.cpu().numpy() == 0)
    assert np.array_equal(mm.means.cpu().numpy(), m["means"])
