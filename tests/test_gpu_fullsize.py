"""Parity at the full benchmark workload, in the launch configurations it times.

Workload: the 4M-Gaussian scene (SH degree 3) and four views (2 x 2048^2 +
2 x 1536^2) rendered in one batched call, with the persistent longest-first
compositing kernels and with one workgroup per tile.

The oracle cannot composite whole 2048^2 views in test time, so:
* every Gaussian's tile rectangle and float32 depth bits (all 4M, every view)
  are compared with the oracle's projection, bit for bit, and the record
  count with the oracle's sum of rectangle areas;
* on a seeded sample of tiles per view (always including the view's longest
  list) the tile's sorted records (keys, values) must be identical, and its
  pixels, final transmittance and last contributor must match the oracle's
  compositing of that list;
* the backward is driven by an upstream gradient that is nonzero only on the
  sampled tiles, so the oracle's backward over those tiles alone yields every
  parameter gradient; Gaussians outside them must get exactly zero.
"""
import numpy as np
import pytest
import torch

import gsscenes
from oracle import backward as obwd
from oracle import binning, blend, project
from oracle import camera as ocam
from tests._parity import rel_l2, tile_report

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

GROUPS = ("means", "log_scales", "quats", "opacity_logits", "sh")
TILE, DEPTH = 16, 256
SIZES = (2048, 2048, 1536, 1536)
N_SAMPLE = 5  # random tiles per view, besides the longest


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2509_05216_amd as P
    return P


@pytest.fixture(scope="module")
def ctx(P):
    return P.Context(0)


def _cams():
    base = ocam.orbit_cameras(16, 2.5, 60.0, 2048, 2048)
    out = []
    for i, s in enumerate(SIZES):
        c = dict(base[i * 4])
        c.update(fx=c["fx"] * s / 2048, fy=c["fy"] * s / 2048, cx=s / 2, cy=s / 2, width=s,
                 height=s)
        out.append(ocam.to_float32(c))
    return out


@pytest.fixture(scope="module")
def full(P, ctx):
    scene = gsscenes.make_scene("kingsnake4m")
    cams = _cams()
    params = P.Params.from_numpy(scene.params)
    print(f"\n[fullsize] scene {scene.params['means'].shape[1]} Gaussians", flush=True)
    return scene, cams, params


def _sub_proj(pr, idx):
    n = pr["m"].shape[1]
    return {k: (v[..., idx] if isinstance(v, np.ndarray) and v.ndim >= 1 and v.shape[-1] == n
                else v) for k, v in pr.items()}


def test_fullsize_forward_backward_sampled(P, ctx, full):
    scene, cams, params = full
    n = scene.params["means"].shape[1]
    gcams = [P.camera_from_dict(c) for c in cams]
    imgs, frame = P.render_fwd(ctx, params, gcams, tile=TILE, lds_depth=DEPTH,
                               flags=P.PERSISTENT | P.LONGEST_FIRST)
    torch.cuda.synchronize()
    st = frame.stats()
    keys = frame.export("keys").cpu().numpy().view(np.uint64)
    vals = frame.export("values").cpu().numpy().view(np.uint32).astype(np.int64)
    ranges = frame.export("ranges").cpu().numpy().view(np.uint32).reshape(-1, 2).astype(np.int64)
    finT = frame.export("final_T").cpu().numpy()
    ncon = frame.export("n_contrib").cpu().numpy().view(np.uint32).astype(np.int64)
    rects = frame.export("rects").cpu().numpy().view(np.uint32).reshape(len(cams), n, 2)
    depth = frame.export("depths").cpu().numpy().view(np.uint32).reshape(len(cams), n)
    print(f"[fullsize] K = {st['n_records']}", flush=True)

    rng = np.random.default_rng(2024)
    dl = [torch.zeros((3, s, s), dtype=torch.float32, device="cuda") for s in SIZES]
    acc_all, subs = [], []
    tile_off = pix_off = 0
    k_total = 0
    for v, (cam, s) in enumerate(zip(cams, SIZES)):
        pr = project.project(scene.params, cam, TILE)
        tx = ty = s // TILE
        # every Gaussian: rectangle (bit-exact) and depth bits of the touched ones
        t = pr["touched"]
        r = rects[v]
        x0, y0 = r[:, 0] & 0xFFFF, r[:, 0] >> 16
        x1, y1 = r[:, 1] & 0xFFFF, r[:, 1] >> 16
        assert np.array_equal(x1[~t] < x0[~t], np.ones((~t).sum(), bool)), v
        for got, want in ((x0, 0), (y0, 1), (x1, 2), (y1, 3)):
            assert np.array_equal(got[t].astype(np.int64), pr["rect"][want, t]), (v, want)
        assert np.array_equal(depth[v][t], np.asarray(pr["depth32"], np.float32)[t].view(np.uint32)), v
        assert np.all(depth[v][~t] == 0xFFFFFFFF), v
        area = (pr["rect"][2, t] - pr["rect"][0, t] + 1) * (pr["rect"][3, t] - pr["rect"][1, t] + 1)
        k_view = int(area.sum())
        vr = ranges[tile_off:tile_off + tx * ty]
        lens = vr[:, 1] - vr[:, 0]
        assert int(lens.sum()) == k_view, v
        k_total += k_view
        # sampled tiles: longest list plus seeded random non-empty ones
        nonempty = np.nonzero(lens > 0)[0]
        pick = [int(np.argmax(lens))] + [int(x) for x in rng.choice(nonempty, N_SAMPLE,
                                                                    replace=False)]
        bits = binning.depth_bits(pr["depth32"])
        acc = dict(m=np.zeros((2, n)), conic=np.zeros((3, n)), opacity=np.zeros(n),
                   rgb=np.zeros((3, n)))
        img = imgs[v].cpu().numpy()
        for lt in pick:
            cx, cy = lt % tx, lt // tx
            members = np.nonzero(t & (pr["rect"][0] <= cx) & (cx <= pr["rect"][2])
                                 & (pr["rect"][1] <= cy) & (cy <= pr["rect"][3]))[0]
            g = members[np.argsort(bits[members], kind="stable")]
            a, b = vr[lt]
            want_keys = (np.uint64(tile_off + lt) << np.uint64(32)) | bits[g]
            assert np.array_equal(keys[a:b], want_keys), (v, lt)
            assert np.array_equal(vals[a:b], v * n + g), (v, lt)
            X, Y = blend.tile_pixels(cx, cy, TILE, s, s)
            rep = tile_report(pr, g, X, Y, img[:, Y, X])
            assert not rep["failed"], (v, lt, rep["failed"][:5])
            o = rep["oracle"]
            ok = ~o["flags"]
            pix = pix_off + Y * s + X
            assert np.abs(finT[pix] - o["T"])[ok].max() < 1e-5, (v, lt)
            assert np.array_equal(ncon[pix][ok], o["n"][ok]), (v, lt)
            print(f"[fullsize] view {v} tile {lt}: list {g.size}, max err "
                  f"{rep['max_err']:.2e}, flagged {rep['n_flagged']}", flush=True)
            # upstream gradient on this tile only (zero at flagged pixels, where the
            # two sides may legitimately take different branches)
            w = rng.normal(size=(3, X.size)) * ok[None, :]
            dl[v][:, torch.as_tensor(Y), torch.as_tensor(X)] = torch.tensor(
                w, dtype=torch.float32, device="cuda")
            blend.backward_tile(pr, g, X + 0.5, Y + 0.5, w, (0.0, 0.0, 0.0), acc)
        live = np.nonzero(np.abs(np.concatenate([acc[k].reshape(-1, n) for k in acc])).sum(0)
                          > 0)[0]
        subs.append(live)
        sub = _sub_proj(pr, live)
        acc_all.append(obwd.param_grads(
            sub, gsscenes.subset(scene.params, live), cam,
            {k: a_[..., live] for k, a_ in acc.items()}))
        del pr, sub
        tile_off += tx * ty
        pix_off += s * s
    assert st["n_records"] == k_total

    grads = P.render_bwd(ctx, frame, params, dl)
    torch.cuda.synchronize()
    gg = grads.to_numpy()
    union = np.unique(np.concatenate(subs))
    outside = np.ones(n, bool)
    outside[union] = False
    for k in GROUPS:
        want = np.zeros(gg[k][..., union].shape)
        for live, gv in zip(subs, acc_all):
            want[..., np.searchsorted(union, live)] += gv[k]
        e = rel_l2(gg[k][..., union], want)
        print(f"[fullsize] {k}: rel L2 {e:.2e} over {union.size} Gaussians", flush=True)
        assert e < 1e-3, (k, e)
        assert np.all(gg[k][..., outside] == 0), k
    frame.release()


def test_fullsize_grid_equals_persistent(P, ctx, full):
    """The one-workgroup-per-tile launch gives the same images and records."""
    scene, cams, params = full
    gcams = [P.camera_from_dict(c) for c in cams]
    a, fa = P.render_fwd(ctx, params, gcams, tile=TILE, lds_depth=DEPTH,
                         flags=P.PERSISTENT | P.LONGEST_FIRST)
    b, fb = P.render_fwd(ctx, params, gcams, tile=TILE, lds_depth=DEPTH, flags=0)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    assert torch.equal(fa.export("keys"), fb.export("keys"))
    assert torch.equal(fa.export("n_contrib"), fb.export("n_contrib"))
    fa.release()
    fb.release()
