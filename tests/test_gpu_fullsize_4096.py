"""Parity at 4096^2, the resolution of the 18M-Gaussian mixing-layer workload.

Scene: the mixing-layer recipe (tanh layer displaced by sinusoidal modes plus
noise, SH degree 3, log-scales log(h) +- 0.5) on a seeded 1024^3 grid with
6M Gaussians, so that scene generation and the oracle's projection fit the
test's time; two 4096^2 views in one batched call (about 88M records per
view at tile 8).  Launch configurations: tile 8, LDS depth 64, one workgroup
per tile (what the autotuner picks for this workload) and tile 16, depth 256,
persistent longest-first.

At this size mean2D reaches 4096 px, where a float32 mean keeps only ~2.4e-4 px;
the splat records carry the integer part and the fraction separately, and
the bit-exact rectangles and the per-pixel image tolerance check that path.
Checks, as for the 2048^2 workload: every Gaussian's rectangle and float32
depth bits against the oracle's projection (all 6M, both views) and the
record count; sampled tiles' records, pixels, final T and last contributor;
parameter gradients from an upstream gradient that is nonzero only on the
sampled tiles.
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
S = 4096
N_SAMPLE = 4  # random tiles per view, besides the longest


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
def big(P):
    scene = gsscenes.make_scene("miranda18m", n=6_000_000, G=1024)
    base = ocam.orbit_cameras(16, 2.5, 60.0, S, S)
    cams = [ocam.to_float32(base[0]), ocam.to_float32(base[8])]
    params = P.Params.from_numpy(scene.params)
    print(f"\n[4096] scene {scene.params['means'].shape[1]} Gaussians", flush=True)
    return scene, cams, params, {}


def _sub_proj(pr, idx):
    n = pr["m"].shape[1]
    return {k: (v[..., idx] if isinstance(v, np.ndarray) and v.ndim >= 1 and v.shape[-1] == n
                else v) for k, v in pr.items()}


@pytest.mark.parametrize("tile,depth,flags", [(8, 64, 0), (16, 256, 3)])
def test_4096_forward_backward_sampled(P, ctx, big, tile, depth, flags):
    scene, cams, params, cache = big
    n = scene.params["means"].shape[1]
    gcams = [P.camera_from_dict(c) for c in cams]
    imgs, frame = P.render_fwd(ctx, params, gcams, tile=tile, lds_depth=depth, flags=flags)
    torch.cuda.synchronize()
    st = frame.stats()
    keys_d = frame.export("keys")
    vals_d = frame.export("values")
    ranges = frame.export("ranges").cpu().numpy().view(np.uint32).reshape(-1, 2).astype(np.int64)
    finT = frame.export("final_T")
    ncon = frame.export("n_contrib")
    rects = frame.export("rects").cpu().numpy().view(np.uint32).reshape(len(cams), n, 2)
    depth_bits = frame.export("depths").cpu().numpy().view(np.uint32).reshape(len(cams), n)
    print(f"[4096] tile {tile}: K = {st['n_records']}", flush=True)

    rng = np.random.default_rng(4096 + tile)
    dl = [torch.zeros((3, S, S), dtype=torch.float32, device="cuda") for _ in cams]
    acc_all, subs = [], []
    tile_off = pix_off = 0
    k_total = 0
    tx = ty = S // tile
    for v, cam in enumerate(cams):
        key = (v, tile)
        if key not in cache:
            cache.clear()  # one projection held at a time
            cache[key] = project.project(scene.params, cam, tile)
        pr = cache[key]
        t = pr["touched"]
        r = rects[v]
        x0, y0 = r[:, 0] & 0xFFFF, r[:, 0] >> 16
        x1, y1 = r[:, 1] & 0xFFFF, r[:, 1] >> 16
        assert np.all(x1[~t] < x0[~t]), v
        for got, want in ((x0, 0), (y0, 1), (x1, 2), (y1, 3)):
            assert np.array_equal(got[t].astype(np.int64), pr["rect"][want, t]), (v, want)
        assert np.array_equal(depth_bits[v][t],
                              np.asarray(pr["depth32"], np.float32)[t].view(np.uint32)), v
        assert np.all(depth_bits[v][~t] == 0xFFFFFFFF), v
        area = (pr["rect"][2, t] - pr["rect"][0, t] + 1) * (pr["rect"][3, t] - pr["rect"][1, t] + 1)
        vr = ranges[tile_off:tile_off + tx * ty]
        lens = vr[:, 1] - vr[:, 0]
        assert int(lens.sum()) == int(area.sum()), v
        k_total += int(area.sum())
        nonempty = np.nonzero(lens > 0)[0]
        pick = [int(np.argmax(lens))] + [int(x) for x in rng.choice(nonempty, N_SAMPLE,
                                                                    replace=False)]
        bits = binning.depth_bits(pr["depth32"])
        acc = dict(m=np.zeros((2, n)), conic=np.zeros((3, n)), opacity=np.zeros(n),
                   rgb=np.zeros((3, n)))
        for lt in pick:
            cx, cy = lt % tx, lt // tx
            members = np.nonzero(t & (pr["rect"][0] <= cx) & (cx <= pr["rect"][2])
                                 & (pr["rect"][1] <= cy) & (cy <= pr["rect"][3]))[0]
            g = members[np.argsort(bits[members], kind="stable")]
            a, b = (int(x) for x in vr[lt])
            got_keys = keys_d[a:b].cpu().numpy().view(np.uint64)
            got_vals = vals_d[a:b].cpu().numpy().view(np.uint32).astype(np.int64)
            want_keys = (np.uint64(tile_off + lt) << np.uint64(32)) | bits[g]
            assert np.array_equal(got_keys, want_keys), (v, lt)
            assert np.array_equal(got_vals, v * n + g), (v, lt)
            X, Y = blend.tile_pixels(cx, cy, tile, S, S)
            Xt, Yt = torch.as_tensor(X, device="cuda"), torch.as_tensor(Y, device="cuda")
            img = imgs[v][:, Yt, Xt].cpu().numpy()
            rep = tile_report(pr, g, X, Y, img)
            assert not rep["failed"], (v, lt, rep["failed"][:5])
            o = rep["oracle"]
            ok = ~o["flags"]
            pix = torch.as_tensor(pix_off + Y * S + X, device="cuda")
            fT = finT[pix].cpu().numpy()
            nc = ncon[pix].cpu().numpy().view(np.uint32).astype(np.int64)
            assert np.abs(fT - o["T"])[ok].max() < 1e-5, (v, lt)
            assert np.array_equal(nc[ok], o["n"][ok]), (v, lt)
            print(f"[4096] tile {tile} view {v} tile {lt}: list {g.size}, max err "
                  f"{rep['max_err']:.2e}, flagged {rep['n_flagged']}", flush=True)
            w = rng.normal(size=(3, X.size)) * ok[None, :]
            dl[v][:, Yt, Xt] = torch.tensor(w, dtype=torch.float32, device="cuda")
            blend.backward_tile(pr, g, X + 0.5, Y + 0.5, w, (0.0, 0.0, 0.0), acc)
        live = np.nonzero(np.abs(np.concatenate([acc[k].reshape(-1, n) for k in acc])).sum(0)
                          > 0)[0]
        subs.append(live)
        acc_all.append(obwd.param_grads(
            _sub_proj(pr, live), gsscenes.subset(scene.params, live), cam,
            {k: a_[..., live] for k, a_ in acc.items()}))
        tile_off += tx * ty
        pix_off += S * S
    assert st["n_records"] == k_total
    del keys_d, vals_d

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
        print(f"[4096] tile {tile} {k}: rel L2 {e:.2e} over {union.size} Gaussians", flush=True)
        assert e < 1e-3, (k, e)
        assert np.all(gg[k][..., outside] == 0), k
    frame.release()
