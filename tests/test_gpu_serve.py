"""The serving form: resident scenes, continuous batching, memory admission.

A request's image must be the same rendered alone and in a mix of scenes and
resolutions, and must match the oracle."""
import numpy as np
import pytest
import torch

import gsscenes
from oracle import camera as ocam
from oracle import pipeline
from tests._parity import assert_image

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
def scenes(P):
    a = gsscenes.make_scene("tiny", n=6000)
    b = gsscenes.make_scene("iso1m", n=4000, G=96)
    return [a, b], [P.Params.from_numpy(a.params), P.Params.from_numpy(b.params)]


def _requests(P, n=24, seed=0):
    rng = np.random.default_rng(seed)
    sizes = [(96, 96), (128, 96), (160, 160), (64, 80)]
    reqs = []
    for i in range(n):
        W, H = sizes[rng.integers(0, len(sizes))]
        d = ocam.to_float32(ocam.orbit_cameras(16, 2.5, 60.0, W, H)[rng.integers(0, 16)])
        reqs.append((int(rng.integers(0, 2)), d, P.camera_from_dict(d)))
    return reqs


def test_results_same_alone_and_in_the_mix(P, ctx, scenes):
    _, params = scenes
    reqs = _requests(P)
    alone = []
    for sid, _, cam in reqs:
        imgs, fr = P.render_fwd(ctx, params[sid], [cam])
        alone.append(imgs[0])
    torch.cuda.synchronize()
    srv = P.Server(ctx, n_slots=3, max_batch_views=4)
    ids = [srv.add_scene(p) for p in params]
    tickets = [srv.submit(ids[sid], cam) for sid, _, cam in reqs]
    for t, out in tickets:
        srv.wait(t)
    torch.cuda.synchronize()
    st = srv.stats()
    assert st["completed"] == len(reqs) and st["batches"] <= len(reqs)
    assert st["mean_batch_views"] >= 1.0 and st["p50_ms"] <= st["p99_ms"]
    for (t, out), ref in zip(tickets, alone):
        assert torch.equal(out, ref)
    srv.close()


def test_served_image_matches_oracle(P, ctx, scenes):
    raw, params = scenes
    srv = P.Server(ctx, n_slots=2, max_batch_views=3)
    ids = [srv.add_scene(p) for p in params]
    reqs = _requests(P, n=6, seed=1)
    tickets = [srv.submit(ids[sid], cam) for sid, _, cam in reqs]
    srv.drain()
    torch.cuda.synchronize()
    for (sid, d, _), (t, out) in zip(reqs, tickets):
        fw = pipeline.forward_view(raw[sid].params, d, 16)
        assert_image(fw, out.cpu().numpy())
    srv.close()


def test_memory_admission_defers_and_stays_correct(P, ctx, scenes):
    _, params = scenes
    reqs = _requests(P, n=16, seed=2)
    srv = P.Server(ctx, n_slots=4, max_batch_views=2, mem_budget=1)
    ids = [srv.add_scene(p) for p in params]
    tickets = [srv.submit(ids[sid], cam) for sid, _, cam in reqs]
    srv.drain()
    torch.cuda.synchronize()
    st = srv.stats()
    assert st["completed"] == len(reqs)
    assert st["deferred"] > 0           # batches waited for memory
    for (sid, _, cam), (t, out) in zip(reqs, tickets):
        imgs, _ = P.render_fwd(ctx, params[sid], [cam])
        torch.cuda.synchronize()
        assert torch.equal(out, imgs[0])
    srv.close()


def test_invalid_requests_are_rejected(P, ctx, scenes):
    _, params = scenes
    srv = P.Server(ctx, n_slots=1, max_batch_views=1, max_queue=2)
    sid = srv.add_scene(params[0])
    cam = P.camera(np.eye(3), [0, 0, 3], 50, 50, 16, 16, 32, 32)
    with pytest.raises(P.IsogsError):
        srv.submit(sid + 5, cam)
    t, out = srv.submit(sid, cam)
    srv.wait(t)
    with pytest.raises(P.IsogsError):
        srv.wait(t)                      # already collected
    srv.close()


def test_multi_scene_forward_matches_single_scene_and_oracle(P, ctx, scenes):
    """Views of two scenes (interleaved, mixed sizes) in one forward: every view
    bit-identical to rendering it alone, and within the image bar of the oracle;
    the persistent longest-first form gives the same images."""
    raw, params = scenes
    reqs = _requests(P, n=7, seed=5)
    sids = [sid for sid, _, _ in reqs]
    assert len(set(sids)) == 2
    cams = [cam for _, _, cam in reqs]
    outs = {}
    for flags in (0, P.PERSISTENT | P.LONGEST_FIRST):
        imgs, fr = P.render_fwd_multi(ctx, [params[s] for s in sids], cams, flags=flags)
        torch.cuda.synchronize()
        outs[flags] = [i.clone() for i in imgs]
        with pytest.raises(P.IsogsError):          # forward only
            P.render_bwd(ctx, fr, params[0], [torch.zeros_like(i) for i in imgs])
        with pytest.raises(P.IsogsError):
            fr.export("screen_grads")
        fr.release()
    for k, (sid, d, cam) in enumerate(reqs):
        alone, fr = P.render_fwd(ctx, params[sid], [cam])
        torch.cuda.synchronize()
        assert torch.equal(outs[0][k], alone[0])
        assert torch.equal(outs[P.PERSISTENT | P.LONGEST_FIRST][k], alone[0])
        fr.release()
        if k < 3:
            assert_image(pipeline.forward_view(raw[sid].params, d, 16), outs[0][k].cpu().numpy())


def test_server_batches_across_scenes(P, ctx, scenes):
    """Requests of different scenes submitted together land in shared batches."""
    _, params = scenes
    reqs = _requests(P, n=12, seed=6)
    srv = P.Server(ctx, n_slots=1, max_batch_views=6)
    ids = [srv.add_scene(p) for p in params]
    tickets = [srv.submit(ids[sid], cam) for sid, _, cam in reqs]
    srv.drain()
    torch.cuda.synchronize()
    st = srv.stats()
    assert st["completed"] == 12 and st["mean_batch_views"] > 1.0
    for (sid, _, cam), (t, out) in zip(reqs, tickets):
        imgs, fr = P.render_fwd(ctx, params[sid], [cam])
        torch.cuda.synchronize()
        assert torch.equal(out, imgs[0])
        fr.release()
    srv.close()
