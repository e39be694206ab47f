"""Benchmark of the rasterizer's training step on one MI355X.

Workload: the 4M-Gaussian scene (seeded 1024^3 blob + spectral-noise field,
isosurface points, SH degree 3, log-scales log(h) +- 0.5, random rotations),
trained against ray-cast isosurface targets.  Two forms of the same step:

* batched: 4 views per step (2 x 2048^2 + 2 x 1536^2) in one render call
  (one projection over all views, one sort, one compositing launch), loss
  gradient, backward;
* plain: one 2048^2 view per step and per launch.

fwd+bwd = projection .. backward (loss gradient included, Adam excluded);
the Adam step over all 4M Gaussians is timed beside it.  Inputs are resident
in HBM before the timed region.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "fwd+bwd Mpix/s @4M Gaussians 2048^2 (plain vs batched); serve p50/p99 ms"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3        # published vector peak (packed FP32)
FP32_NONPACKED_TFLOPS = 78.6    # 256 CUs x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz: no packed FP32
# algorithmic FLOP per (pixel, list position up to the pixel's last contributor): the
# forward's offset, quadratic form, exponential, alpha and transmittance update and
# colour sum (about 20, the exponential counted once), the backward 2.5 times that
FLOP_PAIR_FWD = 20
FLOP_PAIR_BWD = 50
# HBM bytes per launch of a kernel, from calibrated rocprofv3 FETCH_SIZE / WRITE_SIZE runs
# (profiles/hbm_traffic_kingsnake4m.md), one entry per measured launch configuration and
# valid only while the kernel source is unchanged: when the source hash no longer matches,
# or the timed configuration was not measured, the figure is null.
MEASURED_TRAFFIC = [
    {"kernel": "blend_bwd", "views": 4, "tile": 16, "lds_depth": 256, "flags": 3,
     "source": "paper_2509_05216_amd/csrc/blend.hip",
     "sha256": "5d593090c3691b52f4876bd4eefe434331da63c566c5787084f1d76af20f5965",
     "read_bytes": 3174.1e6, "write_bytes": 933.9e6},
]


def measured_traffic(kernel, views, render):
    import hashlib
    for m in MEASURED_TRAFFIC:
        if (m["kernel"], m["views"], m["tile"], m["lds_depth"], m["flags"]) != (
                kernel, views, render["tile"], render["lds_depth"], render["flags"]):
            continue
        with open(os.path.join(ROOT, m["source"]), "rb") as fh:
            if hashlib.sha256(fh.read()).hexdigest() != m["sha256"]:
                return None
        return round(m["read_bytes"] + m["write_bytes"])
    return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=None, help="Gaussian count override (smaller runs)")
    ap.add_argument("--grid", type=int, default=None, help="field grid override")
    ap.add_argument("--tile", type=int, default=16)
    ap.add_argument("--lds-depth", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--wide", action="store_true",
                    help="also time the 4M scene with log-scales U(-5,-3) (splat-size sensitivity; "
                         "about a minute)")
    ap.add_argument("--only", choices=["all", "batched", "plain"], default="all")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-train", action="store_true", help="skip the 1M-Gaussian training run")
    ap.add_argument("--no-c3", action="store_true", help="skip the in-situ 18M-Gaussian 4096^2 step")
    ap.add_argument("--cpu-c1", action="store_true",
                    help="also run the oracle over one whole 1024^2 view of the 1M scene (minutes)")
    ap.add_argument("--train-iters", type=int, default=500)
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--workload", choices=["kingsnake4m", "miranda18m"], default="kingsnake4m",
                    help="kingsnake4m: 4M Gaussians, 2x2048^2 + 2x1536^2 batched and 2048^2 plain "
                         "(the headline); miranda18m: 18M Gaussians, a batch of two 4096^2 views")
    ap.add_argument("--no-graph", action="store_true",
                    help="skip the graph-captured forms (e.g. for counter collection)")
    ap.add_argument("--config", default=None,
                    help="TILE,LDS_DEPTH,FLAGS for the batched form instead of autotuning")
    return ap.parse_args()


def make_targets(scene, cams_d, coarse=128):
    """Ray-cast the field at coarse resolution and upsample (nearest) per view."""
    import gsscenes
    out = []
    for c in cams_d:
        W, H = c["width"], c["height"]
        s = W // coarse
        small = gsscenes.raycast(scene.field, c["R"], c["t"], c["fx"] / s, c["fy"] / s,
                                 c["cx"] / s, c["cy"] / s, W // s, H // s, step=0.02)
        out.append(np.ascontiguousarray(np.repeat(np.repeat(small, s, 1), s, 2)))
    return out


def event_times(torch, steps):
    """HIP events (on torch's current stream, the stream every call here uses) that
    bracket each of `steps` steps."""
    return [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]


def step_ms(ev, wall_ms, steps):
    """Median and mean of the per-step event intervals, and the wall-clock mean."""
    per = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    return {"median": float(np.median(per)), "mean_event": float(np.mean(per)),
            "min": float(np.min(per)), "max": float(np.max(per)), "mean_wall": wall_ms / steps}


def run_graph(P, ctx, params, cams, targets, steps, warmup, render, with_adam, torch):
    """Time `steps` replays of the captured step; returns per-step ms and records."""
    g = P.StepGraph(ctx, params, cams, targets, with_adam=with_adam, render=render)
    for _ in range(warmup):
        g.run()
    torch.cuda.synchronize()
    ev = event_times(torch, steps)
    t0 = time.perf_counter()
    ev[0].record()
    for i in range(steps):
        g.launch()
        ev[i + 1].record()
    over, rec = g.sync()
    torch.cuda.synchronize()
    t = step_ms(ev, (time.perf_counter() - t0) * 1e3, steps)
    if over:
        raise RuntimeError("record capacity overflowed during the timed replays")
    loss = float(g.loss.item())
    cap, _ = g.info()
    g.close()
    return t, rec, cap, loss


def wide_scales(P, ctx, params, cams, targets, steps, warmup, torch):
    """The 4M scene with every log-scale drawn from U(-5, -3) instead of log(h) +- 0.5
    (seeded; splats of several to tens of pixels, far longer tile lists): the batched
    step timed as graph replays for a few render options (no autotuning: one step takes
    hundreds of milliseconds), for the sensitivity of the step to splat size."""
    rng = np.random.default_rng(20_000)
    n = params.n
    wide = P.Params(params.means, torch.tensor(rng.uniform(-5.0, -3.0, (3, n)).astype(np.float32),
                                               device="cuda"),
                    params.quats, params.opacity_logits, params.sh, params.sh_degree)
    pixels = sum(c.width * c.height for c in cams)
    frame = P.Frame()
    images = [torch.empty((3, c.height, c.width), device="cuda") for c in cams]
    P.render_fwd(ctx, wide, cams, images, frame=frame)
    st = frame.stats()
    frame.release()
    log(f"wide-scale 4M scene: K={st['n_records']}, {st['n_visible']} visible entries")
    rows = []
    # tile 16 and 32 (at tile 8 the records pass three billion)
    for render in ({"tile": 16, "lds_depth": 256, "flags": 3}, {"tile": 32, "lds_depth": 256, "flags": 3}):
        try:
            gtm, rec, cap, gloss = run_graph(P, ctx, wide, cams, targets, steps, warmup, render,
                                             False, torch)
        except P.IsogsError as e:  # e.g. more records than a frame holds at small tiles
            rows.append({**render, "error": str(e)})
            log(f"wide-scale 4M step {render}: {e}")
            continue
        ms = gtm["median"]
        rows.append({**render, "ms_per_step": round(ms, 3),
                     "mpix_per_s": round(pixels / (ms * 1e-3) / 1e6, 3), "loss": round(gloss, 6)})
        log(f"wide-scale 4M step {render}: {ms:.1f} ms")
    best = min((r for r in rows if "ms_per_step" in r), key=lambda r: r["ms_per_step"])
    return {"ms_per_step": best["ms_per_step"], "mpix_per_s": best["mpix_per_s"],
            "records_K": st["n_records"], "visible": st["n_visible"],
            "tiles_per_entry": round(st["n_records"] / max(st["n_visible"], 1), 3),
            "options": rows,
            "workload": ("kingsnake4m points, log-scales U(-5,-3) per axis (seeded), SH3; the "
                         "headline's 4 views per step, one hipGraph replay per step, the faster "
                         "of tile 16 and tile 32 (persistent longest-first, LDS depth 256)")}


def run_steps(P, ctx, params, cams, targets, steps, warmup, tile, depth, torch, flags=0):
    """Time `steps` fwd+bwd steps; returns per-step ms, stage totals and a frame."""
    frame = P.Frame()
    images = [torch.empty((3, c.height, c.width), device="cuda") for c in cams]
    grads = params.zeros_like()

    def one():
        P.render_fwd(ctx, params, cams, images, tile=tile, lds_depth=depth, flags=flags,
                     frame=frame)
        loss, dl = P.loss_grad(ctx, images, targets, cams)
        P.render_bwd(ctx, frame, params, dl, grads)
        return loss

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    ctx.set_timing(True)
    ev = event_times(torch, steps)
    t0 = time.perf_counter()
    ev[0].record()
    for i in range(steps):
        loss = one()
        ev[i + 1].record()
    torch.cuda.synchronize()
    t = step_ms(ev, (time.perf_counter() - t0) * 1e3, steps)
    stages = ctx.stage_times()
    ctx.set_timing(False)
    return t, stages, frame, float(loss.item()), images, grads


def serve_run(P, ctx, scene_params, requests, arrivals, outs, warm_cams, torch, **server_opts):
    """Replay the arrival process against a server; returns its statistics."""
    srv = P.Server(ctx, **server_opts)
    ids = [srv.add_scene(p) for p in scene_params]
    # warm-up: a burst over every (scene, size) so every slot has sized its buffers
    warm = []
    for _ in range(server_opts.get("n_slots", 1)):
        for sid in ids:
            for size, ring in outs.items():
                warm.append(srv.submit(sid, warm_cams[size], ring[len(warm) % len(ring)][0])[0])
    for t in warm:
        srv.wait(t)
    srv.drain()
    srv.reset_stats()
    busy = {size: [None] * len(ring) for size, ring in outs.items()}
    nxt = {size: 0 for size in outs}
    t0 = time.perf_counter()
    for (sid, cams), at in zip(requests, arrivals):
        ((size, cam),) = cams.items()
        k = nxt[size] % len(outs[size])
        nxt[size] += 1
        if busy[size][k] is not None:          # output buffer still in use
            srv.wait(busy[size][k])
        delay = t0 + at - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        t, _ = srv.submit(ids[sid], cam, outs[size][k][0])
        busy[size][k] = t
    srv.drain()
    st = srv.stats()
    srv.close()
    return st


def train_for_serving(P, ctx, params, field_name, torch, iters=200, G=256, res=512, n_views=32,
                      seed=7):
    """A copy of `params` trained for `iters` iterations (L1 + SSIM, no density control)
    on ray-cast 512^2 orbit views of its field's volume; returns it and the loss before /
    after (the mean over the first and last ten iterations)."""
    import gsscenes
    from paper_2509_05216_amd import iso
    from paper_2509_05216_amd.train import Trainer
    field, _ = gsscenes.make_field(field_name)
    vol = iso.Volume(gsscenes.sample_volume(field, G, device="cuda"))
    cams = P.orbit_cameras(n_views, 2.5, 60.0, res, res)
    targets = [t.clone() for t in iso.raycast(ctx, vol, cams[:16], 0.5, 2.0 / (G - 1))]
    targets += [t.clone() for t in iso.raycast(ctx, vol, cams[16:], 0.5, 2.0 / (G - 1))]
    del vol
    p = P.Params(*(t.clone() for t in params.tensors()), params.sh_degree)
    tr = Trainer(ctx, p, cams, targets, densify=False, seed=seed)
    hist = tr.run(iters, log_every=1)
    tr.close()
    first = float(np.mean([h["loss"] for h in hist[:10]]))
    last = float(np.mean([h["loss"] for h in hist[-10:]]))
    return tr.params, round(first, 5), round(last, 5)


def serve_bench(P, ctx, params4m, torch, n_requests=2000, rate=200.0):
    """Three resident scenes (100k, 1M, 4M Gaussians, SH3), each first trained for 200
    iterations on ray-cast views of its field; Poisson arrivals; sizes 512^2 / 1024^2 /
    2048^2; servers batching across scenes and resolutions (4, 2 and 1 slots, up to 8
    views per batch) vs serial per-request rendering."""
    import gsscenes
    t0 = time.perf_counter()
    s100k = gsscenes.make_scene("serve")
    s1m = gsscenes.make_scene("iso1m")
    raw = [(P.Params.from_numpy(s100k.params), "serve"), (P.Params.from_numpy(s1m.params), "iso1m"),
           (params4m, "kingsnake4m")]
    log(f"serve scenes in {time.perf_counter() - t0:.1f}s")
    t0 = time.perf_counter()
    scenes, training = [], []
    for prm, fname in raw:
        tp, l0, l1 = train_for_serving(P, ctx, prm, fname, torch)
        scenes.append(tp)
        training.append({"scene": fname, "gaussians": prm.n, "iterations": 200,
                         "loss_first10": l0, "loss_last10": l1})
    del raw
    log(f"serve scenes trained in {time.perf_counter() - t0:.1f}s: {training}")
    arrivals, u_scene, u_size = gsscenes.arrival_times(rate, n_requests)
    sizes = [512, 1024, 2048]
    orbit = {s: P.orbit_cameras(64, 2.5, 60.0, s, s) for s in sizes}
    requests = []
    for i in range(n_requests):
        sid = min(int(u_scene[i] * 3), 2)
        s = sizes[min(int(u_size[i] * 3), 2)]
        requests.append((sid, {s: orbit[s][(i * 37) % 64]}))
    outs = {s: [(torch.empty((3, s, s), device="cuda"),) for _ in range(32)] for s in sizes}
    warm = {s: orbit[s][1] for s in sizes}
    pix = sum(next(iter(c)) ** 2 for _, c in requests)
    res = {"training": training}
    for name, opts in (("batched", dict(n_slots=4, max_batch_views=8)),
                       ("batched_2slots", dict(n_slots=2, max_batch_views=8)),
                       ("batched_1slot", dict(n_slots=1, max_batch_views=8)),
                       ("serial", dict(n_slots=1, max_batch_views=1))):
        st = serve_run(P, ctx, scenes, requests, arrivals, outs, warm, torch, **opts)
        res[name] = {"p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3),
                     "mean_ms": round(st["mean_ms"], 3), "max_ms": round(st["max_ms"], 3),
                     "mpix_per_s": round(st["mpix_per_s"], 1), "completed": st["completed"],
                     "batches": st["batches"], "mean_batch_views": round(st["mean_batch_views"], 2),
                     "deferred": st["deferred"], "peak_scratch_bytes": st["peak_bytes"],
                     "slots": opts["n_slots"], "max_batch_views": opts["max_batch_views"]}
        log(f"serve {name}: p50 {st['p50_ms']:.2f} ms, p99 {st['p99_ms']:.2f} ms, "
            f"{st['mpix_per_s']:.0f} Mpix/s, {st['mean_batch_views']:.2f} views per batch")
    # saturation: the same requests submitted at once (offered load far above capacity)
    burst = [0.0] * min(600, n_requests)
    for name, opts in (("batched_saturated", dict(n_slots=4, max_batch_views=8)),
                       ("serial_saturated", dict(n_slots=1, max_batch_views=1))):
        st = serve_run(P, ctx, scenes, requests[:len(burst)], burst, outs, warm, torch, **opts)
        res[name] = {"mpix_per_s": round(st["mpix_per_s"], 1), "p50_ms": round(st["p50_ms"], 3),
                     "p99_ms": round(st["p99_ms"], 3),
                     "mean_batch_views": round(st["mean_batch_views"], 2)}
        log(f"serve {name}: {st['mpix_per_s']:.0f} Mpix/s")
    res["workload"] = (f"{n_requests} requests, Poisson {rate:.0f}/s, scenes 100k/1M/4M "
                       f"Gaussians (SH3, trained 200 iterations) resident, sizes "
                       f"512^2/1024^2/2048^2 uniform, batches across scenes and sizes, "
                       f"{pix / 1e6:.0f} Mpix total")
    del scenes
    return res


def train_c1(P, ctx, torch, iters=500, n_target=1_000_000, G=512, res=1024, n_views=128,
             n_held=16, seed=1001):
    """The 1M-Gaussian training run, in situ on the device: the seeded 512^3 blob +
    noise volume, its isosurface points (subsampled to about 1M by the keep rule),
    Gaussians initialised from them (SH3 N(0, 0.1), log-scales U(-5, -3), random
    rotations, opacity logit 0.1), ray-cast targets of a 128-view 1024^2 orbit,
    500 iterations of L1 + SSIM with density control every 100 iterations from
    iteration 200 to 400; PSNR / SSIM on 16 held-out views (another orbit) every 100."""
    import gsscenes
    from paper_2509_05216_amd import iso
    from paper_2509_05216_amd.train import Schedule, Trainer
    out = {}
    t0 = time.perf_counter()
    field, _ = gsscenes.make_field("iso1m")
    vol = iso.Volume(gsscenes.sample_volume(field, G, device="cuda"))
    torch.cuda.synchronize()
    out["volume_s"] = round(time.perf_counter() - t0, 2)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record()
    m = iso.count(ctx, vol)
    ev[1].record()
    pts = iso.extract(ctx, vol, 0.5, min(1.0, n_target / m), seed)
    params = P.init_from_points(ctx, pts.contiguous(), 3, log_scale_range=(-5.0, -3.0),
                                random_quats=True, opacity_logit=0.1, sh_std=0.1, seed=seed)
    ev[2].record()
    h = 2.0 / (G - 1)
    cams = P.orbit_cameras(n_views, 2.5, 60.0, res, res)
    held = P.orbit_cameras(n_held + 1, 2.5, 60.0, res, res)[1:]
    targets = []
    for i in range(0, n_views, 16):
        targets += iso.raycast(ctx, vol, cams[i:i + 16], 0.5, h)
    refs = iso.raycast(ctx, vol, held, 0.5, h)
    ev[3].record()
    torch.cuda.synchronize()
    out.update(crossings=m, gaussians=pts.shape[1],
               extract_ms=round(ev[0].elapsed_time(ev[1]) + ev[1].elapsed_time(ev[2]), 3),
               raycast_ms=round(ev[2].elapsed_time(ev[3]), 2),
               raycast_mpix_per_s=round((n_views + n_held) * res * res /
                                        (ev[2].elapsed_time(ev[3]) * 1e-3) / 1e6, 1))
    del vol
    sched = Schedule(densify_from=100, densify_until=450, densify_interval=100,
                     opacity_reset_interval=3000, extent=2.5, seed=seed)
    tr = Trainer(ctx, params, cams, targets, schedule=sched, seed=seed)
    curve = [{"it": 0, **{k: round(v, 4) for k, v in tr.evaluate(held, refs).items()
                          if k != "per_view"}}]
    t1 = time.perf_counter()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    loss_curve = []
    train_ms = 0.0
    for blk in range(iters // 100):
        e0.record()
        tr.run(100, log_every=10)
        e1.record()
        torch.cuda.synchronize()
        train_ms += e0.elapsed_time(e1)
        ev_ = tr.evaluate(held, refs)
        curve.append({"it": tr.it, "n": tr.params.n,
                      **{k: round(v, 4) for k, v in ev_.items() if k != "per_view"}})
    out["wall_s"] = round(time.perf_counter() - t1, 2)
    out["ms_per_iteration"] = round(train_ms / iters, 3)
    out["loss_every_10"] = [round(r["loss"], 5) for r in tr.history if "loss" in r
                            and r["it"] % 10 == 0]
    out["densify"] = [{"it": r["it"], **{k: r["densify"][k] for k in ("n_in", "n_out", "cloned",
                                                                      "split", "pruned")}}
                      for r in tr.history if "densify" in r]
    out["held_out"] = curve
    out["workload"] = (f"seeded {G}^3 blob+noise volume on the device, {pts.shape[1]} Gaussians "
                       f"from its isosurface, {n_views}-view {res}^2 orbit (ray-cast targets), "
                       f"{iters} iterations L1+SSIM, density control at 200/300/400, "
                       f"{n_held} held-out views")
    tr.close()
    return out


def miranda_insitu(P, torch, steps, warmup, n_target=18_000_000, G=2048, res=4096, seed=1003):
    """The 18M-Gaussian workload built in situ on the device and timed: the seeded
    2048^3 mixing-layer volume (34 GB, slab by slab on the device), its isosurface
    points subsampled to about 18M by the keep rule, Gaussians initialised from them
    (log-scales log h +- 0.5, random rotations, SH3 N(0, 0.1), opacity logit 0.1),
    ray-cast targets of two 4096^2 orbit views; then the batched step (autotuned,
    captured in a graph) on its own context, with the peak device memory."""
    import gsscenes
    from paper_2509_05216_amd import iso
    out = {}
    ctx = P.Context(0)
    t0 = time.perf_counter()
    field, _ = gsscenes.make_field("miranda18m")
    vol = iso.Volume(gsscenes.sample_volume(field, G, device="cuda", progress=log))
    torch.cuda.synchronize()
    out["volume_s"] = round(time.perf_counter() - t0, 2)
    out["volume_bytes"] = vol.values.numel() * 4
    h = 2.0 / (G - 1)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record()
    m = iso.count(ctx, vol)
    pts = iso.extract(ctx, vol, 0.5, min(1.0, n_target / m), seed)
    params = P.init_from_points(ctx, pts.contiguous(), 3, log_scale=float(np.log(h)),
                                log_scale_jitter=0.5, random_quats=True, opacity_logit=0.1,
                                sh_std=0.1, seed=seed)
    ev[1].record()
    all_cams = P.orbit_cameras(16, 2.5, 60.0, res, res)
    cams = [all_cams[0], all_cams[8]]
    targets = [t.clone() for t in iso.raycast(ctx, vol, cams, 0.5, 2 * h)]
    ev[2].record()
    torch.cuda.synchronize()
    out.update(crossings=m, gaussians=params.n,
               extract_init_ms=round(ev[0].elapsed_time(ev[1]), 2),
               raycast_ms=round(ev[1].elapsed_time(ev[2]), 2))
    del vol, pts
    torch.cuda.empty_cache()
    torch.cuda.reset_peak_memory_stats()
    log(f"18M scene in situ: {params.n} Gaussians from {m} crossings, "
        f"{time.perf_counter() - t0:.1f}s")
    best, table = P.autotune(ctx, params, cams, reps=3, use_cache=False, cache=None)
    gtm, rec, cap, gloss = run_graph(P, ctx, params, cams, targets, steps, warmup, best, False,
                                     torch)
    pa = P.Params(*(t.clone() for t in params.tensors()), params.sh_degree)
    atm, _, _, _ = run_graph(P, ctx, pa, cams, targets, steps, warmup, best, True, torch)
    del pa
    lib_now, lib_peak = ctx.memory()
    free_b, total_b = torch.cuda.mem_get_info()
    pix = 2 * res * res
    out.update(
        ms_per_step=round(gtm["median"], 3), ms_stats={k: round(v, 4) for k, v in gtm.items()},
        mpix_per_s=round(pix / (gtm["median"] * 1e-3) / 1e6, 3),
        gaussians_per_s=round(params.n * 2 / (gtm["median"] * 1e-3), 1),
        ms_with_adam=round(atm["median"], 3), records_K=rec, capacity=cap, loss=round(gloss, 6),
        autotune={"best": best, "table": sorted(table, key=lambda r: r["ms"])[:4]},
        memory={"library_peak_bytes": lib_peak, "torch_peak_bytes": torch.cuda.max_memory_allocated(),
                "device_used_bytes": total_b - free_b, "device_total_bytes": total_b},
        workload=(f"miranda18m in situ: {params.n} Gaussians from the isosurface of a seeded "
                  f"{G}^3 mixing-layer volume on the device, SH3, a batch of two {res}^2 views, "
                  f"one hipGraph replay per step (tuned {best})"))
    ctx.close()
    return out


def frame_counts(frame, n, torch):
    st = frame.stats()
    nc = frame.export("n_contrib").to(torch.int64)
    pairs = int(nc.sum().item())
    rects = frame.export("rects").view(-1, 2).cpu().numpy().view(np.uint32)
    x0, x1 = rects[:, 0] & 0xFFFF, rects[:, 1] & 0xFFFF
    visible = int((x1 >= x0).sum())
    return st, pairs, visible


def algorithmic(stage, n, views, visible, K, pixels, pairs):
    """(bytes, flops) per launch-set of a stage, per the algorithmic model."""
    vn = n * views
    model = {
        "project": (12 * n + 224 * visible + 48 * visible, 0),
        "depth_sort": (16 * vn, 0),
        "scan": (12 * vn, 0),
        "emit": (24 * visible + 8 * K, 0),
        "tile_sort": (16 * K, 0),
        "ranges": (8 * K, 0),
        "blend_fwd": (40 * K + 20 * pixels, FLOP_PAIR_FWD * pairs),
        "loss": (36 * pixels, 0),
        "blend_bwd": (40 * K + 20 * pixels + 36 * visible, FLOP_PAIR_BWD * pairs),
        "project_bwd": (516 * visible, 0),
    }
    return model.get(stage, (0, 0))


def roofline(stages, steps, n, views, visible, K, pixels, pairs, traffic=None):
    tot = {k: v[0] for k, v in stages.items() if v[1] > 0}
    dom = max(tot, key=tot.get)
    launches = stages[dom][1]
    avg_ms = stages[dom][0] / max(launches, 1)
    byts, flops = algorithmic(dom, n, views, visible, K, pixels, pairs)
    if flops > 0:
        ach = flops / (avg_ms * 1e-3) / 1e12
        return dom, {"bound": "alu", "achieved": round(ach, 3), "peak": FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(ach / FP32_PEAK_TFLOPS, 4),
                     "peak_nonpacked": FP32_NONPACKED_TFLOPS,
                     "frac_nonpacked": round(ach / FP32_NONPACKED_TFLOPS, 4),
                     "flop_per_pair": FLOP_PAIR_BWD if dom == "blend_bwd" else FLOP_PAIR_FWD,
                     "pairs": pairs,
                     "traffic": traffic, "kernel": dom, "avg_ms": round(avg_ms, 4),
                     "algorithmic_flop": flops, "algorithmic_bytes": byts,
                     "hbm_GBps_algorithmic": round(byts / (avg_ms * 1e-3) / 1e9, 1)}
    ach = byts / (avg_ms * 1e-3) / 1e9
    return dom, {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
                 "avg_ms": round(avg_ms, 4), "algorithmic_bytes": byts}


# ---------------------------------------------------------------- CPU baseline
# The oracle (float64 numpy, as it stands) on the host's cores: per-Gaussian
# stages split into chunks over threads (numpy releases the GIL in its loops),
# per-tile stages and whole views over forked worker processes that inherit the
# projection.  BLAS stays single-threaded inside each worker.
_CPU = {}


def _cpu_cores():
    return max(1, min(len(os.sched_getaffinity(0)), 16))


def _chunked(fn, n, cores):
    """fn(a, b) over `cores` contiguous chunks of range(n), on threads."""
    import concurrent.futures as cf
    bounds = np.linspace(0, n, cores + 1).astype(np.int64)
    with cf.ThreadPoolExecutor(max_workers=cores) as ex:
        return list(ex.map(lambda i: fn(int(bounds[i]), int(bounds[i + 1])), range(cores)))


def _slice_params(params, a, b):
    return {k: (v[..., a:b] if isinstance(v, np.ndarray) else v) for k, v in params.items()}


def _merge(parts):
    out = {}
    for k, v in parts[0].items():
        if isinstance(v, np.ndarray) and v.ndim >= 1:
            out[k] = np.concatenate([p[k] for p in parts], axis=v.ndim - 1)
        else:
            out[k] = v
    return out


def _tile_worker(tiles):
    from oracle import blend
    pr, W, H, tile, target = _CPU["pr"], _CPU["W"], _CPU["H"], _CPU["tile"], _CPU["target"]
    tx = (W + tile - 1) // tile
    rect, touched, bits = pr["rect"], pr["touched"], pr["depth32"].view(np.uint32)
    n = pr["m"].shape[1]
    acc = dict(m=np.zeros((2, n)), conic=np.zeros((3, n)), opacity=np.zeros(n),
               rgb=np.zeros((3, n)))
    for t in tiles:
        x, y = t % tx, t // tx
        members = np.nonzero(touched & (rect[0] <= x) & (x <= rect[2]) & (rect[1] <= y)
                             & (y <= rect[3]))[0]
        g = members[np.argsort(bits[members], kind="stable")]
        X, Y = blend.tile_pixels(x, y, tile, W, H)
        blend.composite_tile(pr, g, X + 0.5, Y + 0.5, (0, 0, 0))
        d = np.asarray(target[:, Y, X], np.float64) * 1e-3
        blend.backward_tile(pr, g, X + 0.5, Y + 0.5, d, (0, 0, 0), acc)
    return acc


def _loss_worker(cells):
    from oracle import loss as oloss
    target, c = _CPU["target"], _CPU["cell"]
    for (y0, x0) in cells:
        crop = np.asarray(target[:, y0:y0 + c, x0:x0 + c], np.float64)
        oloss.view_loss(crop * 0.9, crop)
        oloss.view_loss_grad(crop * 0.9, crop)
    return len(cells)


def _view_worker(k):
    from oracle import loss as oloss
    from oracle import pipeline
    params, cams, targets = _CPU["params"], _CPU["cams"], _CPU["targets"]
    f = pipeline.forward_view(params, cams[k], 16)
    L = oloss.view_loss(f["image"], targets[k]) / len(cams)
    d = oloss.view_loss_grad(f["image"], targets[k]) / len(cams)
    _, g = pipeline.backward_view(params, cams[k], f, d)
    return L, g


def cpu_c0_full(cores):
    """The whole oracle fwd + loss + bwd of the 10k-Gaussian scene over its 8 views of
    256^2 (one view per worker process)."""
    import multiprocessing as mp

    import gsscenes
    from oracle import camera as ocam
    scene = gsscenes.make_scene("tiny")
    cams = [ocam.to_float32(c) for c in ocam.orbit_cameras(8, 2.5, 60.0, 256, 256)]
    targets = make_targets(scene, cams, coarse=128)
    _CPU.update(params=scene.params, cams=cams, targets=targets)
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(min(cores, len(cams))) as pool:
        res = pool.map(_view_worker, range(len(cams)))
    dt = time.perf_counter() - t0
    _CPU.clear()
    return {"mpix_per_s": round(8 * 256 * 256 / dt / 1e6, 6), "seconds": round(dt, 2),
            "loss": round(float(sum(r[0] for r in res)), 6),
            "processes": min(cores, len(cams)),
            "sample": "full run: 10k Gaussians, 8 views of 256^2, fwd + L1/SSIM + bwd"}


def cpu_c1_view(cores):
    """The oracle's fwd + loss + bwd of one whole 1024^2 view of the 1M-Gaussian scene on
    the host's cores (every tile; no sampling)."""
    import gsscenes
    from oracle import camera as ocam
    scene = gsscenes.make_scene("iso1m")
    cam = ocam.to_float32(ocam.orbit_cameras(128, 2.5, 60.0, 1024, 1024)[0])
    target = make_targets(scene, [cam], coarse=128)[0]
    r = cpu_baseline(scene, cam, target, tile_frac=1.0, with_c0=False)
    return {"mpix_per_s": r["value"], "seconds": r["seconds"], "stages_s": r["stages_s"],
            "cores": r["cores"],
            "sample": "full run: 1M Gaussians (SH3), one 1024^2 view, every tile, fwd + L1/SSIM + bwd"}


def cpu_baseline(scene, cam_d, target, tile_frac=1 / 64, tile=16, with_c0=True):
    """The oracle's fwd+bwd on one 2048^2 view of the 4M scene on the host's cores:
    projection and parameter backward on all Gaussians (threads over chunks),
    binning + compositing fwd/bwd on a seeded 1/64 of the tiles (processes), scaled
    by that sample's share of the total list length; the loss over the whole view;
    plus the full 10k-Gaussian 8-view run."""
    import multiprocessing as mp

    from threadpoolctl import threadpool_limits

    from oracle import backward as obwd
    from oracle import project
    cores = _cpu_cores()
    params = scene.params
    n = params["means"].shape[1]
    W, H = cam_d["width"], cam_d["height"]
    tx, ty = (W + tile - 1) // tile, (H + tile - 1) // tile
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        parts = _chunked(lambda a, b: project.project(_slice_params(params, a, b), cam_d, tile),
                         n, cores)
        pr = _merge(parts)
        t_proj = time.perf_counter() - t0
        log(f"oracle projection of {n} Gaussians: {t_proj:.1f}s on {cores} threads")
        rng = np.random.default_rng(1234)
        n_tiles = max(1, int(round(tx * ty * tile_frac)))
        sample = rng.choice(tx * ty, size=n_tiles, replace=False)
        rect, touched = pr["rect"], pr["touched"]
        cnt = np.zeros((ty + 1, tx + 1), np.int64)
        ids = np.nonzero(touched)[0]
        np.add.at(cnt, (rect[1, ids], rect[0, ids]), 1)
        np.add.at(cnt, (rect[1, ids], rect[2, ids] + 1), -1)
        np.add.at(cnt, (rect[3, ids] + 1, rect[0, ids]), -1)
        np.add.at(cnt, (rect[3, ids] + 1, rect[2, ids] + 1), 1)
        lens = np.cumsum(np.cumsum(cnt, 0), 1)[:ty, :tx].ravel()
        _CPU.update(pr=pr, W=W, H=H, tile=tile, target=target)
        t0 = time.perf_counter()
        with mp.get_context("fork").Pool(cores) as pool:
            accs = pool.map(_tile_worker, [list(c) for c in np.array_split(sample, cores)])
        t_tiles = time.perf_counter() - t0
        log(f"oracle compositing fwd/bwd of {n_tiles} tiles: {t_tiles:.1f}s on {cores} processes")
        _CPU.clear()
        acc = {k: sum(a[k] for a in accs) for k in accs[0]}
        share = lens[sample].sum() / max(lens.sum(), 1)
        t0 = time.perf_counter()
        bounds = np.linspace(0, n, cores + 1).astype(np.int64)
        _chunked(lambda a, b: obwd.param_grads(
            parts[int(np.searchsorted(bounds, a))], _slice_params(params, a, b), cam_d,
            {k: v[..., a:b] for k, v in acc.items()}), n, cores)
        t_pbwd = time.perf_counter() - t0
        # the loss and its gradient over the whole view, as 256^2 cells over the processes
        cells = [(y, x) for y in range(0, H, 256) for x in range(0, W, 256)]
        _CPU.update(target=target, cell=256)
        t0 = time.perf_counter()
        with mp.get_context("fork").Pool(cores) as pool:
            pool.map(_loss_worker, [cells[i::cores] for i in range(cores)])
        t_loss = time.perf_counter() - t0
        _CPU.clear()
    total = t_proj + t_pbwd + t_tiles / max(share, 1e-12) + t_loss
    c0 = cpu_c0_full(cores) if with_c0 else None
    return {"value": round(W * H / total / 1e6, 6), "unit": "Mpix/s", "cores": cores,
            "kind": "oracle",
            "sample": (f"one {W}x{H} view of the {n}-Gaussian scene, float64 numpy on {cores} "
                       f"cores: projection and parameter backward on all Gaussians ({cores} "
                       f"threads over chunks), binning + compositing fwd/bwd on {n_tiles} seeded "
                       f"tiles (1/64 of the view; {cores} processes) scaled by their "
                       f"{share:.4f} share of list length (estimate), L1+SSIM loss and gradient "
                       f"over the whole view as 256^2 cells ({cores} processes)"),
            "seconds": round(t_proj + t_tiles + t_pbwd + t_loss, 2),
            "est_seconds_full_view": round(total, 1),
            "stages_s": {"project": round(t_proj, 2), "tiles_sample": round(t_tiles, 2),
                         "param_bwd": round(t_pbwd, 2), "loss": round(t_loss, 2)},
            "c0_full": c0}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "split is not implemented here", file=sys.stderr)
        sys.exit(2)
    import torch

    import gsscenes
    import paper_2509_05216_amd as P

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    t0 = time.perf_counter()
    scene = gsscenes.make_scene(args.workload, n=args.n, G=args.grid, progress=log)
    n = scene.params["means"].shape[1]
    log(f"scene: {n} Gaussians in {time.perf_counter() - t0:.1f}s")
    ctx = P.Context(0)
    params = P.Params.from_numpy(scene.params)
    if args.workload == "miranda18m":
        sizes, stride = [4096, 4096], 8
        args.only = "batched"  # the 18M workload is the two-view batch only
        args.no_serve = True
    else:
        sizes, stride = [2048, 2048, 1536, 1536], 4
    all_cams = P.orbit_cameras(16, 2.5, 60.0, sizes[0], sizes[0])
    cams = []
    for i, s in enumerate(sizes):
        c = all_cams[i * stride]
        d = P.camera_to_dict(c)
        cams.append(P.camera(d["R"], d["t"], d["fx"] * s / sizes[0], d["fy"] * s / sizes[0],
                             s / 2, s / 2, s, s))
    cams_d = [P.camera_to_dict(c) for c in cams]
    t0 = time.perf_counter()
    targets_np = make_targets(scene, cams_d)
    targets = [torch.tensor(t, device="cuda") for t in targets_np]
    log(f"targets in {time.perf_counter() - t0:.1f}s")
    torch.cuda.synchronize()

    res = {}
    tune = None
    if args.only in ("all", "batched"):
        t0 = time.perf_counter()
        if args.config:
            tl, dp, fl = (int(x) for x in args.config.split(","))
            best = {"tile": tl, "lds_depth": dp, "flags": fl}
            tune = {"best": best, "fixed": True}
        else:
            best, table = P.autotune(ctx, params, cams, reps=5, use_cache=False, cache=None)
            tune = {"best": best, "seconds": round(time.perf_counter() - t0, 2),
                    "table": sorted(table, key=lambda r: r["ms"])[:6]}
        log(f"batched options: {best}")
        # eager run of the tuned configuration: per-stage HIP-event times
        tm, stages, frame, loss, _, _ = run_steps(P, ctx, params, cams, targets, args.steps,
                                                  args.warmup, best["tile"], best["lds_depth"],
                                                  torch, flags=best["flags"])
        ms = tm["median"]
        st, pairs, vis = frame_counts(frame, n, torch)
        res["batched"] = dict(ms=ms, timing=tm, stages=stages, K=st["n_records"], pixels=st["n_pixels"],
                              pairs=pairs, visible=vis, views=len(cams), loss=loss)
        log(f"batched (eager, tuned): {ms:.2f} ms/step, K={st['n_records']}, pairs={pairs}")
        frame.release()
    if args.only in ("all", "batched") and not args.no_graph:
        # the captured step: fwd+bwd, then fwd+bwd+Adam
        gtm, rec, cap, gloss = run_graph(P, ctx, params, cams, targets, args.steps, args.warmup,
                                         best, False, torch)
        gms = gtm["median"]
        res["batched_graph"] = dict(ms=gms, timing=gtm, K=rec, capacity=cap, pixels=st["n_pixels"],
                                    views=len(cams),
                                    loss=gloss, visible=vis, pairs=pairs, stages={})
        log(f"batched (graph): {gms:.2f} ms/step")
        pa = P.Params(*(t.clone() for t in params.tensors()), params.sh_degree)
        atm, _, _, _ = run_graph(P, ctx, pa, cams, targets, args.steps, args.warmup, best, True,
                                 torch)
        ams = atm["median"]
        res["batched_graph"]["ms_with_adam"] = ams
        del pa
        log(f"batched (graph + Adam): {ams:.2f} ms/step")
    if args.only in ("all", "plain"):
        tm, stages, frame, loss, _, _ = run_steps(P, ctx, params, cams[:1], targets[:1],
                                                  args.steps, args.warmup, args.tile,
                                                  args.lds_depth, torch)
        ms = tm["median"]
        st, pairs, vis = frame_counts(frame, n, torch)
        res["plain"] = dict(ms=ms, timing=tm, stages=stages, K=st["n_records"], pixels=st["n_pixels"],
                            pairs=pairs, visible=vis, views=1, loss=loss)
        log(f"plain: {ms:.2f} ms/step, K={st['n_records']}, pairs={pairs}")
        frame.release()
    # device memory of the training step (before the Adam and copy-probe legs allocate
    # their own buffers): the library's buffers (current and high-water), the caller's
    # tensors (torch's high-water mark) and the device's use as the HIP runtime reports it
    lib_now, lib_peak = ctx.memory()
    free_b, total_b = torch.cuda.mem_get_info()
    memory = {"library_bytes": lib_now, "library_peak_bytes": lib_peak,
              "torch_peak_bytes": torch.cuda.max_memory_allocated(),
              "device_used_bytes": total_b - free_b, "device_total_bytes": total_b}
    # Adam over all Gaussians, timed on its own
    grads = params.zeros_like()
    m, v = params.zeros_like(), params.zeros_like()
    for i in range(2):
        P.adam_step(ctx, params, grads, m, v, i + 1)
    torch.cuda.synchronize()
    ctx.set_timing(True)
    for i in range(args.steps):
        P.adam_step(ctx, params, grads, m, v, i + 3)
    torch.cuda.synchronize()
    adam_ms = ctx.stage_times()["adam"][0] / args.steps
    ctx.set_timing(False)
    nb = (scene.params["sh_degree"] + 1) ** 2 * 3 + 11
    adam_gbs = 28 * nb * n / (adam_ms * 1e-3) / 1e9
    # achievable HBM bandwidth: plain copy of 2 GiB (read + write)
    probe_bytes = 2 << 30
    src = torch.ones(probe_bytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    P.bw_probe(ctx, src, dst)
    torch.cuda.synchronize()
    ctx.set_timing(True)
    for _ in range(5):
        P.bw_probe(ctx, src, dst)
    probe_ms = ctx.stage_times()["probe"][0] / 5
    ctx.set_timing(False)
    probe_gbs = 2 * probe_bytes / (probe_ms * 1e-3) / 1e9
    del src, dst

    # headline: the captured batched step; roofline from the eager run of the same
    # (tuned) configuration, whose per-stage HIP-event times are the same kernels
    form = next(k for k in ("batched_graph", "batched", "plain") if k in res)
    head = res[form]
    eager = res.get("batched") or res["plain"]
    value = head["pixels"] / (head["ms"] * 1e-3) / 1e6
    dom, roof = roofline(eager["stages"], args.steps, n, eager["views"], eager["visible"],
                         eager["K"], eager["pixels"], eager["pairs"])
    roof["traffic"] = (measured_traffic(dom, eager["views"], tune["best"])
                       if args.n is None and args.grid is None and tune is not None else None)
    # whole-step fraction of the HBM roofline: the compulsory bytes of every stage
    # (the algorithmic model above) over the captured step's time, against the
    # copy probe's achievable bandwidth and the published peak
    step_bytes = sum(algorithmic(st_, n, eager["views"], eager["visible"], eager["K"],
                                 eager["pixels"], eager["pairs"])[0]
                     for st_ in ("project", "depth_sort", "scan", "emit", "tile_sort", "ranges",
                                 "blend_fwd", "loss", "blend_bwd", "project_bwd"))
    step_gbs = step_bytes / (head["ms"] * 1e-3) / 1e9
    step_hbm = {"algorithmic_bytes": int(step_bytes), "ms": round(head["ms"], 4),
                "GBps": round(step_gbs, 1), "frac_of_probe": round(step_gbs / probe_gbs, 4),
                "frac_of_peak": round(step_gbs / HBM_PEAK_GBS, 4)}
    if args.workload == "miranda18m":
        field = "seeded 2048^3 mixing-layer isosurface"
        views_desc = "2 views of 4096^2"
    else:
        field = "seeded 1024^3 blob+noise isosurface"
        views_desc = "4 views (2x2048^2 + 2x1536^2)"
    if form != "plain":
        how = "one hipGraph replay" if form == "batched_graph" else "eager launches"
        wl = (f"{args.workload}: {n} Gaussians on a {field}, SH3; "
              f"batched form: {views_desc} per step, {how} "
              f"(projection, sort, persistent/grid blend, loss gradient, backward), tuned "
              f"tile {tune['best']['tile']}, LDS depth {tune['best']['lds_depth']}, "
              f"flags {tune['best']['flags']}")
    else:
        wl = f"{args.workload}: {n} Gaussians, SH3; plain form: one {sizes[0]}^2 view per step"
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "Mpix/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(head["ms"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl, "views_per_step": head["views"],
                   "pixels_per_step": head["pixels"], "gaussians": n},
        "gaussians_per_s": round(n * head["views"] / (head["ms"] * 1e-3), 1),
        "memory": memory,
        "step_hbm": step_hbm,
        "roofline": roof,
        "timing": ("per-step HIP events on the launch stream, median over the timed steps "
                   "after the warm-up steps; mean_wall = synchronised wall clock / steps"),
        "forms": {k: {"ms_per_step": round(r["ms"], 3),
                      "ms_stats": {a: round(b, 4) for a, b in r["timing"].items()},
                      "mpix_per_s": round(r["pixels"] / (r["ms"] * 1e-3) / 1e6, 3),
                      "records_K": r["K"], "visible": r["visible"], "pairs": r["pairs"],
                      "tiles_per_entry": round(r["K"] / max(r["visible"], 1), 3),
                      "loss": round(r["loss"], 6),
                      **({"ms_with_adam": round(r["ms_with_adam"], 3), "capacity": r["capacity"]}
                         if "ms_with_adam" in r else {}),
                      "stages_ms_per_step": {s: round(t / args.steps, 4)
                                             for s, (t, c) in r["stages"].items() if c}}
                  for k, r in res.items()},
        "batched_vs_plain": (round((res["batched_graph"]["pixels"] / res["batched_graph"]["ms"])
                                   / (res["plain"]["pixels"] / res["plain"]["ms"]), 3)
                             if "batched_graph" in res and "plain" in res else None),
        "autotune": tune,
        "adam": {"ms": round(adam_ms, 4), "GBps_algorithmic": round(adam_gbs, 1),
                 "frac_of_probe": round(adam_gbs / probe_gbs, 4)},
        "hbm_probe": {"GBps": round(probe_gbs, 1), "bytes_per_launch": 2 * probe_bytes,
                      "ms": round(probe_ms, 4), "frac_of_peak": round(probe_gbs / HBM_PEAK_GBS, 4)},
    }
    if args.wide and args.workload == "kingsnake4m" and args.only in ("all", "batched"):
        t0 = time.perf_counter()
        wsc = wide_scales(P, ctx, params, cams, targets, min(args.steps, 5), min(args.warmup, 2),
                          torch)
        out["forms"]["batched_graph_wide_scales"] = wsc
        log(f"wide-scale 4M step: {wsc['ms_per_step']:.2f} ms, {wsc['mpix_per_s']:.0f} Mpix/s, "
            f"K={wsc['records_K']} ({time.perf_counter() - t0:.1f}s)")
    if not args.no_train and args.workload == "kingsnake4m":
        t0 = time.perf_counter()
        out["train_c1"] = train_c1(P, ctx, torch, iters=args.train_iters)
        log(f"training run in {time.perf_counter() - t0:.1f}s: "
            f"{out['train_c1']['held_out'][-1]}")
    if not args.no_serve:
        out["serve"] = serve_bench(P, ctx, params, torch, n_requests=args.serve_requests)
    if not args.no_c3 and args.workload == "kingsnake4m":
        del params
        torch.cuda.empty_cache()
        t0 = time.perf_counter()
        c3 = miranda_insitu(P, torch, args.steps, args.warmup)
        out["forms"]["miranda18m_batched_graph"] = c3
        log(f"18M step: {c3['ms_per_step']:.2f} ms, {c3['mpix_per_s']:.0f} Mpix/s "
            f"({time.perf_counter() - t0:.1f}s)")
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(scene, cams_d[0], targets_np[0], tile=args.tile)
        if args.cpu_c1:
            out["cpu_baseline"]["c1_full_view"] = cpu_c1_view(_cpu_cores())
        log(f"cpu baseline in {time.perf_counter() - t0:.1f}s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
