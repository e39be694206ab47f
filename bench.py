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
FP32_PEAK_TFLOPS = 157.3
# algorithmic FLOP per (pixel, list position up to the pixel's last contributor)
FLOP_PAIR_FWD = 23
FLOP_PAIR_BWD = 68
# HBM bytes per launch of a kernel, from calibrated rocprofv3 FETCH_SIZE / WRITE_SIZE runs
# (profiles/hbm_traffic_kingsnake4m.md), valid only while the kernel source is unchanged:
# the figure is dropped (traffic = null) when the source hash no longer matches.
MEASURED_TRAFFIC = {
    "blend_bwd": {"source": "paper_2509_05216_amd/csrc/blend.hip",
                  "sha256": "1953ad7eb534dcf81ae396938eaec72fad9b5229af48b87b292def31cf2c98aa",
                  "read_bytes": 2887.4e6, "write_bytes": 3893.5e6, "views": 4},
}


def measured_traffic(kernel, views):
    import hashlib
    m = MEASURED_TRAFFIC.get(kernel)
    if m is None or m["views"] != views:
        return None
    with open(os.path.join(ROOT, m["source"]), "rb") as fh:
        if hashlib.sha256(fh.read()).hexdigest() != m["sha256"]:
            return None
    return round(m["read_bytes"] + m["write_bytes"])


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=None, help="Gaussian count override (smaller runs)")
    ap.add_argument("--grid", type=int, default=None, help="field grid override")
    ap.add_argument("--tile", type=int, default=16)
    ap.add_argument("--lds-depth", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-tiles", type=int, default=96, help="tiles in the CPU-baseline sample")
    ap.add_argument("--only", choices=["all", "batched", "plain"], default="all")
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


def run_steps(P, ctx, params, cams, targets, steps, warmup, tile, depth, torch):
    """Time `steps` fwd+bwd steps; returns per-step ms, stage totals and a frame."""
    frame = P.Frame()
    images = [torch.empty((3, c.height, c.width), device="cuda") for c in cams]
    grads = params.zeros_like()

    def one():
        P.render_fwd(ctx, params, cams, images, tile=tile, lds_depth=depth, frame=frame)
        loss, dl = P.loss_grad(ctx, images, targets, cams)
        P.render_bwd(ctx, frame, params, dl, grads)
        return loss

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    ctx.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        loss = one()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    stages = ctx.stage_times()
    ctx.set_timing(False)
    return ms, stages, frame, float(loss.item()), images, grads


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
                     "traffic": traffic, "kernel": dom, "avg_ms": round(avg_ms, 4),
                     "algorithmic_flop": flops, "algorithmic_bytes": byts,
                     "hbm_GBps_algorithmic": round(byts / (avg_ms * 1e-3) / 1e9, 1)}
    ach = byts / (avg_ms * 1e-3) / 1e9
    return dom, {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
                 "avg_ms": round(avg_ms, 4), "algorithmic_bytes": byts}


def cpu_baseline(scene, cam_d, target, n_tiles, tile=16):
    """The oracle's fwd+bwd on a bounded sample of one 2048^2 view (single thread).

    Per-Gaussian work (projection, parameter chain rule) runs on all N; the
    per-tile work (binning, compositing forward and backward) on a seeded
    sample of tiles, scaled by its share of the total list length; the loss
    on a 256^2 crop, scaled by pixel count.
    """
    from threadpoolctl import threadpool_limits

    from oracle import blend, loss as oloss, project, backward as obwd
    with threadpool_limits(limits=1):
        params = scene.params
        W, H = cam_d["width"], cam_d["height"]
        tx, ty = (W + tile - 1) // tile, (H + tile - 1) // tile
        t0 = time.perf_counter()
        pr = project.project(params, cam_d, tile)
        t_proj = time.perf_counter() - t0
        rng = np.random.default_rng(1234)
        sample = rng.choice(tx * ty, size=min(n_tiles, tx * ty), replace=False)
        rect = pr["rect"]
        touched = pr["touched"]
        # total list length of every tile (for scaling) from the rectangles
        cnt = np.zeros((ty + 1, tx + 1), np.int64)
        ids = np.nonzero(touched)[0]
        np.add.at(cnt, (rect[1, ids], rect[0, ids]), 1)
        np.add.at(cnt, (rect[1, ids], rect[2, ids] + 1), -1)
        np.add.at(cnt, (rect[3, ids] + 1, rect[0, ids]), -1)
        np.add.at(cnt, (rect[3, ids] + 1, rect[2, ids] + 1), 1)
        lens = np.cumsum(np.cumsum(cnt, 0), 1)[:ty, :tx].ravel()
        n = params["means"].shape[1]
        acc = dict(m=np.zeros((2, n)), conic=np.zeros((3, n)), opacity=np.zeros(n),
                   rgb=np.zeros((3, n)))
        bits = pr["depth32"].view(np.uint32)
        t0 = time.perf_counter()
        for t in sample:
            x, y = t % tx, t // tx
            members = np.nonzero(touched & (rect[0] <= x) & (x <= rect[2]) & (rect[1] <= y)
                                 & (y <= rect[3]))[0]
            g = members[np.argsort(bits[members], kind="stable")]
            X, Y = blend.tile_pixels(x, y, tile, W, H)
            blend.composite_tile(pr, g, X + 0.5, Y + 0.5, (0, 0, 0))
            d = np.asarray(target[:, Y, X], np.float64) * 1e-3
            blend.backward_tile(pr, g, X + 0.5, Y + 0.5, d, (0, 0, 0), acc)
        t_tiles = time.perf_counter() - t0
        share = lens[sample].sum() / max(lens.sum(), 1)
        t0 = time.perf_counter()
        obwd.param_grads(pr, params, cam_d, acc)
        t_pbwd = time.perf_counter() - t0
        crop = np.asarray(target[:, :256, :256], np.float64)
        t0 = time.perf_counter()
        oloss.view_loss(crop * 0.9, crop)
        oloss.view_loss_grad(crop * 0.9, crop)
        t_loss = (time.perf_counter() - t0) * (W * H) / (256 * 256)
    total = t_proj + t_pbwd + t_tiles / max(share, 1e-12) + t_loss
    return {"value": round(W * H / total / 1e6, 6), "unit": "Mpix/s", "cores": 1,
            "kind": "oracle",
            "sample": (f"one {W}x{H} view of the {n}-Gaussian scene, float64 numpy, 1 thread: "
                       f"projection and parameter backward on all Gaussians, binning + "
                       f"compositing fwd/bwd on {len(sample)} seeded tiles scaled by their "
                       f"{share:.4f} share of list length, loss on a 256^2 crop scaled by "
                       f"pixels (estimate)"),
            "seconds": round(t_proj + t_tiles + t_pbwd + t_loss / ((W * H) / (256 * 256)), 2),
            "est_seconds_full_view": round(total, 1)}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "split is not part of this build", file=sys.stderr)
        sys.exit(2)
    import torch

    import gsscenes
    import paper_2509_05216_amd as P

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    t0 = time.perf_counter()
    scene = gsscenes.make_scene("kingsnake4m", n=args.n, G=args.grid)
    n = scene.params["means"].shape[1]
    log(f"scene: {n} Gaussians in {time.perf_counter() - t0:.1f}s")
    ctx = P.Context(0)
    params = P.Params.from_numpy(scene.params)
    sizes = [2048, 2048, 1536, 1536]
    all_cams = P.orbit_cameras(16, 2.5, 60.0, 2048, 2048)
    cams = []
    for i, s in enumerate(sizes):
        c = all_cams[i * 4]
        d = P.camera_to_dict(c)
        cams.append(P.camera(d["R"], d["t"], d["fx"] * s / 2048, d["fy"] * s / 2048, s / 2, s / 2,
                             s, s))
    cams_d = [P.camera_to_dict(c) for c in cams]
    t0 = time.perf_counter()
    targets_np = make_targets(scene, cams_d)
    targets = [torch.tensor(t, device="cuda") for t in targets_np]
    log(f"targets in {time.perf_counter() - t0:.1f}s")
    torch.cuda.synchronize()

    res = {}
    if args.only in ("all", "batched"):
        ms, stages, frame, loss, _, _ = run_steps(P, ctx, params, cams, targets, args.steps,
                                                  args.warmup, args.tile, args.lds_depth, torch)
        st, pairs, vis = frame_counts(frame, n, torch)
        res["batched"] = dict(ms=ms, stages=stages, K=st["n_records"], pixels=st["n_pixels"],
                              pairs=pairs, visible=vis, views=4, loss=loss)
        log(f"batched: {ms:.2f} ms/step, K={st['n_records']}, pairs={pairs}")
        frame.release()
    if args.only in ("all", "plain"):
        ms, stages, frame, loss, _, _ = run_steps(P, ctx, params, cams[:1], targets[:1],
                                                  args.steps, args.warmup, args.tile,
                                                  args.lds_depth, torch)
        st, pairs, vis = frame_counts(frame, n, torch)
        res["plain"] = dict(ms=ms, stages=stages, K=st["n_records"], pixels=st["n_pixels"],
                            pairs=pairs, visible=vis, views=1, loss=loss)
        log(f"plain: {ms:.2f} ms/step, K={st['n_records']}, pairs={pairs}")
        frame.release()
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

    head = res.get("batched") or res["plain"]
    form = "batched" if "batched" in res else "plain"
    value = head["pixels"] / (head["ms"] * 1e-3) / 1e6
    dom, roof = roofline(head["stages"], args.steps, n, head["views"], head["visible"], head["K"],
                         head["pixels"], head["pairs"])
    roof["traffic"] = measured_traffic(dom, head["views"]) if args.n is None else None
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "Mpix/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(head["ms"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": (f"kingsnake4m: {n} Gaussians on a seeded 1024^3 blob+noise "
                                f"isosurface, SH3, {form} form"
                                + (": 4 views (2x2048^2 + 2x1536^2) per step in one call"
                                   if form == "batched" else ": one 2048^2 view per step")),
                   "tile": args.tile, "lds_depth": args.lds_depth,
                   "views_per_step": head["views"], "pixels_per_step": head["pixels"]},
        "gaussians_per_s": round(n * head["views"] / (head["ms"] * 1e-3), 1),
        "roofline": roof,
        "forms": {k: {"ms_per_step": round(r["ms"], 3),
                      "mpix_per_s": round(r["pixels"] / (r["ms"] * 1e-3) / 1e6, 3),
                      "records_K": r["K"], "visible": r["visible"], "pairs": r["pairs"],
                      "loss": round(r["loss"], 6),
                      "stages_ms_per_step": {s: round(t / args.steps, 4)
                                             for s, (t, c) in r["stages"].items() if c}}
                  for k, r in res.items()},
        "adam": {"ms": round(adam_ms, 4), "GBps_algorithmic": round(adam_gbs, 1),
                 "frac_of_probe": round(adam_gbs / probe_gbs, 4),
                 "step_ms_with_adam": round(head["ms"] + adam_ms, 3)},
        "hbm_probe": {"GBps": round(probe_gbs, 1), "bytes_per_launch": 2 * probe_bytes,
                      "ms": round(probe_ms, 4), "frac_of_peak": round(probe_gbs / HBM_PEAK_GBS, 4)},
    }
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(scene, cams_d[0], targets_np[0], args.cpu_tiles,
                                           args.tile)
        log(f"cpu baseline in {time.perf_counter() - t0:.1f}s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
