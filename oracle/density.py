"""Adaptive density control of the 3D-GS training (clone, split, prune, opacity
reset).  Test infrastructure: the plain float64 definition the device path is
checked against; nothing in the product imports it.

The paper trains the cited 3D-GS model on the orbit views (Sec. III, Method
Overview) and states none of its training schedule; the density control here
is that model's, with these readings (each a choice where the paper is silent):

* statistics, per Gaussian, over the views since the last densification: the
  sum of the norms of its positional screen gradient in normalised device
  coordinates, (dL/dm_x W/2, dL/dm_y H/2) times a caller scale (the number of
  views of a batch whose loss is their mean, so that each view counts as in
  single-view training), the number of views in which it touched a tile, and
  the largest pixel radius it had in those views;
* the mean gradient g = sum / count (0 where the count is 0) selects a Gaussian
  when g >= tau (0.0002); a selected Gaussian whose largest scale is at most
  percent_dense (0.01) times the scene extent is cloned (an exact copy), one
  above it is split into n_split (2) children placed at mu + R(q) (s * z), z a
  standard normal draw, with scales s / split_div (1.6), the parent's rotation,
  opacity and colour, and the parent removed;
* prune: opacity below min_opacity (0.005); when a screen limit is set (after
  the first opacity reset), also a largest pixel radius above it (20) or a
  largest scale above max_world (0.1) times the extent.  New Gaussians have
  radius 0 and are tested on opacity and scale only;
* output order: the surviving originals in index order, then the surviving
  clones in the order of their sources, then the surviving children, source by
  source, child 0 before child 1;  Adam moments are copied for originals and
  start at zero for clones and children;
* opacity reset: opacity = min(opacity, 0.01) (logit form), with its Adam
  moments set to zero;
* split draws: Philox4x32-10 (the generator of the initialisation) with key =
  (seed low word, seed high word), counter = (source index, 16 + child, 0, 0);
  the first three of the four Box-Muller normals of its two pairs.
"""
from __future__ import annotations

import numpy as np

from .init import MASK, box_muller, philox4x32_10
from .project import quat_to_rot

GRAD_THRESHOLD = 0.0002
PERCENT_DENSE = 0.01
MIN_OPACITY = 0.005
MAX_SCREEN = 20.0
MAX_WORLD = 0.1
N_SPLIT = 2
SPLIT_DIV = 1.6
RESET_OPACITY = 0.01
KEYS = ("means", "log_scales", "quats", "opacity_logits", "sh")


def accumulate(stats, screen_mean_grads, touched, radius, widths, heights, scale=1.0):
    """Adds one batch of views to the statistics.

    screen_mean_grads: (V, 2, N) dL/d mean2D in pixels; touched (V, N) bool;
    radius (V, N) integer pixel radii; widths / heights of the V views.
    stats: dict(grad (N,), count (N,), max_radius (N,)), updated in place."""
    for v in range(len(widths)):
        t = np.asarray(touched[v], bool)
        gx = np.asarray(screen_mean_grads[v][0], np.float64) * (0.5 * widths[v])
        gy = np.asarray(screen_mean_grads[v][1], np.float64) * (0.5 * heights[v])
        stats["grad"][t] += scale * np.sqrt(gx * gx + gy * gy)[t]
        stats["count"][t] += 1
        stats["max_radius"][t] = np.maximum(stats["max_radius"][t], np.asarray(radius[v])[t])
    return stats


def split_normals(n_src, src_index, child, seed):
    """Standard normals (3, n_src) of child `child` of the given source indices."""
    idx = np.asarray(src_index, np.uint64)
    z0 = np.zeros(idx.shape, np.uint64)
    d = philox4x32_10([idx, z0 + 16 + child, z0, z0], (seed & MASK, (seed >> 32) & MASK))
    a0, a1 = box_muller(d[0], d[1])
    a2, _ = box_muller(d[2], d[3])
    return np.stack([a0, a1, a2], 0)


def densify(params, m, v, stats, extent, *, tau=GRAD_THRESHOLD, percent_dense=PERCENT_DENSE,
            min_opacity=MIN_OPACITY, max_screen=0.0, max_world=MAX_WORLD, n_split=N_SPLIT,
            split_div=SPLIT_DIV, seed=0):
    """One densification: returns (params, m, v, info) of the new set.

    max_screen <= 0 disables the screen and world size prune."""
    n = np.asarray(params["means"]).shape[1]
    P = {k: np.asarray(params[k], np.float64).reshape(-1, n) for k in KEYS}
    M = {k: np.asarray(m[k], np.float64).reshape(-1, n) for k in KEYS}
    Vv = {k: np.asarray(v[k], np.float64).reshape(-1, n) for k in KEYS}
    count = np.asarray(stats["count"], np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        g = np.where(count > 0, np.asarray(stats["grad"], np.float64) / count, 0.0)
    scale = np.exp(P["log_scales"])
    smax = scale.max(0)
    selected = g >= tau
    clone = selected & (smax <= percent_dense * extent)
    split = selected & (smax > percent_dense * extent)
    opacity = 1.0 / (1.0 + np.exp(-P["opacity_logits"][0]))
    low = opacity < min_opacity
    size_on = max_screen > 0
    big_ws = smax > max_world * extent
    big_vs = np.asarray(stats["max_radius"], np.float64) > max_screen
    keep_orig = ~split & ~low & ~(size_on & (big_vs | big_ws))
    keep_clone = clone & ~low & ~(size_on & big_ws)
    # children
    src = np.nonzero(split)[0]
    child_ls = P["log_scales"][:, src] - np.log(split_div)
    child_max = np.exp(child_ls).max(0) if src.size else np.zeros(0)
    keep_child = ~low[src] & ~(size_on & (child_max > max_world * extent))
    qn = P["quats"][:, src] / np.sqrt((P["quats"][:, src] ** 2).sum(0))
    Rq = quat_to_rot(qn)                                    # (3, 3, S)
    out_p = {k: [P[k][:, keep_orig], P[k][:, np.nonzero(keep_clone)[0]]] for k in KEYS}
    out_m = {k: [M[k][:, keep_orig], np.zeros((M[k].shape[0], int(keep_clone.sum())))]
             for k in KEYS}
    out_v = {k: [Vv[k][:, keep_orig], np.zeros((Vv[k].shape[0], int(keep_clone.sum())))]
             for k in KEYS}
    # children, source by source, child 0 before child 1
    ch = {k: np.zeros((P[k].shape[0], src.size, n_split)) for k in KEYS}
    for c in range(n_split):
        z = split_normals(src.size, src, c, seed)
        local = scale[:, src] * z                           # s * z
        ch["means"][:, :, c] = P["means"][:, src] + np.einsum("ijs,js->is", Rq, local)
        ch["log_scales"][:, :, c] = child_ls
        for k in ("quats", "opacity_logits", "sh"):
            ch[k][:, :, c] = P[k][:, src]
    kc = np.repeat(keep_child, n_split)
    for k in KEYS:
        flat = ch[k].reshape(P[k].shape[0], -1)[:, kc]
        out_p[k].append(flat)
        out_m[k].append(np.zeros_like(flat))
        out_v[k].append(np.zeros_like(flat))
    res_p = {k: np.concatenate(out_p[k], 1) for k in KEYS}
    res_p["opacity_logits"] = res_p["opacity_logits"][0]
    res_m = {k: np.concatenate(out_m[k], 1) for k in KEYS}
    res_m["opacity_logits"] = res_m["opacity_logits"][0]
    res_v = {k: np.concatenate(out_v[k], 1) for k in KEYS}
    res_v["opacity_logits"] = res_v["opacity_logits"][0]
    for d in (res_p, res_m, res_v):
        d["sh_degree"] = params["sh_degree"]
    info = dict(n_in=n, n_out=res_p["means"].shape[1], kept=int(keep_orig.sum()),
                cloned=int(keep_clone.sum()), split=int(src.size),
                children=int(kc.sum()), pruned=int((~keep_orig & ~split).sum()),
                clone_mask=clone, split_mask=split, keep_orig=keep_orig, keep_clone=keep_clone,
                split_src=src, keep_child=keep_child, mean_grad=g)
    return res_p, res_m, res_v, info


def opacity_reset(params, m, v, max_opacity=RESET_OPACITY):
    """opacity = min(opacity, max_opacity) in logit form; its Adam moments zeroed."""
    lim = np.log(max_opacity / (1.0 - max_opacity))
    p = dict(params)
    p["opacity_logits"] = np.minimum(np.asarray(params["opacity_logits"], np.float64), lim)
    m2, v2 = dict(m), dict(v)
    m2["opacity_logits"] = np.zeros_like(np.asarray(m["opacity_logits"], np.float64))
    v2["opacity_logits"] = np.zeros_like(np.asarray(v["opacity_logits"], np.float64))
    return p, m2, v2
