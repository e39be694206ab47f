"""Front-to-back alpha compositing over a tile's sorted list, and its derivative.

Reading used (3D-GS compositing, adopted by citation in Sec. III): for a pixel
centre q and a listed Gaussian g with d = q - mean2D,

    power = -1/2 (A dx^2 + C dy^2) - B dx dy      skip the pair if power > 0
    alpha = min(0.99, opacity * exp(power))        skip the pair if alpha < 1/255
    T'    = T (1 - alpha)                          stop (without blending) if T' < 1e-4
    C    += rgb alpha T ;  T = T' ;  n = position + 1

and out = C + T_final * bg.  The derivative is that of this forward exactly:
with S_k the colour composited behind contributor k (plus T_final bg),
d out / d rgb_k = alpha_k T_k and d out / d alpha_k = rgb_k T_k - S_k/(1-alpha_k);
alpha has zero derivative where the 0.99 clamp is active.

``flags`` mark pixels where a decision fell within a relative 1e-5 of its
threshold (absolute 1e-6 for power vs 0): float32 and float64 evaluations may
legitimately take different branches there.
"""
from __future__ import annotations

import numpy as np

ALPHA_MIN = 1.0 / 255.0
ALPHA_MAX = 0.99
T_MIN = 1e-4
FLAG_REL = 1e-5
FLAG_POW = 1e-6


def _pairs(proj, gids, px, py):
    m = proj["m"][:, gids]
    con = proj["conic"][:, gids]
    dx = px[:, None] - m[0][None, :]
    dy = py[:, None] - m[1][None, :]
    power = -0.5 * (con[0][None] * dx * dx + con[2][None] * dy * dy) - con[1][None] * dx * dy
    G = np.exp(power)
    a_raw = proj["opacity"][gids][None, :] * G
    return dx, dy, power, G, a_raw, con


def composite_tile(proj, gids, px, py, bg, flip=None):
    """Vectorised forward of one tile.  px, py: pixel centres (P,); gids: list (L,).

    ``flip`` (optional, bool (P, L)) inverts the listed threshold decisions; it
    is used only to evaluate the other branch at flagged pairs.
    Returns dict(out (3,P), T (P,), n (P,), flags (P,), flagpos list, state...).
    """
    P, L = px.shape[0], gids.shape[0]
    bg = np.asarray(bg, np.float64)
    if L == 0:
        out = np.repeat(bg[:, None], P, 1)
        return dict(out=out, T=np.ones(P), n=np.zeros(P, np.int64), flags=np.zeros(P, bool),
                    flagpos=[[] for _ in range(P)], contrib=np.zeros((P, 0), bool))
    dx, dy, power, G, a_raw, con = _pairs(proj, gids, px, py)
    alpha = np.minimum(ALPHA_MAX, a_raw)
    valid = (power <= 0) & (alpha >= ALPHA_MIN)
    f_pow = np.abs(power) < FLAG_POW
    f_amin = np.abs(a_raw * 255.0 - 1.0) < FLAG_REL
    f_amax = np.abs(a_raw / ALPHA_MAX - 1.0) < FLAG_REL
    if flip is not None:
        valid = valid ^ (flip & (f_pow | f_amin))
    a_eff = np.where(valid, alpha, 0.0)
    Tincl = np.cumprod(1.0 - a_eff, axis=1)
    stop_here = valid & (Tincl < T_MIN)
    f_T = valid & (np.abs(Tincl / T_MIN - 1.0) < FLAG_REL)
    if flip is not None:
        stop_here = stop_here ^ (flip & f_T)
    has_stop = stop_here.any(1)
    s = np.where(has_stop, np.argmax(stop_here, 1), L)
    k = np.arange(L)[None, :]
    contrib = valid & (k < s[:, None])
    Texcl = np.concatenate([np.ones((P, 1)), Tincl[:, :-1]], 1)
    w = np.where(contrib, a_eff * Texcl, 0.0)
    rgb = proj["rgb"][:, gids]
    C = w @ rgb.T                                                  # (P, 3)
    Tfin = np.where(has_stop, Texcl[np.arange(P), np.minimum(s, L - 1)], Tincl[:, -1])
    n = np.where(contrib.any(1), L - np.argmax(contrib[:, ::-1], 1), 0)
    decided = k <= s[:, None]
    fl = decided & (f_pow | (f_amin & (power <= 0)) | (f_amax & (power <= 0)) | f_T)
    flagpos = [np.nonzero(fl[p])[0].tolist() for p in range(P)]
    out = C.T + Tfin[None, :] * bg[:, None]
    return dict(out=out, T=Tfin, n=n.astype(np.int64), flags=fl.any(1), flagpos=flagpos,
                contrib=contrib, w=w, Texcl=Texcl, alpha=alpha, a_raw=a_raw, G=G, dx=dx,
                dy=dy, con=con, rgb=rgb)


def tile_pixels(tx, ty, tile, W, H):
    xs = np.arange(tx * tile, min((tx + 1) * tile, W))
    ys = np.arange(ty * tile, min((ty + 1) * tile, H))
    X, Y = np.meshgrid(xs, ys)
    return X.ravel(), Y.ravel()


def render_view(proj, lists, bg=(0.0, 0.0, 0.0)):
    """Image (3, H, W), final T, n_contrib and near-threshold flags of one view."""
    keys, gids, ranges = lists
    W, H, tile = proj["W"], proj["H"], proj["tile"]
    tiles_x = (W + tile - 1) // tile
    img = np.zeros((3, H, W))
    Tf = np.zeros((H, W))
    nc = np.zeros((H, W), np.int64)
    flags = np.zeros((H, W), bool)
    for t in range(ranges.shape[0]):
        tx, ty = t % tiles_x, t // tiles_x
        X, Y = tile_pixels(tx, ty, tile, W, H)
        g = gids[ranges[t, 0]:ranges[t, 1]]
        r = composite_tile(proj, g, X + 0.5, Y + 0.5, bg)
        img[:, Y, X] = r["out"]
        Tf[Y, X] = r["T"]
        nc[Y, X] = r["n"]
        flags[Y, X] = r["flags"]
    return img, Tf, nc, flags


def pixel_loop(proj, x, y, bg=(0.0, 0.0, 0.0), tile=None, order=None):
    """Brute force for one pixel: every Gaussian in (depth bits, index) order.

    With ``tile`` given, a Gaussian takes part only if its tile rectangle holds
    the pixel's tile; without it every visible Gaussian takes part.
    Returns (out (3,), T, index of the last contributor or -1).
    """
    if order is None:
        bits = proj["depth32"].view(np.uint32)
        ids = np.nonzero(proj["touched"] if tile is not None else proj["ok"])[0]
        order = ids[np.argsort(bits[ids], kind="stable")]
    T = 1.0
    C = np.zeros(3)
    last = -1
    qx, qy = x + 0.5, y + 0.5
    for g in order:
        if tile is not None:
            r = proj["rect"][:, g]
            if not (r[0] <= x // tile <= r[2] and r[1] <= y // tile <= r[3]):
                continue
        A, B, Cc = proj["conic"][:, g]
        dx = qx - proj["m"][0, g]
        dy = qy - proj["m"][1, g]
        power = -0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy
        if power > 0:
            continue
        alpha = min(ALPHA_MAX, proj["opacity"][g] * np.exp(power))
        if alpha < ALPHA_MIN:
            continue
        Tn = T * (1.0 - alpha)
        if Tn < T_MIN:
            break
        C += proj["rgb"][:, g] * alpha * T
        T = Tn
        last = g
    return C + T * np.asarray(bg, np.float64), T, last


def backward_tile(proj, gids, px, py, dout, bg, acc):
    """Accumulate screen-space gradients of one tile into ``acc``.

    dout: (3, P) upstream gradient of the tile's pixels.  acc holds arrays
    m (2,N), conic (3,N), opacity (N,), rgb (3,N).
    """
    if gids.shape[0] == 0:
        return
    f = composite_tile(proj, gids, px, py, bg)
    w, contrib, alpha, a_raw, G = f["w"], f["contrib"], f["alpha"], f["a_raw"], f["G"]
    rgb = f["rgb"]                                         # (3, L)
    dout = np.asarray(dout, np.float64)                    # (3, P)
    # d out / d rgb_k = alpha_k T_k
    np.add.at(acc["rgb"].T, gids, (w.T @ dout.T))
    # colour behind k: S_k = sum_{j>k} rgb_j w_j + T_final bg
    wc = w[:, :, None] * rgb.T[None, :, :]                  # (P, L, 3)
    suffix = np.cumsum(wc[:, ::-1, :], axis=1)[:, ::-1, :] - wc
    S = suffix + f["T"][:, None, None] * np.asarray(bg, np.float64)[None, None, :]
    Tk = np.where(contrib, f["Texcl"], 0.0)
    dalpha = ((rgb.T[None] * Tk[:, :, None] - S / (1.0 - alpha)[:, :, None])
              * dout.T[:, None, :]).sum(2)
    dalpha = np.where(contrib, dalpha, 0.0)
    live = contrib & (a_raw <= ALPHA_MAX)
    dpower = np.where(live, dalpha * alpha, 0.0)
    dop = np.where(live, dalpha * G, 0.0)
    dx, dy, con = f["dx"], f["dy"], f["con"]
    np.add.at(acc["opacity"], gids, dop.sum(0))
    np.add.at(acc["conic"][0], gids, (dpower * -0.5 * dx * dx).sum(0))
    np.add.at(acc["conic"][1], gids, (dpower * -dx * dy).sum(0))
    np.add.at(acc["conic"][2], gids, (dpower * -0.5 * dy * dy).sum(0))
    np.add.at(acc["m"][0], gids, (dpower * (con[0][None] * dx + con[1][None] * dy)).sum(0))
    np.add.at(acc["m"][1], gids, (dpower * (con[1][None] * dx + con[2][None] * dy)).sum(0))


def backward_view(proj, lists, dimg, bg=(0.0, 0.0, 0.0)):
    keys, gids, ranges = lists
    W, H, tile = proj["W"], proj["H"], proj["tile"]
    tiles_x = (W + tile - 1) // tile
    n = proj["m"].shape[1]
    acc = dict(m=np.zeros((2, n)), conic=np.zeros((3, n)), opacity=np.zeros(n),
               rgb=np.zeros((3, n)))
    for t in range(ranges.shape[0]):
        tx, ty = t % tiles_x, t // tiles_x
        X, Y = tile_pixels(tx, ty, tile, W, H)
        g = gids[ranges[t, 0]:ranges[t, 1]]
        backward_tile(proj, g, X + 0.5, Y + 0.5, dimg[:, Y, X], bg, acc)
    return acc
