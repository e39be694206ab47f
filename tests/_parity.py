"""Comparators between the HIP path and the oracle (test infrastructure).

Images: max absolute error per channel <= tol, except at pixels where the
oracle flagged a threshold decision within a relative 1e-5 of its threshold;
there the pixel is accepted if some choice of branches at the flagged pairs
(up to 4 pairs, 16 combinations) reproduces the device value within tol.
"""
from itertools import product

import numpy as np

from oracle import blend


def other_branch_matches(pr, g, x, y, got, bg=(0.0, 0.0, 0.0), tol=1e-4):
    """True when some choice of branches at the pixel's flagged pairs (first 4)
    reproduces the device value ``got`` (3,) of pixel (x, y) over list g."""
    px, py = np.array([x + 0.5]), np.array([y + 0.5])
    base = blend.composite_tile(pr, g, px, py, bg)
    pos = base["flagpos"][0][:4]
    for bits in product([0, 1], repeat=len(pos)):
        if not any(bits):
            continue
        flip = np.zeros((1, g.size), bool)
        for b, p in zip(bits, pos):
            flip[0, p] = bool(b)
        alt = blend.composite_tile(pr, g, px, py, bg, flip=flip)
        if np.abs(alt["out"][:, 0] - got).max() <= tol:
            return True
    return False


def tile_report(pr, g, X, Y, got, bg=(0.0, 0.0, 0.0), tol=1e-4):
    """Compare the device values got (3, P) of pixels (X, Y) of one tile whose
    sorted list is g with the oracle's compositing of that list."""
    got = np.asarray(got, np.float64)
    r = blend.composite_tile(pr, g, X + 0.5, Y + 0.5, bg)
    err = np.abs(got - r["out"]).max(0)
    bad = err > tol
    failed = [(int(X[i]), int(Y[i]), float(err[i])) for i in np.nonzero(bad)[0]
              if not (r["flags"][i] and other_branch_matches(pr, g, X[i], Y[i], got[:, i], bg,
                                                             tol))]
    ok = ~r["flags"]
    return dict(max_err=float(err[ok].max()) if ok.any() else 0.0, failed=failed,
                oracle=r, n_flagged=int(r["flags"].sum()))


def image_report(fw, img_gpu, tol=1e-4, bg=(0.0, 0.0, 0.0)):
    img_gpu = np.asarray(img_gpu, np.float64)
    err = np.abs(img_gpu - fw["image"]).max(0)
    bad = err > tol
    flags = fw["flags"]
    unflagged_bad = bad & ~flags
    rescued, failed = 0, []
    pr = fw["proj"]
    keys, gids, ranges = fw["lists"]
    tile = pr["tile"]
    tiles_x = fw["tiles"][0]
    for y, x in zip(*np.nonzero(bad & flags)):
        t = (y // tile) * tiles_x + x // tile
        g = gids[ranges[t, 0]:ranges[t, 1]]
        if other_branch_matches(pr, g, x, y, img_gpu[:, y, x], bg, tol):
            rescued += 1
        else:
            failed.append((int(x), int(y), float(err[y, x])))
    return dict(max_err=float(err[~flags].max()) if (~flags).any() else 0.0,
                n_flagged=int(flags.sum()), n_bad_unflagged=int(unflagged_bad.sum()),
                bad_unflagged=[(int(x), int(y), float(err[y, x]))
                               for y, x in zip(*np.nonzero(unflagged_bad))][:10],
                rescued=rescued, failed=failed, flagged_mask=flags)


def assert_image(fw, img_gpu, tol=1e-4, bg=(0.0, 0.0, 0.0)):
    r = image_report(fw, img_gpu, tol, bg)
    assert r["n_bad_unflagged"] == 0, r["bad_unflagged"]
    assert not r["failed"], r["failed"]
    return r


def rel_l2(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
