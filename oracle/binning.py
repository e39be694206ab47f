"""Tile binning: one record per (Gaussian, touched tile), ordered for blending.

Reading used (the paper inherits tile rasterization from 3D-GS, Sec. III):
records are ordered by the 64-bit key (tile << 32) | bits(float32 depth), ties
broken by Gaussian index.  Depths are above the near plane (> 0), so the
unsigned order of their float32 bit patterns is their numeric order.  A
tile's range is [first, last + 1) of its records in that order, or [0, 0) when
it has none.

The oracle builds each tile's list directly from the definition: every
Gaussian whose tile rectangle contains the tile, ordered by (depth bits,
index).  The test-suite pins this against a global sort of all keys.
"""
from __future__ import annotations

import numpy as np


def depth_bits(depth32):
    return np.asarray(depth32, np.float32).view(np.uint32).astype(np.uint64)


def tile_lists(proj, tiles_x, tiles_y, tile_offset=0):
    """Sorted records of one view.

    Returns (keys uint64 [K], gids int64 [K], ranges int64 [tiles, 2]) with
    ranges relative to this view's records.
    """
    rect = proj["rect"]
    touched = proj["touched"]
    bits = depth_bits(proj["depth32"])
    keys, gids = [], []
    ranges = np.zeros((tiles_x * tiles_y, 2), np.int64)
    pos = 0
    for ty in range(tiles_y):
        in_y = touched & (rect[1] <= ty) & (ty <= rect[3])
        for tx in range(tiles_x):
            members = np.nonzero(in_y & (rect[0] <= tx) & (tx <= rect[2]))[0]
            t = ty * tiles_x + tx
            if members.size == 0:
                continue
            order = np.argsort(bits[members], kind="stable")   # ties keep index order
            g = members[order]
            keys.append((np.uint64(tile_offset + t) << np.uint64(32)) | bits[g])
            gids.append(g)
            ranges[t] = (pos, pos + g.size)
            pos += g.size
    if keys:
        return np.concatenate(keys), np.concatenate(gids).astype(np.int64), ranges
    return np.zeros(0, np.uint64), np.zeros(0, np.int64), ranges


def emitted_records(proj, tiles_x, tile_offset=0):
    """Unsorted records in emission order (index, then row-major tile)."""
    rect = proj["rect"]
    bits = depth_bits(proj["depth32"])
    keys, gids = [], []
    for g in np.nonzero(proj["touched"])[0]:
        for ty in range(rect[1, g], rect[3, g] + 1):
            for tx in range(rect[0, g], rect[2, g] + 1):
                keys.append((np.uint64(tile_offset + ty * tiles_x + tx) << np.uint64(32)) | bits[g])
                gids.append(g)
    return np.array(keys, np.uint64), np.array(gids, np.int64)
