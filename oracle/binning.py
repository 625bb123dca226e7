"""Tile-binning oracle (test infrastructure only).

Binning is acceleration, not part of what the rasterizer computes: a
Gaussian is listed in every tile that holds an integer pixel inside the
rect [mx - rx, mx + rx] x [my - ry, my + ry] clipped to the image, and each
tile list is ordered by (depth, index).  With the integer half-widths at
least the extent of the Gaussian's support (alpha >= alpha_min), the lists
contain every Gaussian that can touch a pixel of the tile, so the image does
not depend on the tile size.

The oracle works from the FP32 projection outputs of the path under test
(mean, integer half-widths, depth) because the lists are a discrete function
of those values: the rect is formed with one IEEE binary32 rounding per
bound (mx - rx, mx + rx, ...), then ceil / floor, clipping and integer
division by the tile size.  Emission is Gaussian-index order with tiles row-major inside the
rect; a stable sort on the 64-bit key (tile << 32 | binary32 bits of depth)
then gives the per-tile (depth, index) order.  Depths are positive, so their
bit patterns order like their values.
"""
from __future__ import annotations

import numpy as np


def tile_rects(mx, my, rx, ry, width: int, height: int, tile: int):
    """Per-Gaussian inclusive tile rect (tx0, ty0, tx1, ty1) and tile count."""
    mx = np.asarray(mx, np.float32)
    my = np.asarray(my, np.float32)
    fx = np.asarray(rx).astype(np.float32)
    fy = np.asarray(ry).astype(np.float32)
    with np.errstate(invalid="ignore", over="ignore"):
        fu0 = np.maximum(np.ceil(mx - fx), np.float32(0))
        fu1 = np.minimum(np.floor(mx + fx), np.float32(width - 1))
        fv0 = np.maximum(np.ceil(my - fy), np.float32(0))
        fv1 = np.minimum(np.floor(my + fy), np.float32(height - 1))
    ok = (np.asarray(rx) > 0) & (np.asarray(ry) > 0) & (fu0 <= fu1) & (fv0 <= fv1)
    u0 = np.where(ok, fu0, 0).astype(np.int64)
    u1 = np.where(ok, fu1, 0).astype(np.int64)
    v0 = np.where(ok, fv0, 0).astype(np.int64)
    v1 = np.where(ok, fv1, 0).astype(np.int64)
    tx0, tx1, ty0, ty1 = u0 // tile, u1 // tile, v0 // tile, v1 // tile
    count = np.where(ok, (tx1 - tx0 + 1) * (ty1 - ty0 + 1), 0)
    return tx0, ty0, tx1, ty1, count


def bin_and_sort(mx, my, rx, ry, depth, width: int, height: int, tile: int = 16):
    """Returns dict(tiles_touched, keys u64[M], values u32[M], ranges u32[T,2])."""
    tiles_x = (width + tile - 1) // tile
    tiles_y = (height + tile - 1) // tile
    T = tiles_x * tiles_y
    tx0, ty0, tx1, ty1, count = tile_rects(mx, my, rx, ry, width, height, tile)
    M = int(count.sum())
    gid = np.repeat(np.arange(len(count), dtype=np.int64), count)
    start = np.concatenate([[0], np.cumsum(count)[:-1]]) if len(count) else np.zeros(0, np.int64)
    local = np.arange(M, dtype=np.int64) - np.repeat(start, count)
    wdt = (tx1 - tx0 + 1)[gid]
    tx = tx0[gid] + local % wdt
    ty = ty0[gid] + local // wdt
    tile_id = (ty * tiles_x + tx).astype(np.uint64)
    zbits = np.asarray(depth, np.float32).view(np.uint32).astype(np.uint64)[gid]
    keys = (tile_id << np.uint64(32)) | zbits
    order = np.argsort(keys, kind="stable")
    keys = keys[order]
    values = gid[order].astype(np.uint32)
    ranges = np.zeros((T, 2), np.uint32)
    if M:
        tsorted = (keys >> np.uint64(32)).astype(np.int64)
        first = np.ones(M, bool)
        first[1:] = tsorted[1:] != tsorted[:-1]
        last = np.ones(M, bool)
        last[:-1] = tsorted[1:] != tsorted[:-1]
        ranges[tsorted[first], 0] = np.nonzero(first)[0]
        ranges[tsorted[last], 1] = np.nonzero(last)[0] + 1
    return dict(tiles_touched=count.astype(np.int32), keys=keys, values=values, ranges=ranges,
                tiles_x=tiles_x, tiles_y=tiles_y)
