"""Oracle of the large-scene cells (test infrastructure only): Lloyd's
k-means over the Gaussians' means in FP64 and the visibility of a cell's
bounding sphere from a camera.

* Initial centroids: the means at indices floor((j + 1/2) n / k),
  j = 0..k-1 (the scene's Gaussians are seeded frame by frame along the
  trajectory, so this spreads them along it); each iteration assigns every
  mean to its nearest centroid by the squared distance (dx dx + dy dy) +
  dz dz in binary64 (ties to the lower centroid), then moves each centroid
  to the mean of its members (a centroid without members stays).
* A cell is the set of Gaussians assigned to one centroid; its bounding
  sphere has the centroid as centre and, as radius, the largest
  centre-to-mean distance plus a margin of three times the largest axis
  scale of its Gaussians (their splats reach beyond the means).
* A sphere is visible from a world->camera pose [R | t] with pinhole
  intrinsics when it reaches in front of the near plane and meets the four
  side planes of the image's frustum widened by the rasterizer's guard band
  factor.
"""
from __future__ import annotations

import numpy as np


def init_indices(n: int, k: int):
    return np.floor((np.arange(k) + 0.5) * n / k).astype(np.int64)


def assign(means, cent):
    """Nearest centroid of every mean (binary64, ties to the lower index)."""
    m = np.asarray(means, np.float32).astype(np.float64)
    c = np.asarray(cent, np.float64)
    best = np.full(m.shape[1], np.inf)
    out = np.zeros(m.shape[1], np.int32)
    for j in range(c.shape[0]):
        d = m - c[j][:, None]
        dist = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
        better = dist < best
        best = np.where(better, dist, best)
        out = np.where(better, j, out)
    return out


def update(means, labels, cent):
    m = np.asarray(means, np.float32).astype(np.float64)
    c = np.array(cent, np.float64)
    for j in range(c.shape[0]):
        sel = labels == j
        if sel.any():
            c[j] = m[:, sel].mean(axis=1)
    return c


def kmeans(means, k: int, iters: int):
    """(centroids [k][3], labels [n]) after `iters` Lloyd iterations and a
    final assignment."""
    m = np.asarray(means, np.float32)
    cent = m[:, init_indices(m.shape[1], k)].T.astype(np.float64)
    for _ in range(iters):
        cent = update(m, assign(m, cent), cent)
    return cent, assign(m, cent)


def cell_spheres(means, log_scales, labels, cent, margin_scales: float = 3.0):
    """Per cell: radius = max centre-to-mean distance + margin x max axis scale."""
    m = np.asarray(means, np.float32).astype(np.float64)
    s = np.exp(np.asarray(log_scales, np.float32).astype(np.float64).max(axis=0))
    k = cent.shape[0]
    rad = np.zeros(k)
    for j in range(k):
        sel = labels == j
        if sel.any():
            d = m[:, sel] - cent[j][:, None]
            rad[j] = np.sqrt((d * d).sum(0)).max() + margin_scales * s[sel].max()
    return rad


def sphere_visible(c, r, R, t, fx, fy, cx, cy, W, H, near=0.2, guard=1.3):
    """Whether the sphere (centre c, radius r) meets the camera's frustum."""
    p = np.asarray(R, np.float64) @ np.asarray(c, np.float64) + np.asarray(t, np.float64)
    if p[2] + r <= near:
        return False
    # side planes through the camera centre: x / z = xmax etc., widened by the guard band
    xr, xl = guard * (W - cx) / fx, guard * cx / fx
    yb, yt = guard * (H - cy) / fy, guard * cy / fy
    for n in (np.array([1.0, 0.0, -xr]), np.array([-1.0, 0.0, -xl]), np.array([0.0, 1.0, -yb]),
              np.array([0.0, -1.0, -yt])):
        if n @ p > r * np.linalg.norm(n):
            return False
    return True
