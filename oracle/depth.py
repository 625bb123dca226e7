"""Oracle of the guided-matching depth of new primitives (the paper's
appendix on depth for Gaussian primitives, used by section 4.2), test
infrastructure only.

For every pixel (x, y) of frame i, with monocular depth Z* there:

* candidates: N inverse depths d_k uniform over [1/Z* - r, 1/Z* + r]
  (r = 0.1), d_k = 1/Z* - r + 2 r k / (N - 1), the lower end raised to
  d_min > 0 so that every candidate lies in front of the camera;
* one neighbouring frame j per pixel (the paper's adaptive choice, read
  here as the neighbour that separates the candidates most): the neighbour
  whose reprojections of the nearest and farthest candidates are farthest
  apart in pixels, among those where both fall inside the image (ties to
  the lower index; none: the pixel gets no estimate);
* reprojection: X = K^-1 (x, y, 1) / d_k in frame i's camera, p = K (R X +
  t) with (R, t) the pose of j relative to i, (u, v) = p_xy / p_z;
* correlation C_k = <F_i(x, y), F_j(u, v)>, F_j sampled bilinearly (pixel
  centres at integer coordinates; a tap outside the image counts as 0); a
  candidate behind camera j has no correlation;
* the best candidate k* = argmax C_k (the lowest k on ties), refined by the
  vertex of the parabola through (k* - 1, k*, k* + 1) when both neighbours
  exist and the parabola opens downwards; depth = 1 / d(k* + delta).

Features are given as FP16 [H][W][C] (channel-last) and used exactly as
stored; everything else is FP64.
"""
from __future__ import annotations

import numpy as np

R_INV = 0.1
D_MIN = 1e-3


def candidates(zmono, n: int, r: float = R_INV, d_min: float = D_MIN):
    """[n][H][W] inverse depths."""
    inv = 1.0 / np.asarray(zmono, np.float64)
    lo = np.maximum(inv - r, d_min)
    hi = inv + r
    k = np.arange(n, dtype=np.float64)[:, None, None]
    return lo[None] + (hi - lo)[None] * k / (n - 1)


def reproject(K, R, t, x, y, d):
    """Pixel coordinates in the neighbour and its camera depth."""
    fx, fy, cx, cy = K
    X = (x - cx) / fx / d
    Y = (y - cy) / fy / d
    Z = 1.0 / d
    pc = [R[r][0] * X + R[r][1] * Y + R[r][2] * Z + t[r] for r in range(3)]
    return fx * pc[0] / pc[2] + cx, fy * pc[1] / pc[2] + cy, pc[2]


def bilinear(F, u, v):
    """F [H][W][C] sampled at (u, v) arrays; taps outside the image are 0."""
    H, W, C = F.shape
    F = F.astype(np.float64)
    x0 = np.floor(u).astype(np.int64)
    y0 = np.floor(v).astype(np.int64)
    ax, ay = u - x0, v - y0
    out = np.zeros(u.shape + (C,))
    for dy, wy in ((0, 1 - ay), (1, ay)):
        for dx, wx in ((0, 1 - ax), (1, ax)):
            xx, yy = x0 + dx, y0 + dy
            ok = (xx >= 0) & (xx < W) & (yy >= 0) & (yy < H)
            tap = np.zeros(u.shape + (C,))
            tap[ok] = F[yy[ok], xx[ok]]
            out += (wx * wy)[..., None] * tap
    return out


def choose_neighbour(K, poses, zmono, n: int, W: int, H: int):
    """Per pixel the neighbour index (-1: none) by the separation rule."""
    d = candidates(zmono, n)
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    best = np.full((H, W), -1.0)
    choice = np.full((H, W), -1, np.int64)
    for j, (R, t) in enumerate(poses):
        u0, v0, z0 = reproject(K, R, t, xx, yy, d[0])
        u1, v1, z1 = reproject(K, R, t, xx, yy, d[-1])
        inside = lambda u, v, z: (z > 0) & (u >= 0) & (u <= W - 1) & (v >= 0) & (v <= H - 1)
        ok = inside(u0, v0, z0) & inside(u1, v1, z1)
        sep = np.hypot(u1 - u0, v1 - v0)
        take = ok & (sep > best)
        best = np.where(take, sep, best)
        choice = np.where(take, j, choice)
    return choice


def correlations(Fi, Fjs, K, poses, zmono, n: int, mask=None):
    """[n][H][W] correlation volume against each pixel's chosen neighbour
    (-inf where a candidate has none, and outside mask if given), the
    candidates and the choice."""
    H, W, _ = Fi.shape
    d = candidates(zmono, n)
    choice = choose_neighbour(K, poses, zmono, n, W, H)
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    fi = Fi.astype(np.float64)
    C = np.full((n, H, W), -np.inf)
    for j, (R, t) in enumerate(poses):
        sel = (choice == j) if mask is None else (choice == j) & mask
        if not sel.any():
            continue
        for k in range(n):
            u, v, z = reproject(K, R, t, xx[sel], yy[sel], d[k][sel])
            s = bilinear(Fjs[j], u, v)
            ck = np.einsum("pc,pc->p", fi[sel], s)
            C[k][sel] = np.where(z > 0, ck, -np.inf)
    return C, d, choice


def refine(C, d):
    """Argmax (lowest k on ties) and parabola vertex; returns depth (nan: no
    estimate), k*, delta."""
    n, H, W = C.shape
    kb = np.argmax(C, axis=0)
    cb = np.take_along_axis(C, kb[None], 0)[0]
    valid = np.isfinite(cb)
    km, kp = np.clip(kb - 1, 0, n - 1), np.clip(kb + 1, 0, n - 1)
    cm = np.take_along_axis(C, km[None], 0)[0]
    cp = np.take_along_axis(C, kp[None], 0)[0]
    inner = (kb > 0) & (kb < n - 1) & np.isfinite(cm) & np.isfinite(cp)
    with np.errstate(invalid="ignore"):  # -inf - -inf where a pixel has no estimate
        den = np.where(inner, cm - 2 * cb + cp, 0.0)
        fit = inner & (den < 0)
        delta = np.where(fit, 0.5 * (cm - cp) / np.where(fit, den, 1.0), 0.0)
    step = (np.take_along_axis(d, np.full((1, H, W), n - 1), 0)[0] - d[0]) / (n - 1)
    dk = np.take_along_axis(d, kb[None], 0)[0] + delta * step
    depth = np.where(valid, 1.0 / dk, np.nan)
    return depth, kb, delta


def guided_depth(Fi, Fjs, K, poses, zmono, n: int = 32, mask=None):
    """Depth per pixel (nan: no estimate, also where Z* is not a positive
    finite number, and outside mask if given)."""
    zmono = np.asarray(zmono, np.float64)
    has = np.isfinite(zmono) & (zmono > 0)
    zsafe = np.where(has, zmono, 1.0)
    C, d, choice = correlations(Fi, Fjs, K, poses, zsafe, n, mask)
    C[:, ~has] = -np.inf
    choice = np.where(has, choice, -1)
    depth, kb, delta = refine(C, d)
    return dict(depth=depth, best=np.where(np.isfinite(depth), kb, -1), delta=delta, choice=choice, corr=C,
                cand=d)
