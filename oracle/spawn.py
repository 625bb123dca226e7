"""Oracle of the primitive-spawning step (test infrastructure only).

Section 4.2 of the paper: a pixel's probability of spawning a Gaussian is
the clamped norm of the Laplacian-of-Gaussian response of the input image
(Eq. 1), reduced by the same quantity on the image rendered from the new
view (Eq. 2, zero on the first frame) and floored at zero (Eq. 3).  A spawned
Gaussian sits at the pixel's depth on its ray; its isotropic scale is the
expected nearest-neighbour distance of a 2D Poisson process whose intensity
is the pre-penalty probability (Clark-Evans), 1/(2 sqrt(P_L)) pixels,
converted to world units with depth / focal length.

Readings (the paper does not fix them): LoG with sigma = 1 px sampled on the
integer grid out to radius ceil(4 sigma), taps shifted to sum to zero,
replicated borders; L2 norm over the RGB responses of [0,1] images; P_L
floored at 1e-4 in the scale rule; opacity 0.1, the pixel's colour as the DC
term, rotation aligned with the camera axes.

Two forms:
* `*_f64` -- the definition in float64 (checked against closed forms).
* `probability_f32` -- the same arithmetic in binary32 with the operation
  order fixed (taps visited row by row, each product rounded then added;
  squares of R, G, B added in that order; correctly rounded sqrt).  The
  spawn decisions are integer functions of these values, so the path under
  test and this reference take them in the same precision and can be
  compared bit for bit.

Decisions:
* q(p) = floor(P_s(p) * 2^24) (exact in binary32 arithmetic);
* Bernoulli: spawn iff u(p) < q(p), u(p) the top 24 bits of SplitMix64
  applied to seed + p (counter-based, one draw per pixel index p);
* fixed-K: systematic sampling of the integer masses: with S = sum q and a
  24-bit offset o, threshold j = floor((j S + floor(S o / 2^24)) / K),
  j = 0..K-1; a pixel spawns once if any threshold falls inside its
  [prefix, prefix + q) interval.
"""
from __future__ import annotations

import math

import numpy as np

MASK64 = (1 << 64) - 1


def log_kernel_f64(sigma: float = 1.0):
    """Analytic LoG taps on the integer grid, radius ceil(4 sigma), shifted by
    their exactly rounded mean so that they sum to zero."""
    r = int(math.ceil(4 * sigma))
    n = 2 * r + 1
    k = np.zeros((n, n))
    for y in range(-r, r + 1):
        for x in range(-r, r + 1):
            rr = float(x * x + y * y)
            g = math.exp(-rr / (2 * sigma * sigma)) / (2 * math.pi * sigma * sigma)
            k[y + r, x + r] = (rr - 2 * sigma * sigma) / sigma ** 4 * g
    return k - math.fsum(k.ravel()) / (n * n)


def _padded(img, r):
    return np.pad(img, ((0, 0), (r, r), (r, r)), mode="edge")


def log_response_f64(img, sigma: float = 1.0):
    img = np.asarray(img, np.float64)
    k = log_kernel_f64(sigma)
    r = k.shape[0] // 2
    P = _padded(img, r)
    H, W = img.shape[1:]
    out = np.zeros_like(img)
    for dy in range(2 * r + 1):
        for dx in range(2 * r + 1):
            out += k[dy, dx] * P[:, dy:dy + H, dx:dx + W]
    return out


def prob_f64(img, rendered=None, sigma: float = 1.0):
    """(P_L, P_tilde, P_s) in float64."""
    L = log_response_f64(img, sigma)
    PL = np.minimum(np.sqrt((L * L).sum(0)), 1.0)
    if rendered is None:
        Pt = np.zeros_like(PL)
    else:
        Lt = log_response_f64(rendered, sigma)
        Pt = np.minimum(np.sqrt((Lt * Lt).sum(0)), 1.0)
    return PL, Pt, np.maximum(PL - Pt, 0.0)


def _norm_f32(img, taps):
    img = np.asarray(img, np.float32)
    r = taps.shape[0] // 2
    P = _padded(img, r)
    H, W = img.shape[1:]
    acc = np.zeros(img.shape, np.float32)
    for dy in range(2 * r + 1):
        for dx in range(2 * r + 1):
            acc = acc + taps[dy, dx] * P[:, dy:dy + H, dx:dx + W]
    sq = acc[0] * acc[0]
    sq = sq + acc[1] * acc[1]
    sq = sq + acc[2] * acc[2]
    return np.minimum(np.sqrt(sq), np.float32(1.0))


def probability_f32(img, rendered=None, sigma: float = 1.0):
    """(P_L, P_s) in binary32 with the fixed operation order."""
    taps = log_kernel_f64(sigma).astype(np.float32)
    PL = _norm_f32(img, taps)
    if rendered is None:
        return PL, PL.copy()
    Pt = _norm_f32(rendered, taps)
    return PL, np.maximum(PL - Pt, np.float32(0.0))


def splitmix64(x: int) -> int:
    """One step of SplitMix64 (Steele, Lea, Flood 2014): the output for state x."""
    z = (x + 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def uniform24(seed: int, count: int) -> np.ndarray:
    """u(p) for p = 0..count-1: top 24 bits of splitmix64(seed + p), the same
    steps as `splitmix64` on uint64 arrays (wrapping arithmetic)."""
    z = np.arange(count, dtype=np.uint64) + np.uint64(seed & MASK64)
    z = z + np.uint64(0x9E3779B97F4A7C15)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(40)).astype(np.int64)


def quantize(ps_f32):
    return np.floor(np.asarray(ps_f32, np.float32).astype(np.float64) * (1 << 24)).astype(np.int64)


def mask_bernoulli(q, seed: int):
    u = uniform24(seed, q.size).reshape(q.shape)
    return u < q


def mask_fixed_k(q, k: int, offset24: int):
    qf = np.asarray(q, np.int64).reshape(-1)
    S = int(qf.sum())
    sel = np.zeros(qf.size, bool)
    if S == 0 or k <= 0:
        return sel.reshape(np.shape(q))
    U = (S >> 24) * offset24 + (((S & 0xFFFFFF) * offset24) >> 24)
    prefix = np.concatenate([[0], np.cumsum(qf)[:-1]])
    for j in range(k):
        t = (j * S + U) // k  # exact Python integers
        p = int(np.searchsorted(prefix, t, side="right") - 1)
        while qf[p] == 0:  # the threshold falls in the next non-empty interval to the left
            p -= 1
        sel[p] = True
    return sel.reshape(np.shape(q))


def quat_from_rotation(Rm):
    """Unit quaternion (w, x, y, z) with w >= 0 of a rotation matrix."""
    m = np.asarray(Rm, np.float64)
    tr = m[0, 0] + m[1, 1] + m[2, 2]
    if tr > 0:
        s = math.sqrt(tr + 1.0) * 2
        q = [0.25 * s, (m[2, 1] - m[1, 2]) / s, (m[0, 2] - m[2, 0]) / s, (m[1, 0] - m[0, 1]) / s]
    elif m[0, 0] > m[1, 1] and m[0, 0] > m[2, 2]:
        s = math.sqrt(1.0 + m[0, 0] - m[1, 1] - m[2, 2]) * 2
        q = [(m[2, 1] - m[1, 2]) / s, 0.25 * s, (m[0, 1] + m[1, 0]) / s, (m[0, 2] + m[2, 0]) / s]
    elif m[1, 1] > m[2, 2]:
        s = math.sqrt(1.0 + m[1, 1] - m[0, 0] - m[2, 2]) * 2
        q = [(m[0, 2] - m[2, 0]) / s, (m[0, 1] + m[1, 0]) / s, 0.25 * s, (m[1, 2] + m[2, 1]) / s]
    else:
        s = math.sqrt(1.0 + m[2, 2] - m[0, 0] - m[1, 1]) * 2
        q = [(m[1, 0] - m[0, 1]) / s, (m[0, 2] + m[2, 0]) / s, (m[1, 2] + m[2, 1]) / s, 0.25 * s]
    q = np.array(q)
    return q if q[0] >= 0 else -q


def rule_attributes(pixels, PL, img, depth, R, t, fx, fy, cx, cy, opacity=0.1, min_prob=1e-4):
    """Gaussian parameters (FP64) spawned at flat pixel indices by the rule.

    mean = R^T (D ((u - cx)/fx, (v - cy)/fy, 1) - t); scale = D / (2 f sqrt(max(P_L, min_prob)))
    on three axes with f = sqrt(fx fy); colour = the pixel's as the DC SH term; opacity logit of
    `opacity`; rotation = the camera's axes (R^T)."""
    H, W = depth.shape
    pixels = np.asarray(pixels, np.int64)
    v, u = pixels // W, pixels % W
    D = np.asarray(depth, np.float64).reshape(-1)[pixels]
    pc = np.stack([D * (u - cx) / fx, D * (v - cy) / fy, D])
    R = np.asarray(R, np.float64)
    means = R.T @ (pc - np.asarray(t, np.float64)[:, None])
    f = math.sqrt(fx * fy)
    s = D / (2.0 * f * np.sqrt(np.maximum(np.asarray(PL, np.float64).reshape(-1)[pixels], min_prob)))
    log_scales = np.tile(np.log(s), (3, 1))
    q = quat_from_rotation(R.T)
    quats = np.tile(q[:, None], (1, len(pixels)))
    rgb = np.asarray(img, np.float64).reshape(3, -1)[:, pixels]
    sh0 = (rgb - 0.5) * 2.0 * math.sqrt(math.pi)
    logit = math.log(opacity / (1 - opacity))
    return dict(means=means, log_scales=log_scales, quats=quats,
                opacity_logits=np.full(len(pixels), logit), sh0=sh0)
