"""Oracle of the multi-scale training helpers of the joint optimisation
(section 4.3), test infrastructure only.

* Coarse-to-fine: a newly added image first trains at 2^l downsampling
  (l = 3) and l drops by one every five iterations until full size.  The
  coarse image is the box-filtered copy: coarse pixel (x, y) is the mean of
  the fine pixels (s x + j, s y + i), i, j < s = 2^l; the right and bottom
  remainders that do not fill a block are dropped.  With pixel centres at
  integer coordinates the coarse pixel's centre sits at the centroid
  s x + (s - 1) / 2 of its fine pixels, so the coarse camera has
  f' = f / s and c' = (c + 1/2) / s - 1/2.
* Opacity culling (as in 3DGS): a Gaussian is removed when its opacity
  sigmoid(logit) is below the threshold t.  The decision is taken in
  binary32 on the logit: kept iff logit >= thr, thr = binary32 rounding of
  ln(t / (1 - t)) computed in binary64 (sigmoid is increasing, so this is
  the opacity test up to the rounding of thr).  The kept Gaussians keep
  their order.
"""
from __future__ import annotations

import math

import numpy as np


def level_at(iteration: int, start_level: int = 3, every: int = 5) -> int:
    """Downsampling level of a newly added image at a joint iteration."""
    return max(0, start_level - iteration // every)


def downsample(image, level: int):
    """[C][H][W] -> [C][H >> level][W >> level] block means (FP64)."""
    img = np.asarray(image, np.float64)
    s = 1 << level
    c, h, w = img.shape
    hc, wc = h // s, w // s
    blocks = img[:, :hc * s, :wc * s].reshape(c, hc, s, wc, s)
    return blocks.mean(axis=(2, 4))


def camera_level(width, height, fx, fy, cx, cy, level: int):
    """Image size and intrinsics of the 2^level-downsampled camera."""
    s = float(1 << level)
    return (width >> level, height >> level, fx / s, fy / s, (cx + 0.5) / s - 0.5, (cy + 0.5) / s - 0.5)


def opacity_threshold_logit(min_opacity: float) -> np.float32:
    return np.float32(math.log(min_opacity / (1.0 - min_opacity)))


def prune_keep(opacity_logits, min_opacity: float):
    """Ascending indices of the Gaussians opacity culling keeps."""
    lg = np.asarray(opacity_logits, np.float32)
    return np.nonzero(lg >= opacity_threshold_logit(min_opacity))[0]


def gather_planes(src, index):
    """[P][n] planes -> [P][m]: column j is column index[j] of src."""
    return np.asarray(src)[:, np.asarray(index, np.int64)]


# ------------------------------------------------ 3D smoothing filter
# Mip-Splatting's 3D smoothing filter, which the paper's "proper filtering"
# of multi-scale training cites: each Gaussian is convolved with an
# isotropic 3D Gaussian low-pass of variance v = (s_f / nu)^2, nu the
# highest sampling rate (pixels per world unit, f / depth) at which any
# training camera sees it, s_f a constant (0.2 in Mip-Splatting).  The
# convolution adds v to the covariance, i.e. to each axis variance in the
# same rotation, and the opacity is scaled so that the Gaussian's integral
# o sqrt(det Sigma) is unchanged:
#   s'_k^2 = s_k^2 + v,   o' = o prod_k s_k / s'_k.


def sampling_rate(means, R, t, fx, fy, cx, cy, width, height, near=0.2, guard=1.15):
    """Per Gaussian: fx / z in the camera when its mean lies in front of the
    near plane and inside the image widened by `guard` (Mip-Splatting's
    1.15 screen margin), else 0 (FP64)."""
    m = np.asarray(means, np.float32).astype(np.float64)
    p = np.asarray(R, np.float64) @ m + np.asarray(t, np.float64)[:, None]
    z = p[2]
    with np.errstate(divide="ignore", invalid="ignore"):
        u = fx * p[0] / z + cx
        v = fy * p[1] / z + cy
        inside = (z > near) & (u >= -(guard - 1) / 2 * width) & (u <= (guard + 1) / 2 * width) & \
                 (v >= -(guard - 1) / 2 * height) & (v <= (guard + 1) / 2 * height)
        return np.where(inside, fx / z, 0.0)


def filter_variance(nu_max, s_f: float = 0.2):
    """(s_f / nu)^2 where a camera saw the Gaussian, else 0."""
    nu = np.asarray(nu_max, np.float64)
    with np.errstate(divide="ignore"):
        return np.where(nu > 0, (s_f / np.where(nu > 0, nu, 1.0)) ** 2, 0.0)


def apply_filter3d(log_scales, opacity_logits, var):
    """The filtered Gaussian as (log-scales', opacity logit') in FP64."""
    ls = np.asarray(log_scales, np.float64)
    a = np.asarray(opacity_logits, np.float64)
    v = np.asarray(var, np.float64)
    ls2 = 0.5 * np.log(np.exp(2.0 * ls) + v)
    o = 1.0 / (1.0 + np.exp(-a))
    o2 = o * np.exp((ls - ls2).sum(axis=0))
    return ls2, np.log(o2) - np.log1p(-o2)


def filter3d_vjp(log_scales, opacity_logits, var, g_ls2, g_logit2):
    """Gradients with respect to (log-scales, logit) from those with respect
    to the filtered (log-scales', logit'), by the chain rule of
    apply_filter3d."""
    ls = np.asarray(log_scales, np.float64)
    a = np.asarray(opacity_logits, np.float64)
    v = np.asarray(var, np.float64)
    s2 = np.exp(2.0 * ls)
    ls2 = 0.5 * np.log(s2 + v)
    o = 1.0 / (1.0 + np.exp(-a))
    f = np.exp((ls - ls2).sum(axis=0))
    o2 = o * f
    g_o2 = np.asarray(g_logit2, np.float64) / (o2 * (1.0 - o2))  # d logit' / d o' = 1 / (o'(1 - o'))
    dls2 = s2 / (s2 + v)  # d ls'_k / d ls_k
    g_ls = np.asarray(g_ls2, np.float64) * dls2 + g_o2 * o2 * (1.0 - dls2)
    g_a = g_o2 * f * o * (1.0 - o)
    return g_ls, g_a
