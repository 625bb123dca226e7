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
