"""Oracle of the anchor decisions of the scalable construction (section
4.4), test infrastructure only.

* Creation trigger: the size of a primitive seen from a camera is S / D,
  S its scale and D the distance of its centre to the camera centre; read
  here as S = the largest of its three axis scales and the size in pixels
  f S / D with f = sqrt(fx fy).  An anchor is created when more than 40 %
  of the active Gaussians are smaller than tau_min = 1 pixel from the
  previous camera.  The per-Gaussian test f S < tau D is taken in binary64
  with S = exp(max log-scale) and D = |mu - C|.
* Blending: with the two nearest anchors at distances d1 <= d2 and overlap
  o in (0, 0.5), r = d1 / d2 and the nearer anchor's weight is 1 for
  r < 1 - o and 1 - (r - (1 - o)) 0.5 / o otherwise; the other anchor gets
  the complement.  A weight w applied to a Gaussian set scales its
  opacities: logit' = logit(w sigmoid(logit)).
"""
from __future__ import annotations

import numpy as np


def camera_centre(R, t):
    return -np.asarray(R, np.float64).T @ np.asarray(t, np.float64)


def small_flags(means, log_scales, R, t, f: float, tau: float = 1.0):
    """Per Gaussian: smaller than tau pixels from the camera (FP64)."""
    C = camera_centre(R, t)
    D = np.linalg.norm(np.asarray(means, np.float64) - C[:, None], axis=0)
    S = np.exp(np.max(np.asarray(log_scales, np.float64), axis=0))
    return f * S < tau * D, f * S, tau * D


def trigger(means, log_scales, R, t, f: float, tau: float = 1.0, share: float = 0.4):
    flags, _, _ = small_flags(means, log_scales, R, t, f, tau)
    n = flags.size
    return flags, int(flags.sum()), (n > 0 and flags.sum() > share * n)


def blend_weight(d1: float, d2: float, o: float) -> float:
    r = d1 / d2
    if r < 1.0 - o:
        return 1.0
    return 1.0 - (r - (1.0 - o)) * 0.5 / o


def scale_opacity_logits(logits, w: float):
    op = 1.0 / (1.0 + np.exp(-np.asarray(logits, np.float64)))
    q = w * op
    with np.errstate(divide="ignore"):
        return np.log(q) - np.log1p(-q)
