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

from oracle.spawn import uniform24


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


# --------------------------------------------------------------- merging
# Clustering and primitive merging (section 4.4): a random share 1/(k+1)
# of the too-fine primitives is selected, each selected primitive is
# merged with its k nearest neighbours (k = 3), all others stay unchanged.
# Readings where the paper is silent:
#  * selection: Bernoulli with probability floor(2^24 / (k+1)) / 2^24 per
#    fine primitive, drawn from the counter-based SplitMix64 stream
#    (top 24 bits of splitmix64(seed + index));
#  * neighbours: the k nearest fine, unselected primitives by the squared
#    distance of their means, d2 = (dx dx + dy dy) + dz dz in binary64 on the
#    binary32 means (dx exact), ties to the lower index;
#  * a neighbour claimed by several selected primitives joins the one with
#    the smallest (binary32-rounded d2, selected index) -- a decision both
#    sides take in binary32;
#  * merge (the hierarchical 3DGS merge): weights w_i = o_i s_x s_y s_z
#    (opacity times the volume factor sqrt(det Sigma_i)), mean and second
#    moment preserved: mu = sum w mu / W, Sigma = sum w (Sigma_i +
#    (mu_i - mu)(mu_i - mu)^T) / W, SH coefficients weighted the same way,
#    opacity o = min(0.99, W / sqrt(det Sigma)) (the merged splat keeps the
#    group's opacity-weighted volume up to the cap); a selected primitive
#    that receives no neighbour stays unchanged;
#  * the new active set keeps the original order: each selected primitive's
#    merged Gaussian takes its place, absorbed neighbours are removed.

CLS_OTHER, CLS_SEED, CLS_CAND = 0, 1, 2


def merge_classes(fine, k: int, seed: int):
    """Per Gaussian: CLS_SEED (selected fine), CLS_CAND (fine, not selected)
    or CLS_OTHER."""
    fine = np.asarray(fine) != 0
    thr = (1 << 24) // (k + 1)
    u = uniform24(seed, fine.size)
    cls = np.where(fine, np.where(u < thr, CLS_SEED, CLS_CAND), CLS_OTHER).astype(np.int32)
    return cls


def sq_dist(means, i, js):
    """binary64 squared distances from Gaussian i to Gaussians js, in the
    order (dx dx + dy dy) + dz dz with each operation rounded once."""
    m = np.asarray(means, np.float32)
    return _sq_dist64(m[:, js].astype(np.float64), m[:, i:i + 1].astype(np.float64))


def _sq_dist64(a, b):
    d = a - b
    return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]


def knn(means, cls, k: int):
    """[n][k] int32: for each selected Gaussian its k nearest candidates
    (brute force over all candidates, ascending (d2, index)), -1 padded;
    rows of other Gaussians are -1."""
    cls = np.asarray(cls)
    m64 = np.asarray(means, np.float32).astype(np.float64)
    cand = np.flatnonzero(cls == CLS_CAND)
    cm = m64[:, cand]
    out = np.full((cls.size, k), -1, np.int32)
    for s in np.flatnonzero(cls == CLS_SEED):
        if cand.size == 0:
            continue
        d2 = _sq_dist64(cm, m64[:, s:s + 1])
        if cand.size > k:  # every candidate up to the k-th smallest distance (ties included)
            sel = np.flatnonzero(d2 <= np.partition(d2, k - 1)[k - 1])
        else:
            sel = np.arange(cand.size)
        order = sel[np.lexsort((cand[sel], d2[sel]))][:k]
        out[s, :order.size] = cand[order]
    return out


def owners(means, cls, nbr):
    """[n] int32: for each candidate, the selected Gaussian it joins (the
    claim with the smallest (binary32 d2, selected index)), else -1."""
    n = np.asarray(cls).size
    best = {}
    for s in np.flatnonzero(np.asarray(cls) == CLS_SEED):
        js = nbr[s][nbr[s] >= 0]
        if js.size == 0:
            continue
        d2 = sq_dist(means, s, js).astype(np.float32)
        for j, d in zip(js, d2):
            key = (float(d), int(s))
            if int(j) not in best or key < best[int(j)]:
                best[int(j)] = key
    own = np.full(n, -1, np.int32)
    for j, (_, s) in best.items():
        own[j] = s
    return own


def _quat_rot(q):
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def covariance(log_scales, quat):
    R = _quat_rot(np.asarray(quat, np.float64))
    s2 = np.exp(2.0 * np.asarray(log_scales, np.float64))
    return R @ np.diag(s2) @ R.T


def merge_group(params, members):
    """The merged Gaussian of members (indices into the SoA planes of
    params: means [3][n], log_scales [3][n], quats [4][n],
    opacity_logits [n], sh [b][3][n]): dict with mean, cov, opacity (the
    capped value), sh [b][3], and the weight sum W."""
    m = np.asarray(params["means"], np.float64)[:, members]
    ls = np.asarray(params["log_scales"], np.float64)[:, members]
    q = np.asarray(params["quats"], np.float64)[:, members]
    a = np.asarray(params["opacity_logits"], np.float64)[members]
    sh = np.asarray(params["sh"], np.float64)[:, :, members]
    o = 1.0 / (1.0 + np.exp(-a))
    w = o * np.exp(ls.sum(axis=0))
    W = w.sum()
    mu = (m * w).sum(axis=1) / W
    cov = np.zeros((3, 3))
    for c in range(len(members)):
        d = m[:, c] - mu
        cov += w[c] * (covariance(ls[:, c], q[:, c]) + np.outer(d, d))
    cov /= W
    op = min(0.99, W / np.sqrt(np.linalg.det(cov)))
    return dict(mean=mu, cov=cov, opacity=op, sh=(sh * w).sum(axis=2) / W, W=W)


def merge_plan(params, fine, k: int, seed: int):
    """(cls, nbr, owner, keep) of the merge; keep = ascending source indices
    of the new active set."""
    cls = merge_classes(fine, k, seed)
    nbr = knn(params["means"], cls, k)
    own = owners(params["means"], cls, nbr)
    keep = np.flatnonzero(own < 0).astype(np.int32)
    return cls, nbr, own, keep


def merge_groups(params, cls, own):
    """{selected index: merged Gaussian} for every selected Gaussian that
    received at least one neighbour."""
    groups = {}
    for j in np.flatnonzero(own >= 0):
        groups.setdefault(int(own[j]), []).append(int(j))
    return {s: merge_group(params, [s] + sorted(js)) for s, js in groups.items()}
