"""Pins of the anchor oracle: sizes of Gaussians placed at known distances
(closed form f S / D), the camera centre of a posed camera, the 40 % rule
at its boundary, the blending weight's pieces (1 below 1 - o, 1/2 at equal
distances, continuity at 1 - o, linear in between) and the opacity scaling
(sigmoid of the new logit is w times the old opacity).  Merging: the
selection against the published SplitMix64 generator and its rate, the
k nearest neighbours against scipy's k-d tree and a lattice with ties, the
owner of each absorbed neighbour against every claim, the merge of one and
of two identical Gaussians in closed form, and the merged mean and
covariance against Monte Carlo samples of the weighted mixture."""
import math

import numpy as np

from oracle import anchors as an
from oracle import spawn as _spawn


def test_sizes_at_known_distances():
    R, t = np.eye(3), np.zeros(3)
    # three Gaussians on the z axis-ish at distances 2, 10, 50 (means as [3][n])
    means = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [2.0, 10.0, 50.0]])
    log_scales = np.log(np.array([[0.01, 0.02, 0.5], [0.03, 0.01, 0.01], [0.005, 0.001, 0.002]]))
    # S = the largest axis scale: 0.03, 0.02, 0.5
    flags, fS, tD = an.small_flags(means, log_scales, R, t, f=1000.0)
    assert np.allclose(fS, [30.0, 20.0, 500.0]) and np.allclose(tD, [2.0, 10.0, 50.0])
    assert flags.tolist() == [False, False, False]
    flags, _, _ = an.small_flags(means, log_scales, R, t, f=80.0)
    assert flags.tolist() == [False, True, True]  # 1.2 px, 0.16 px, 0.8 px (tau = 1: size < 1 px)


def test_camera_centre_of_a_posed_camera():
    rng = np.random.default_rng(0)
    q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    R = q * np.sign(np.linalg.det(q))
    C = np.array([1.0, -2.0, 0.5])
    t = -R @ C  # world -> camera: p = R (x - C)
    assert np.allclose(an.camera_centre(R, t), C)
    # a Gaussian at distance 4 from the centre, scale 0.002, f = 1000: 0.5 px
    m = (C + np.array([0.0, 4.0, 0.0]))[:, None]
    flags, fS, tD = an.small_flags(m, np.log(np.full((3, 1), 0.002)), R, t, f=1000.0)
    assert np.allclose(fS / tD, 0.5) and flags.tolist() == [True]


def test_forty_percent_rule():
    n = 10
    means = np.vstack([np.zeros((2, n)), np.full((1, n), 10.0)])
    small, big = math.log(1e-4), math.log(1.0)
    for k, expect in [(4, False), (5, True)]:  # more than 40 %: 5 of 10 triggers, 4 does not
        ls = np.full((3, n), big)
        ls[:, :k] = small
        flags, count, fire = an.trigger(means, ls, np.eye(3), np.zeros(3), f=1000.0)
        assert count == k and fire == expect


def test_blend_weight_pieces():
    o = 0.1
    assert an.blend_weight(1.0, 2.0, o) == 1.0
    assert an.blend_weight(0.899, 1.0, o) == 1.0
    assert abs(an.blend_weight(1.0, 1.0, o) - 0.5) < 1e-15           # equal distances: half each
    assert abs(an.blend_weight(0.9, 1.0, o) - 1.0) < 1e-12            # continuous at r = 1 - o
    w1, w2 = an.blend_weight(0.92, 1.0, o), an.blend_weight(0.96, 1.0, o)
    assert abs((w1 - w2) - 0.04 * 0.5 / o) < 1e-12                    # linear with slope 0.5 / o


def test_opacity_scaling():
    lg = np.array([-3.0, 0.0, 2.5, 8.0])
    for w in (1.0, 0.5, 0.1):
        new = an.scale_opacity_logits(lg, w)
        assert np.allclose(1 / (1 + np.exp(-new)), w / (1 + np.exp(-lg)), rtol=1e-12)


# ------------------------------------------------------------ merging


def _params(rng, n, deg=1):
    return dict(means=rng.standard_normal((3, n)).astype(np.float32),
                log_scales=rng.normal(-3.0, 0.4, (3, n)).astype(np.float32),
                quats=rng.standard_normal((4, n)).astype(np.float32),
                opacity_logits=rng.standard_normal(n).astype(np.float32),
                sh=rng.standard_normal(((deg + 1) ** 2, 3, n)).astype(np.float32))


def test_merge_selection_follows_splitmix64_and_rate():
    rng = np.random.default_rng(1)
    fine = rng.random(20000) < 0.7
    cls = an.merge_classes(fine, 3, 12345)
    for i in range(0, 20000, 997):  # the scalar published generator, independently
        u = _spawn.splitmix64((12345 + i) & ((1 << 64) - 1)) >> 40
        want = an.CLS_OTHER if not fine[i] else (an.CLS_SEED if u < (1 << 24) // 4 else an.CLS_CAND)
        assert cls[i] == want
    rate = (cls == an.CLS_SEED).sum() / fine.sum()
    assert abs(rate - 0.25) < 0.02
    assert ((cls != an.CLS_OTHER) == fine).all()


def test_knn_matches_kdtree_and_lattice():
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(2)
    n = 2000
    means = rng.standard_normal((3, n)).astype(np.float32)
    cls = an.merge_classes(np.ones(n, bool), 3, 5)
    nbr = an.knn(means, cls, 3)
    cand = np.flatnonzero(cls == an.CLS_CAND)
    tree = cKDTree(means[:, cand].T.astype(np.float64))
    seeds = np.flatnonzero(cls == an.CLS_SEED)
    _, idx = tree.query(means[:, seeds].T.astype(np.float64), k=3)
    assert np.array_equal(nbr[seeds], cand[idx])
    assert (nbr[cls != an.CLS_SEED] == -1).all()
    # a lattice on a line at unit spacing: the selected point at 0 has
    # candidates at -2, -1, +1, +2 (equal pairs): ties go to the lower index
    xs = np.array([0.0, -1.0, 1.0, -2.0, 2.0, 5.0], np.float32)
    m = np.stack([xs, np.zeros(6, np.float32), np.zeros(6, np.float32)])
    cls = np.array([1, 2, 2, 2, 2, 2], np.int32)
    assert an.knn(m, cls, 3)[0].tolist() == [1, 2, 3]
    assert an.knn(m, cls, 5)[0].tolist() == [1, 2, 3, 4, 5]
    assert an.knn(m, cls, 7)[0].tolist() == [1, 2, 3, 4, 5, -1, -1]


def test_owners_are_the_nearest_claim():
    rng = np.random.default_rng(3)
    p = _params(rng, 600)
    cls, nbr, own, keep = an.merge_plan(p, rng.random(600) < 0.8, 3, 9)
    for j in np.flatnonzero(own >= 0):
        s = own[j]
        assert cls[j] == an.CLS_CAND and j in nbr[s]
        d_own = np.float32(an.sq_dist(p["means"], s, [j])[0])
        for t in np.flatnonzero((nbr == j).any(axis=1)):  # every claimant
            d = np.float32(an.sq_dist(p["means"], t, [j])[0])
            assert (d_own, s) <= (d, t)
    claimed = set(nbr[nbr >= 0].tolist())
    assert set(np.flatnonzero(own >= 0).tolist()) == claimed
    assert np.array_equal(keep, np.flatnonzero(own < 0))


def test_merge_of_one_and_of_two_identical():
    rng = np.random.default_rng(4)
    p = _params(rng, 5)
    one = an.merge_group(p, [2])
    assert np.allclose(one["mean"], p["means"][:, 2].astype(np.float64), rtol=0, atol=1e-15)
    assert np.allclose(one["cov"], an.covariance(p["log_scales"][:, 2], p["quats"][:, 2]), rtol=1e-12)
    o = 1.0 / (1.0 + np.exp(-np.float64(p["opacity_logits"][2])))
    assert abs(one["opacity"] - min(0.99, o)) < 1e-12
    for k in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        p[k][..., 3] = p[k][..., 2]
    two = an.merge_group(p, [2, 3])
    assert np.allclose(two["mean"], one["mean"], atol=1e-15) and np.allclose(two["cov"], one["cov"], rtol=1e-12)
    assert abs(two["opacity"] - min(0.99, 2 * o)) < 1e-12
    assert np.allclose(two["sh"], p["sh"][:, :, 2], rtol=1e-12)


def test_merge_preserves_mixture_moments_monte_carlo():
    # the merged mean and covariance are those of the weighted mixture,
    # checked by sampling the mixture (independent of the moment formulas)
    rng = np.random.default_rng(5)
    p = _params(rng, 4)
    p["means"] *= 0.05
    mem = [0, 1, 2, 3]
    got = an.merge_group(p, mem)
    o = 1.0 / (1.0 + np.exp(-p["opacity_logits"].astype(np.float64)))
    w = o * np.exp(p["log_scales"].astype(np.float64).sum(axis=0))
    N = 400000
    comp = rng.choice(4, N, p=w / w.sum())
    x = np.zeros((N, 3))
    for c in range(4):
        sel = comp == c
        L = np.linalg.cholesky(an.covariance(p["log_scales"][:, c], p["quats"][:, c]))
        x[sel] = p["means"][:, c].astype(np.float64) + rng.standard_normal((sel.sum(), 3)) @ L.T
    scale = np.sqrt(np.trace(got["cov"]))
    assert np.abs(x.mean(axis=0) - got["mean"]).max() < 5 * scale / np.sqrt(N)
    assert np.abs(np.cov(x.T) - got["cov"]).max() < 0.02 * np.abs(got["cov"]).max()
    # member order does not matter
    perm = an.merge_group(p, [3, 1, 0, 2])
    assert np.allclose(perm["mean"], got["mean"], rtol=1e-13) and np.allclose(perm["cov"], got["cov"], rtol=1e-12)
