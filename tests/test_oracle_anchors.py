"""Pins of the anchor oracle: sizes of Gaussians placed at known distances
(closed form f S / D), the camera centre of a posed camera, the 40 % rule
at its boundary, the blending weight's pieces (1 below 1 - o, 1/2 at equal
distances, continuity at 1 - o, linear in between) and the opacity scaling
(sigmoid of the new logit is w times the old opacity)."""
import math

import numpy as np

from oracle import anchors as an


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
