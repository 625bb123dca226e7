"""Pins of the multi-scale oracle: closed forms of the box filter (constant
and linear images, whose block means are the value at the block centroid),
brute force on a tiny image, the schedule the paper states (2^3 first, one
level less every five iterations), the camera of a level against the
centroid of a coarse pixel's fine pixels, and the opacity test against the
sigmoid away from the threshold."""
import math

import numpy as np

from oracle import multiscale as ms


def test_schedule_three_levels_then_full_size():
    levels = [ms.level_at(i) for i in range(30)]
    assert levels[:5] == [3] * 5 and levels[5:10] == [2] * 5 and levels[10:15] == [1] * 5
    assert levels[15:] == [0] * 15


def test_box_filter_constant_and_linear_images():
    h, w = 37, 53  # ragged: the remainders are dropped
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    img = np.stack([np.full((h, w), 0.3), 0.01 * xx + 0.02 * yy + 0.1, -0.5 * xx + 3.0])
    for level in range(4):
        s = 1 << level
        out = ms.downsample(img, level)
        assert out.shape == (3, h // s, w // s)
        cy, cx = np.mgrid[0:h // s, 0:w // s].astype(np.float64)
        # centroid of the block's fine pixel centres
        gx, gy = s * cx + (s - 1) / 2, s * cy + (s - 1) / 2
        assert np.allclose(out[0], 0.3, atol=1e-15)
        assert np.allclose(out[1], 0.01 * gx + 0.02 * gy + 0.1, atol=1e-13)
        assert np.allclose(out[2], -0.5 * gx + 3.0, atol=1e-12)


def test_box_filter_brute_force_tiny():
    rng = np.random.default_rng(0)
    img = rng.random((2, 9, 11))
    out = ms.downsample(img, 1)
    for c in range(2):
        for y in range(4):
            for x in range(5):
                ref = (img[c, 2 * y, 2 * x] + img[c, 2 * y, 2 * x + 1] + img[c, 2 * y + 1, 2 * x] +
                       img[c, 2 * y + 1, 2 * x + 1]) / 4
                assert abs(out[c, y, x] - ref) < 1e-15


def test_camera_level_maps_block_centroids_to_coarse_centres():
    W, H, fx, fy, cx, cy = 1920, 1080, 1100.0, 1050.0, 959.5, 539.5
    rng = np.random.default_rng(1)
    for level in (1, 2, 3):
        s = 1 << level
        w2, h2, fx2, fy2, cx2, cy2 = ms.camera_level(W, H, fx, fy, cx, cy, level)
        assert (w2, h2) == (W // s, H // s)
        for _ in range(20):
            X = np.array([rng.uniform(-2, 2), rng.uniform(-1, 1), rng.uniform(2, 10)])
            u, v = fx * X[0] / X[2] + cx, fy * X[1] / X[2] + cy
            u2, v2 = fx2 * X[0] / X[2] + cx2, fy2 * X[1] / X[2] + cy2
            # a point on the centroid of coarse pixel (i, j)'s fine pixels
            # lands on that coarse pixel's centre: u = s u2 + (s - 1) / 2
            assert abs(u - (s * u2 + (s - 1) / 2)) < 1e-9 and abs(v - (s * v2 + (s - 1) / 2)) < 1e-9


def test_opacity_culling_matches_sigmoid_away_from_threshold():
    rng = np.random.default_rng(2)
    t = 0.005
    thr = math.log(t / (1 - t))
    lg = rng.uniform(-12, 4, 5000)
    lg = lg[np.abs(lg - thr) > 1e-4].astype(np.float32)
    keep = ms.prune_keep(lg, t)
    op = 1 / (1 + np.exp(-lg.astype(np.float64)))
    assert np.array_equal(keep, np.nonzero(op >= t)[0])
    assert np.all(np.diff(keep) > 0)
    # known values: logit(0.005) = -5.2933...
    assert ms.prune_keep(np.array([-6.0, -5.0, -5.3, -5.29], np.float32), t).tolist() == [1, 3]
    assert abs(float(ms.opacity_threshold_logit(t)) - (-5.293304824724492)) < 1e-6


def test_gather_keeps_order_and_planes():
    src = np.arange(3 * 8, dtype=np.float32).reshape(3, 8)
    out = ms.gather_planes(src, [0, 2, 7])
    assert out.tolist() == [[0, 2, 7], [8, 10, 15], [16, 18, 23]]
