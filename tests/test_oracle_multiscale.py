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


def test_filter3d_closed_forms_and_invariant():
    rng = np.random.default_rng(31)
    n = 50
    ls = rng.normal(-3, 0.6, (3, n))
    a = rng.normal(0, 1, n)
    v = rng.uniform(0, 0.01, n)
    ls2, a2 = ms.apply_filter3d(ls, a, v)
    # each axis variance grows by v, the same rotation
    assert np.allclose(np.exp(2 * ls2), np.exp(2 * ls) + v, rtol=1e-13)
    # the integral o sqrt(det Sigma) = o prod s_k is unchanged
    o = 1 / (1 + np.exp(-a))
    o2 = 1 / (1 + np.exp(-a2))
    assert np.allclose(o2 * np.exp(ls2.sum(0)), o * np.exp(ls.sum(0)), rtol=1e-12)
    # an isotropic Gaussian of scale s: o' = o (s^2 / (s^2 + v))^(3/2)
    s = 0.05
    iso = np.full((3, 1), np.log(s))
    _, ai = ms.apply_filter3d(iso, np.array([0.3]), np.array([0.0004]))
    oi = 1 / (1 + np.exp(-ai[0]))
    assert abs(oi - (1 / (1 + np.exp(-0.3))) * (s * s / (s * s + 0.0004)) ** 1.5) < 1e-14
    # v = 0 is the identity
    l0, a0 = ms.apply_filter3d(ls, a, np.zeros(n))
    assert np.allclose(l0, ls, atol=1e-15) and np.allclose(a0, a, atol=1e-12)


def test_filter3d_vjp_finite_differences():
    rng = np.random.default_rng(32)
    n = 20
    ls = rng.normal(-3, 0.6, (3, n))
    a = rng.normal(0, 1, n)
    v = rng.uniform(1e-4, 4e-3, n)
    w_ls = rng.standard_normal((3, n))
    w_a = rng.standard_normal(n)
    loss = lambda L, A: (w_ls * ms.apply_filter3d(L, A, v)[0]).sum() + \
        (w_a * ms.apply_filter3d(L, A, v)[1]).sum()
    g_ls, g_a = ms.filter3d_vjp(ls, a, v, w_ls, w_a)
    h = 1e-6
    for k in range(3):
        for i in range(0, n, 3):
            d = np.zeros_like(ls)
            d[k, i] = h
            fd = (loss(ls + d, a) - loss(ls - d, a)) / (2 * h)
            assert abs(fd - g_ls[k, i]) <= 1e-6 * (1 + abs(fd))
    for i in range(n):
        d = np.zeros(n)
        d[i] = h
        fd = (loss(ls, a + d) - loss(ls, a - d)) / (2 * h)
        assert abs(fd - g_a[i]) <= 1e-6 * (1 + abs(fd))


def test_sampling_rate_brute_force():
    rng = np.random.default_rng(33)
    m = rng.uniform([-3, -2, -1], [3, 2, 8], (300, 3)).T.astype(np.float32)
    R, t = np.eye(3), np.zeros(3)
    W, H, f = 160, 120, 100.0
    nu = ms.sampling_rate(m, R, t, f, f, W / 2, H / 2, W, H)
    for i in range(m.shape[1]):
        x, y, z = (float(c) for c in m[:, i].astype(np.float64))
        u, vv = (f * x / z + W / 2, f * y / z + H / 2) if z > 0 else (0, 0)
        inside = z > 0.2 and -0.075 * W <= u <= 1.075 * W and -0.075 * H <= vv <= 1.075 * H
        assert nu[i] == (f / z if inside else 0.0)
    var = ms.filter_variance(np.array([0.0, 100.0, 400.0]))
    assert var[0] == 0.0 and abs(var[1] - 4e-6) < 1e-20 and abs(var[2] - 2.5e-7) < 1e-21
