"""Pins of the guided-matching depth oracle: reprojection through an identity
pose and a pure translation against closed forms, bilinear sampling exact on
linear fields and equal to the texel at integer points, the parabola vertex
of an exactly quadratic correlation, the candidate range of the paper's
formula, and recovery of a known plane's depth from two views whose features
are random Fourier features of the plane's texture coordinates."""
import numpy as np

from oracle import depth as gd


def test_candidates_span_the_inverse_depth_range():
    z = np.array([[2.0, 20.0]])
    d = gd.candidates(z, 5)
    assert np.allclose(d[:, 0, 0], [0.4, 0.45, 0.5, 0.55, 0.6])
    # 1/20 - 0.1 < 0: the lower end is raised to d_min
    assert np.isclose(d[0, 0, 1], gd.D_MIN) and np.isclose(d[-1, 0, 1], 0.15)


def test_reprojection_closed_forms():
    K = (100.0, 90.0, 31.5, 23.5)
    I = np.eye(3)
    x, y, d = np.array([3.0, 40.0]), np.array([7.0, 11.0]), np.array([0.5, 0.1])
    u, v, z = gd.reproject(K, I, [0, 0, 0], x, y, d)
    assert np.allclose(u, x) and np.allclose(v, y) and np.allclose(z, 1 / d)
    # a translation by b along the camera's x axis shifts by f b d (disparity)
    b = 0.2
    u, v, z = gd.reproject(K, I, [-b, 0, 0], x, y, d)
    assert np.allclose(u, x - K[0] * b * d) and np.allclose(v, y)


def test_bilinear_exact_on_linear_fields():
    H, W = 9, 13
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    F = np.stack([2 * xx - yy + 1, 0.5 * yy, np.ones_like(xx)], -1)
    rng = np.random.default_rng(0)
    u, v = rng.uniform(0, W - 1, 50), rng.uniform(0, H - 1, 50)
    s = gd.bilinear(F, u, v)
    assert np.allclose(s[:, 0], 2 * u - v + 1) and np.allclose(s[:, 1], 0.5 * v) and np.allclose(s[:, 2], 1)
    s = gd.bilinear(F, np.array([4.0]), np.array([6.0]))
    assert np.array_equal(s[0], F[6, 4])
    # half a pixel outside: the outer taps count as zero
    s = gd.bilinear(F, np.array([-0.5]), np.array([0.0]))
    assert np.allclose(s[0], 0.5 * F[0, 0])


def test_parabola_vertex_of_a_quadratic_correlation():
    n = 9
    k0 = np.array([[3.3, 5.0, 1.5]])
    kk = np.arange(n, dtype=np.float64)[:, None, None]
    C = -(kk - k0[None]) ** 2
    d = np.broadcast_to(0.2 + 0.05 * kk, (n, 1, 3)).copy()
    depth, kb, delta = gd.refine(C, d)
    assert kb.tolist() == [[3, 5, 1]]  # 1.5: the tie goes to the lower k
    assert np.allclose(kb + delta, k0)
    assert np.allclose(depth, 1 / (0.2 + 0.05 * k0))


def _plane_views(Z, b, H=40, W=128, C=32, seed=0):
    """Fronto-parallel plane at depth Z; frame j is frame i moved by b along
    x.  Features: random Fourier features of the plane point (X, Y)."""
    rng = np.random.default_rng(seed)
    K = (300.0, 300.0, (W - 1) / 2, (H - 1) / 2)
    om = rng.normal(0, 60.0, (C, 2))  # periods of ~10 px at this depth and focal length
    ph = rng.uniform(0, 2 * np.pi, C)
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)

    def feats(shift):
        X = (xx - K[2]) / K[0] * Z + shift
        Y = (yy - K[3]) / K[1] * Z
        f = np.sqrt(2.0 / C) * np.cos(X[..., None] * om[:, 0] + Y[..., None] * om[:, 1] + ph)
        return f.astype(np.float16)

    Fi = feats(0.0)
    Fj = feats(b)  # camera j at world x = b sees world X at its pixel x - f b / Z
    return K, Fi, Fj


def test_recovers_a_known_plane():
    # the search range spans f b 0.2 = 18 px of disparity, 0.58 px per candidate
    Z, b = 2.5, 0.3
    K, Fi, Fj = _plane_views(Z, b)
    H, W, _ = Fi.shape
    zmono = np.full((H, W), Z * 1.15)  # the monocular depth is 15 % off
    R, t = np.eye(3), np.array([-b, 0.0, 0.0])
    out = gd.guided_depth(Fi, [Fj], K, [(R, t)], zmono, n=32)
    ok = np.isfinite(out["depth"])
    assert ok.mean() > 0.5  # the rest see the candidate segment leave the neighbour's image
    err = np.abs(out["depth"][ok] / Z - 1)
    # candidate spacing in inverse depth is 0.2 / 31 ~ 1.6 % of 1/Z here
    assert np.median(err) < 0.01 and np.mean(err < 0.02) > 0.95
    assert (out["choice"][ok] == 0).all()


def test_choice_prefers_the_wider_baseline():
    Z = 2.5
    K, Fi, Fj = _plane_views(Z, 0.02)
    H, W, _ = Fi.shape
    zmono = np.full((H, W), Z)
    poses = [(np.eye(3), np.array([-0.01, 0.0, 0.0])), (np.eye(3), np.array([-0.02, 0.0, 0.0]))]
    ch = gd.choose_neighbour(K, poses, zmono, 32, W, H)
    # the nearest candidate (inverse depth 0.5) shifts by f b 0.5 = 1.5 and 3 px to the left:
    # columns >= 3 keep both segments inside and take the wider baseline, columns 2 only the
    # narrower one, columns 0-1 neither
    assert (ch[:, 3:] == 1).all() and (ch[:, 2] == 0).all() and (ch[:, :2] == -1).all()
