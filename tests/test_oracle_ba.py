"""Pins of the mini bundle adjustment oracle (oracle/ba.py): the SE(3)
left update against scipy's matrix exponential of the twist, the pose and
bundle Jacobians against central finite differences, the Huber loss and its
weights, the median + 4 MAD rule on known values, the damping schedule of
the appendix (lambda 1e-5, divided by 2 after a step that lowers the cost,
doubled otherwise) read from the trace, a pose recovered exactly from
noise-free correspondences, RANSAC finding the true inliers among 30 %
outliers, and the bootstrapping recovering focal length, poses and structure
(up to the scale the gauge leaves free) from noise-free observations."""
import numpy as np
import pytest
from scipy.linalg import expm

from oracle import ba


def _twist_matrix(xi):
    M = np.zeros((4, 4))
    M[:3, :3] = ba.hat(xi[3:])
    M[:3, 3] = xi[:3]
    return M


def test_se3_left_update_matches_matrix_exponential():
    rng = np.random.default_rng(0)
    for scale in (1e-9, 1e-3, 0.3, 2.0):
        R0 = ba.so3_exp(rng.standard_normal(3))
        t0 = rng.standard_normal(3)
        xi = rng.standard_normal(6) * scale
        R, t = ba.se3_left_update(R0, t0, xi)
        T0 = np.eye(4)
        T0[:3, :3], T0[:3, 3] = R0, t0
        T = expm(_twist_matrix(xi)) @ T0
        assert np.allclose(R, T[:3, :3], atol=1e-12) and np.allclose(t, T[:3, 3], atol=1e-12)


def _scene(rng, K=200):
    X = np.stack([rng.uniform(-1, 1, K), rng.uniform(-1, 1, K), rng.uniform(3, 6, K)])
    R = ba.so3_exp(rng.standard_normal(3) * 0.05)
    t = rng.standard_normal(3) * 0.1
    return X, R, t


def test_pose_jacobian_finite_differences():
    rng = np.random.default_rng(1)
    X, R, t = _scene(rng, 5)
    f, cx, cy = 500.0, 320.0, 240.0
    _, p = ba.project(R, t, X, f, f, cx, cy)
    J = ba.pose_jacobian(p, f, f)
    h = 1e-6
    for j in range(6):
        e = np.zeros(6)
        e[j] = h
        up = ba.project(*ba.se3_left_update(R, t, e), X, f, f, cx, cy)[0]
        dn = ba.project(*ba.se3_left_update(R, t, -e), X, f, f, cx, cy)[0]
        fd = (up - dn) / (2 * h)
        assert np.allclose(J[:, :, j].T, fd, rtol=1e-6, atol=1e-6)


def test_bundle_jacobian_finite_differences():
    rng = np.random.default_rng(2)
    V, P, W, H = 3, 4, 640, 480
    cx, cy = W / 2, H / 2
    f = 430.0
    Rs = [np.eye(3)] + [ba.so3_exp(rng.standard_normal(3) * 0.05) for _ in range(V - 1)]
    ts = [np.zeros(3)] + [rng.standard_normal(3) * 0.1 for _ in range(V - 1)]
    X = np.stack([rng.uniform(-1, 1, P), rng.uniform(-1, 1, P), rng.uniform(3, 6, P)])
    uv = np.zeros((V, 2, P))
    r0, ps = ba.ba_residuals(f, Rs, ts, X, uv, cx, cy)
    J = ba.ba_jacobian(f, Rs, ps, X)
    nc = 1 + 6 * (V - 1)
    h = 1e-6

    def stacked(f_, Rs_, ts_, X_):
        r, _ = ba.ba_residuals(f_, Rs_, ts_, X_, uv, cx, cy)
        return r.transpose(0, 2, 1).reshape(-1)

    for col in range(nc + 3 * P):
        def perturbed(s):
            f_, Rs_, ts_, X_ = f, list(Rs), list(ts), X.copy()
            if col == 0:
                f_ = f + s
            elif col < nc:
                v, j = 1 + (col - 1) // 6, (col - 1) % 6
                e = np.zeros(6)
                e[j] = s
                Rs_[v], ts_[v] = ba.se3_left_update(Rs[v], ts[v], e)
            else:
                k, a = (col - nc) // 3, (col - nc) % 3
                X_[a, k] += s
            return stacked(f_, Rs_, ts_, X_)
        fd = (perturbed(h) - perturbed(-h)) / (2 * h)
        assert np.allclose(J[:, col], fd, rtol=1e-5, atol=1e-5), col


def test_huber_and_mad_known_values():
    e = np.array([0.0, 0.5, 1.0, 3.0])
    assert np.allclose(ba.huber(e, 1.0), [0.0, 0.125, 0.5, 2.5])
    assert np.allclose(ba.huber_weight(e, 1.0), [1.0, 1.0, 1.0, 1.0 / 3.0])
    # median 3, |e - 3| = 2 1 0 1 2 97 -> MAD 1.5: keep e <= 9
    err = np.array([1.0, 2.0, 3.0, 4.0, 5.0, 100.0])
    assert ba.mad_keep(err).tolist() == [True, True, True, True, True, False]
    assert ba.mad_keep(np.full(5, 2.0)).all()


def test_damping_schedule_from_the_trace():
    rng = np.random.default_rng(3)
    X, R, t = _scene(rng)
    f, cx, cy = 500.0, 320.0, 240.0
    uv, _ = ba.project(R, t, X, f, f, cx, cy)
    for robust in (True, False):
        trace = []
        ba.lm_pose(X, uv, np.eye(3), np.zeros(3), f, f, cx, cy, 12, delta=1.0, robust=robust, trace=trace)
        assert trace[0]["lam"] == 1e-5
        for a, b in zip(trace, trace[1:]):
            assert b["lam"] == (a["lam"] / 2 if a["accepted"] else a["lam"] * 2)
            assert a["accepted"] == (a["cost_new"] < a["cost"])
            if not robust:  # without the per-iteration rejection the cost carries over exactly
                assert b["cost"] == pytest.approx(a["cost_new"] if a["accepted"] else a["cost"], rel=1e-12)


def test_pose_recovered_from_exact_correspondences():
    rng = np.random.default_rng(4)
    X, R, t = _scene(rng)
    f, cx, cy = 500.0, 320.0, 240.0
    uv, _ = ba.project(R, t, X, f, f, cx, cy)
    Rg, tg, _ = ba.lm_pose(X, uv, np.eye(3), np.zeros(3), f, f, cx, cy, 20, delta=1.0)
    assert np.allclose(Rg, R, atol=1e-9) and np.allclose(tg, t, atol=1e-9)


def test_ransac_finds_the_inliers():
    rng = np.random.default_rng(5)
    X, R, t = _scene(rng, 300)
    f, cx, cy = 500.0, 320.0, 240.0
    uv, _ = ba.project(R, t, X, f, f, cx, cy)
    uv = uv + rng.normal(0, 0.3, uv.shape)
    out = rng.random(300) < 0.3
    uv[:, out] += rng.uniform(20, 80, (2, out.sum())) * rng.choice([-1, 1], (2, out.sum()))
    R0 = ba.so3_exp(np.array([0.02, -0.01, 0.015])) @ R
    res = ba.estimate_pose(X, uv, R0, t + 0.03, f, f, cx, cy, n_hyp=64, seed=11)
    assert (res["inliers"] == ~out).mean() > 0.98 and not (res["inliers"] & out).any()
    ang = np.degrees(np.arccos(np.clip((np.trace(res["R_refined"].T @ R) - 1) / 2, -1, 1)))
    assert ang < 0.05 and np.linalg.norm(res["t_refined"] - t) < 5e-3
    # the sample of a hypothesis: distinct, the splitmix64 draws in order
    s = ba.ransac_sample(11, 3, 6, 300)
    assert len(set(s.tolist())) == 6 and s[0] == ba.splitmix64(11 + (3 << 32)) % 300


def test_bootstrap_recovers_focal_poses_and_structure():
    rng = np.random.default_rng(6)
    V, P, W, H = 4, 60, 640, 480
    f_true = 520.0
    cx, cy = W / 2, H / 2
    Rs = [np.eye(3)]
    ts = [np.zeros(3)]
    for v in range(1, V):
        Rs.append(ba.so3_exp(rng.standard_normal(3) * 0.03))
        ts.append(np.array([0.15 * v, 0.02 * rng.standard_normal(), 0.02 * rng.standard_normal()]))
    X = np.stack([rng.uniform(-1.5, 1.5, P), rng.uniform(-1, 1, P), rng.uniform(3, 5, P)])
    uv = np.stack([ba.project(Rs[v], ts[v], X, f_true, f_true, cx, cy)[0] for v in range(V)])
    out = ba.bootstrap_ba(uv, W, H, iters=200)
    r, _ = ba.ba_residuals(out["f"], out["R"], out["t"], out["X"], uv, cx, cy)
    assert np.sqrt((r * r).mean()) < 1e-3
    assert abs(out["f"] - f_true) < 0.5
    s = np.linalg.norm(out["t"][1]) / np.linalg.norm(ts[1])  # the free scale
    for v in range(1, V):
        ang = np.degrees(np.arccos(np.clip((np.trace(out["R"][v].T @ Rs[v]) - 1) / 2, -1, 1)))
        assert ang < 0.05 and np.allclose(out["t"][v] / s, ts[v], atol=2e-3)
    assert np.allclose(out["X"] / s, X, atol=5e-3)


def test_bootstrap_cost_closed_forms():
    """Zero at the exact solution; with residuals planted on a known set, the
    Huber sum of those the median + 4 MAD rule keeps."""
    rng = np.random.default_rng(41)
    V, P, W, H, f = 3, 40, 320, 240, 300.0
    Rs = [np.eye(3)] + [ba.so3_exp(rng.standard_normal(3) * 0.02) for _ in range(V - 1)]
    ts = [np.zeros(3)] + [np.array([0.2 * v, 0.0, 0.0]) for v in range(1, V)]
    X = np.stack([rng.uniform(-1, 1, P), rng.uniform(-1, 1, P), rng.uniform(3, 5, P)])
    uv = np.stack([ba.project(Rs[v], ts[v], X, f, f, W / 2, H / 2)[0] for v in range(V)])
    poses = np.stack([np.concatenate([Rs[v].reshape(9), ts[v]]) for v in range(V)])
    assert ba.bootstrap_cost(f, poses, X, uv, W, H) < 1e-18
    # planted errors along u (view-major order): 58 of 0.25 px, 59 of 0.75 px, 3 of 50 px; the median is
    # 0.75, the MAD 0.5, so the rule keeps errors up to 2.75 and drops the three large ones
    shift = np.array([0.25] * 58 + [0.75] * 59 + [50.0] * 3)
    rng.shuffle(shift)
    uv2 = uv.copy()
    uv2[:, 0, :] -= shift.reshape(V, P)
    c = ba.bootstrap_cost(f, poses, X, uv2, W, H)
    assert abs(c - (58 * 0.5 * 0.25 ** 2 + 59 * 0.5 * 0.75 ** 2)) < 1e-9
    # beyond delta = 1 the Huber cost is delta (e - delta / 2): all errors 3 px, all kept (MAD 0 up to rounding
    # would reject some, so the errors are spread: 3 and 4 px alternately, median 3.5, MAD 0.5)
    uv3 = uv.copy()
    uv3[:, 0, :] -= np.where(np.arange(V * P) % 2 == 0, 3.0, 4.0).reshape(V, P)
    assert abs(ba.bootstrap_cost(f, poses, X, uv3, W, H) - (V * P // 2) * (2.5 + 3.5)) < 1e-9
