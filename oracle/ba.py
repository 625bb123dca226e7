"""FP64 oracle of the initial pose estimation's mini bundle adjustment
(section 4.1 and the appendix on initial pose estimation).  Test
infrastructure only: tests and the benchmark's CPU baseline call it, the
product path never does.

The reprojection model is the pinhole camera of the rasterizer: a world
point X seen by the world->camera pose [R | t] lands at
pi(p) = (fx p_x / p_z + cx, fy p_y / p_z + cy), p = R X + t.

* Levenberg-Marquardt, as the appendix states it: initial damping
  lambda = 1e-5, factor nu = 2: after a step that lowers the cost lambda is
  divided by nu and the step kept, otherwise lambda is multiplied by nu and
  the step dropped.  Damped normal equations (J^T W J + lambda diag(J^T W J))
  delta = -J^T W r (Marquardt's scaling; the paper gives only the schedule).
* Robustness: the Huber loss on each observation's reprojection error e
  (rho(e) = e^2 / 2 for e <= delta, delta (e - delta / 2) above, as
  iteratively reweighted least squares with weights min(1, delta / e)), and
  each iteration discards the observations whose error exceeds the median
  plus four times the median absolute deviation of the errors at the
  iterate.  The cost compared by the schedule is the Huber cost over the
  observations kept at that iteration.
* Pose updates are left perturbations T <- exp(xi^) T, xi = (rho, phi).
* Pose for a new frame from 3D-2D correspondences: RANSAC whose estimator is
  the same solver -- each hypothesis starts at the previous pose and runs a
  few LM iterations (no robust loss) on a minimal set of six correspondences
  drawn with the counter-based SplitMix64 stream; the hypothesis with most
  inliers (reprojection error below a threshold; ties to the lower
  hypothesis) wins, then 20 iterations on all its inliers refine it.
* Bootstrapping: the focal length f (fx = fy = f, principal point fixed),
  the poses of views 1..V-1 (view 0 is the identity, fixing the gauge's
  rotation and translation) and the points, each point observed in every
  view (the fixed-size layout), from f = 0.7 W, identity poses and points at
  depth 1 along view 0's rays; 200 iterations, the Huber loss throughout
  and the median + 4 MAD rejection in the second half.
"""
from __future__ import annotations

import math

import numpy as np

from oracle.spawn import splitmix64

LAMBDA0, NU = 1e-5, 2.0
MASK64 = (1 << 64) - 1


# ------------------------------------------------------------ geometry
def hat(w):
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def so3_exp(w):
    """Rodrigues' formula."""
    th = float(np.linalg.norm(w))
    K = hat(w)
    if th < 1e-12:
        return np.eye(3) + K + 0.5 * K @ K
    return np.eye(3) + math.sin(th) / th * K + (1.0 - math.cos(th)) / (th * th) * K @ K


def se3_left_update(R, t, xi):
    """exp(xi^) T for xi = (rho, phi), with the first-order translation part
    of the exponential replaced by the exact SE(3) V matrix."""
    rho, phi = np.asarray(xi[:3], np.float64), np.asarray(xi[3:], np.float64)
    dR = so3_exp(phi)
    th = float(np.linalg.norm(phi))
    K = hat(phi)
    if th < 1e-12:
        V = np.eye(3) + 0.5 * K + K @ K / 6.0
    else:
        V = np.eye(3) + (1.0 - math.cos(th)) / (th * th) * K + (th - math.sin(th)) / th ** 3 * K @ K
    return dR @ R, dR @ t + V @ rho


def project(R, t, X, fx, fy, cx, cy):
    """X [3][K] -> (uv [2][K], p [3][K])."""
    p = np.asarray(R, np.float64) @ np.asarray(X, np.float64) + np.asarray(t, np.float64)[:, None]
    return np.stack([fx * p[0] / p[2] + cx, fy * p[1] / p[2] + cy]), p


def pose_jacobian(p, fx, fy):
    """d uv / d xi (left twist) at camera-frame points p [3][K]: [K][2][6]."""
    x, y, z = p
    iz, iz2 = 1.0 / z, 1.0 / (z * z)
    Jp = np.zeros((p.shape[1], 2, 3))
    Jp[:, 0, 0] = fx * iz
    Jp[:, 0, 2] = -fx * x * iz2
    Jp[:, 1, 1] = fy * iz
    Jp[:, 1, 2] = -fy * y * iz2
    # d p / d xi = [I | -p^]
    J = np.zeros((p.shape[1], 2, 6))
    J[:, :, :3] = Jp
    for k in range(p.shape[1]):
        J[k, :, 3:] = Jp[k] @ (-hat(p[:, k]))
    return J


# ------------------------------------------------------------ robust loss
def huber(e, delta):
    e = np.asarray(e, np.float64)
    return np.where(e <= delta, 0.5 * e * e, delta * (e - 0.5 * delta))


def huber_weight(e, delta):
    e = np.asarray(e, np.float64)
    return np.where(e <= delta, 1.0, delta / np.maximum(e, 1e-300))


def mad_keep(err):
    """Keep the observations whose error is at most median + 4 MAD."""
    err = np.asarray(err, np.float64)
    if err.size == 0:
        return np.zeros(0, bool)
    med = np.median(err)
    mad = np.median(np.abs(err - med))
    return err <= med + 4.0 * mad


def damped_step(H, g, lam):
    """Solution of (H + lam diag(H)) delta = -g.  A variable without any
    kept observation (zero diagonal, and then zero gradient) does not move."""
    d = np.diag(H)
    live = d > 0
    step = np.zeros_like(g)
    if live.any():
        A = H[np.ix_(live, live)] + lam * np.diag(d[live])
        step[live] = np.linalg.solve(A, -g[live])
    return step


# ------------------------------------------------------- pose refinement
def lm_pose(X, uv, R, t, fx, fy, cx, cy, iters, mask=None, delta=None, robust=True, lam0=LAMBDA0, nu=NU,
            trace=None):
    """LM on the pose alone.  mask: the correspondences that take part;
    robust: Huber loss (threshold delta px) and the median + 4 MAD rejection
    at every iteration.  Returns (R, t, lambda)."""
    X = np.asarray(X, np.float64)
    uv = np.asarray(uv, np.float64)
    use = np.ones(X.shape[1], bool) if mask is None else np.asarray(mask, bool)
    R, t = np.asarray(R, np.float64).copy(), np.asarray(t, np.float64).copy()
    lam = lam0
    for _ in range(iters):
        pr, p = project(R, t, X, fx, fy, cx, cy)
        r = (pr - uv)[:, use]
        e = np.sqrt((r * r).sum(0))
        keep = mad_keep(e) if robust else np.ones(e.size, bool)
        w = huber_weight(e, delta) if robust else np.ones(e.size)
        w = w * keep
        cost = (huber(e, delta) * keep).sum() if robust else 0.5 * (e * e).sum()
        J = pose_jacobian(p[:, use], fx, fy)
        H = np.einsum("k,kai,kaj->ij", w, J, J)
        g = np.einsum("k,kai,ak->i", w, J, r)
        step = damped_step(H, g, lam)
        Rn, tn = se3_left_update(R, t, step)
        prn, _ = project(Rn, tn, X, fx, fy, cx, cy)
        rn = (prn - uv)[:, use]
        en = np.sqrt((rn * rn).sum(0))
        cost_n = (huber(en, delta) * keep).sum() if robust else 0.5 * (en * en).sum()
        accepted = cost_n < cost
        if trace is not None:
            trace.append(dict(cost=cost, cost_new=cost_n, lam=lam, accepted=bool(accepted), kept=int(keep.sum())))
        if accepted:
            R, t, lam = Rn, tn, lam / nu
        else:
            lam = lam * nu
    return R, t, lam


def ransac_sample(seed, h, m, K):
    """The m distinct correspondence indices of hypothesis h: draws
    c = 0, 1, ... of splitmix64(seed + h 2^32 + c) mod K, skipping repeats."""
    out = []
    c = 0
    while len(out) < min(m, K):
        j = splitmix64((seed + (h << 32) + c) & MASK64) % K
        if j not in out:
            out.append(j)
        c += 1
    return np.array(out, np.int64)


def reproj_error(R, t, X, uv, fx, fy, cx, cy):
    pr, p = project(R, t, X, fx, fy, cx, cy)
    d = pr - np.asarray(uv, np.float64)
    e = np.sqrt((d * d).sum(0))
    return np.where(p[2] > 0, e, np.inf)


def ransac_pose(X, uv, R0, t0, fx, fy, cx, cy, n_hyp=128, m=6, hyp_iters=10, tau=2.0, seed=0):
    """Per hypothesis: the pose and its inlier count; the winner."""
    K = np.asarray(X).shape[1]
    poses, counts = [], []
    for h in range(n_hyp):
        idx = ransac_sample(seed, h, m, K)
        mask = np.zeros(K, bool)
        mask[idx] = True
        R, t, _ = lm_pose(X, uv, R0, t0, fx, fy, cx, cy, hyp_iters, mask=mask, robust=False)
        e = reproj_error(R, t, X, uv, fx, fy, cx, cy)
        poses.append((R, t))
        counts.append(int((e < tau).sum()))
    best = int(np.argmax(counts))  # first maximum: ties to the lower hypothesis
    R, t = poses[best]
    inl = reproj_error(R, t, X, uv, fx, fy, cx, cy) < tau
    return dict(best=best, counts=np.array(counts), R=R, t=t, inliers=inl)


def estimate_pose(X, uv, R0, t0, fx, fy, cx, cy, n_hyp=128, m=6, hyp_iters=10, tau=2.0, refine_iters=20, delta=1.0,
                  seed=0):
    """RANSAC, then 20 robust LM iterations on all inliers."""
    rs = ransac_pose(X, uv, R0, t0, fx, fy, cx, cy, n_hyp, m, hyp_iters, tau, seed)
    R, t, lam = lm_pose(X, uv, rs["R"], rs["t"], fx, fy, cx, cy, refine_iters, mask=rs["inliers"], delta=delta)
    rs.update(R_refined=R, t_refined=t, lam=lam)
    return rs


# -------------------------------------------------------- bootstrapping
def bootstrap_init(uv, f0, cx, cy):
    """Points at depth 1 along view 0's rays; identity poses."""
    uv = np.asarray(uv, np.float64)
    V, P = uv.shape[0], uv.shape[2]
    X = np.stack([(uv[0, 0] - cx) / f0, (uv[0, 1] - cy) / f0, np.ones(P)])
    return f0, [np.eye(3) for _ in range(V)], [np.zeros(3) for _ in range(V)], X


def ba_residuals(f, Rs, ts, X, uv, cx, cy):
    """[V][2][P] residuals and [V][3][P] camera-frame points."""
    r, ps = [], []
    for v in range(len(Rs)):
        pr, p = project(Rs[v], ts[v], X, f, f, cx, cy)
        r.append(pr - uv[v])
        ps.append(p)
    return np.stack(r), np.stack(ps)


def ba_jacobian(f, Rs, ps, X):
    """Dense Jacobian of the stacked residuals (view-major, then point,
    then u / v) w.r.t. (f, xi_1..xi_{V-1}, X_1..X_P)."""
    V, P = len(Rs), X.shape[1]
    nc = 1 + 6 * (V - 1)
    J = np.zeros((V * P * 2, nc + 3 * P))
    for v in range(V):
        x, y, z = ps[v]
        Jp = np.zeros((P, 2, 3))
        Jp[:, 0, 0] = f / z
        Jp[:, 0, 2] = -f * x / (z * z)
        Jp[:, 1, 1] = f / z
        Jp[:, 1, 2] = -f * y / (z * z)
        for k in range(P):
            row = 2 * (v * P + k)
            J[row, 0] = x[k] / z[k]
            J[row + 1, 0] = y[k] / z[k]
            if v > 0:
                c0 = 1 + 6 * (v - 1)
                J[row:row + 2, c0:c0 + 3] = Jp[k]
                J[row:row + 2, c0 + 3:c0 + 6] = Jp[k] @ (-hat(ps[v][:, k]))
            J[row:row + 2, nc + 3 * k:nc + 3 * k + 3] = Jp[k] @ Rs[v]
    return J


def bootstrap_ba(uv, W, H, iters=200, delta=1.0, lam0=LAMBDA0, nu=NU, mad_from=None, trace=None):
    """Joint LM over f, poses 1..V-1 and points (dense normal equations).
    The median + 4 MAD rejection applies from iteration mad_from on (default
    iters // 2): from the identity / unit-depth start the first iterations'
    errors measure how far the solution still has to move, not how well an
    observation fits, and rejecting by them would freeze observations that
    have not converged yet."""
    if mad_from is None:
        mad_from = iters // 2
    uv = np.asarray(uv, np.float64)
    cx, cy = W / 2.0, H / 2.0
    f, Rs, ts, X = bootstrap_init(uv, 0.7 * W, cx, cy)
    V, P = uv.shape[0], uv.shape[2]
    lam = lam0
    for it in range(iters):
        r, ps = ba_residuals(f, Rs, ts, X, uv, cx, cy)
        e = np.sqrt((r * r).sum(1)).ravel()  # [V * P]
        keep = mad_keep(e) if it >= mad_from else np.ones(e.size, bool)
        w = huber_weight(e, delta) * keep
        cost = (huber(e, delta) * keep).sum()
        J = ba_jacobian(f, Rs, ps, X)
        wr = np.repeat(w, 2)
        rv = r.transpose(0, 2, 1).reshape(-1)
        Hm = J.T @ (J * wr[:, None])
        g = J.T @ (wr * rv)
        step = damped_step(Hm, g, lam)
        fn = f + step[0]
        Rn, tn = [Rs[0]], [ts[0]]
        for v in range(1, V):
            c0 = 1 + 6 * (v - 1)
            a, b = se3_left_update(Rs[v], ts[v], step[c0:c0 + 6])
            Rn.append(a)
            tn.append(b)
        Xn = X + step[1 + 6 * (V - 1):].reshape(P, 3).T
        rn, _ = ba_residuals(fn, Rn, tn, Xn, uv, cx, cy)
        en = np.sqrt((rn * rn).sum(1)).ravel()
        cost_n = (huber(en, delta) * keep).sum()
        accepted = cost_n < cost
        if trace is not None:
            trace.append(dict(cost=cost, cost_new=cost_n, lam=lam, accepted=bool(accepted)))
        if accepted:
            f, Rs, ts, X, lam = fn, Rn, tn, Xn, lam / nu
        else:
            lam = lam * nu
    return dict(f=f, R=Rs, t=ts, X=X, lam=lam)


def bootstrap_cost(f, poses, X, uv, W, H, delta=1.0):
    """The bootstrapping objective at a solution: the Huber cost of the
    observations the median + 4 MAD rule keeps there.  poses [V][12] (R
    row-major, t), X [3][P], uv [V][2][P]."""
    poses = np.asarray(poses, np.float64)
    Rs = [poses[v, :9].reshape(3, 3) for v in range(poses.shape[0])]
    ts = [poses[v, 9:] for v in range(poses.shape[0])]
    r, _ = ba_residuals(float(f), Rs, ts, np.asarray(X, np.float64), np.asarray(uv, np.float64), W / 2.0, H / 2.0)
    e = np.sqrt((r * r).sum(1)).ravel()
    return float((huber(e, delta) * mad_keep(e)).sum())
