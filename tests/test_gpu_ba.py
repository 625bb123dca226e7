"""GPU parity of the mini bundle adjustment (section 4.1, appendix on initial
pose estimation) with oracle/ba.py, through the C ABI.

* Pose of a new frame (gs_pose_ransac): every hypothesis's inlier count and
  the winner exactly (counts near the threshold are excluded), the
  winner's inlier mask exactly, and the refined pose to 1e-9 (FP64 on both
  sides; the two sides sum in different orders, so the LM decisions match
  except at stagnation); cases: 300 correspondences with 30 % outliers,
  6144 (the paper's keypoint count), fewer correspondences than the
  minimal set, and no inlier at all.
* Bootstrapping (gs_ba_bootstrap): the same damping decisions with the
  cost / candidate cost to 1e-7 relative while the two runs keep one path
  (they may part only at a decision the costs' accuracy cannot settle, or
  after convergence), then final objectives within 5 % and focal lengths
  within 2 % (noisy bootstrapping is nearly flat along the focal / depth
  direction), and the focal length, poses and points
  against the oracle's dense LM when the paths never part, on noise-free
  and noisy 4-view and 8-view problems; at the largest size (8 views x 1024 points) the
  recovery of the ground truth up to the free scale."""
import numpy as np
import pytest
import torch

from oracle import ba

from .gpu_common import gpu

pytestmark = pytest.mark.gpu

F, CX, CY = 500.0, 320.0, 240.0


def _corr(seed, K, outliers=0.3, noise=0.3):
    rng = np.random.default_rng(seed)
    X = np.stack([rng.uniform(-1, 1, K), rng.uniform(-1, 1, K), rng.uniform(3, 6, K)]).astype(np.float32)
    R = ba.so3_exp(rng.standard_normal(3) * 0.05)
    t = rng.standard_normal(3) * 0.1
    uv, _ = ba.project(R, t, X.astype(np.float64), F, F, CX, CY)
    uv = uv + rng.normal(0, noise, uv.shape)
    out = rng.random(K) < outliers
    uv[:, out] += rng.uniform(20, 80, (2, out.sum())) * rng.choice([-1, 1], (2, out.sum()))
    R0 = ba.so3_exp(np.array([0.02, -0.01, 0.015])) @ R
    return X, uv.astype(np.float32), R, t, R0, t + 0.03, out


def _ransac_case(seed, K, n_hyp, outliers=0.3):
    gs = gpu()
    X, uv, R, t, R0, t0, out = _corr(seed, K, outliers)
    pose0 = np.concatenate([R0.reshape(9), t0])
    Xd, uvd = torch.tensor(X, device="cuda"), torch.tensor(uv, device="cuda")
    pose, pose32, inl, n_inl, counts = gs.pose_ransac(Xd, uvd, F, F, CX, CY, pose0, n_hyp=n_hyp, seed=seed)
    torch.cuda.synchronize()
    X64, uv64 = X.astype(np.float64), uv.astype(np.float64)
    ref = ba.estimate_pose(X64, uv64, R0, t0, F, F, CX, CY, n_hyp=n_hyp, seed=seed)
    got = counts.cpu().numpy()
    # a hypothesis count may differ only if one of its errors sits at the threshold
    near = np.zeros(n_hyp, bool)
    for h in range(n_hyp):
        if got[h] != ref["counts"][h]:
            idx = ba.ransac_sample(seed, h, 6, K)
            mask = np.zeros(K, bool)
            mask[idx] = True
            Rh, th, _ = ba.lm_pose(X64, uv64, R0, t0, F, F, CX, CY, 10, mask=mask, robust=False)
            e = ba.reproj_error(Rh, th, X64, uv64, F, F, CX, CY)
            near[h] = (np.abs(e - 2.0) < 1e-9).any()
    assert np.array_equal(got[~near], ref["counts"][~near]), np.flatnonzero(got != ref["counts"])[:10]
    assert not near[ref["best"]]
    assert np.array_equal(inl.cpu().numpy() != 0, ref["inliers"])
    assert int(n_inl.item()) == int(ref["inliers"].sum())
    p = pose.cpu().numpy()
    assert np.abs(p[:9] - ref["R_refined"].reshape(9)).max() < 1e-9
    assert np.abs(p[9:] - ref["t_refined"]).max() < 1e-9
    assert np.array_equal(pose32.cpu().numpy(), p.astype(np.float32))
    print(f"ransac K={K}: best {ref['best']} with {ref['counts'][ref['best']]} inliers, "
          f"{near.sum()} counts at the threshold")
    return ref, R, t


def test_ransac_300_with_outliers():
    ref, R, t = _ransac_case(5, 300, 64)
    ang = np.degrees(np.arccos(np.clip((np.trace(ref["R_refined"].T @ R) - 1) / 2, -1, 1)))
    assert ang < 0.05


def test_ransac_6144_keypoints():
    _ransac_case(6, 6144, 32, outliers=0.2)


def test_ransac_edge_cases():
    _ransac_case(7, 4, 8, outliers=0.0)  # fewer correspondences than the minimal set
    _ransac_case(8, 50, 8, outliers=1.0)  # no inlier: the refinement holds still


def _bootstrap_problem(seed, V, P, noise):
    rng = np.random.default_rng(seed)
    W, H = 640, 480
    f_true = 520.0
    Rs, ts = [np.eye(3)], [np.zeros(3)]
    for v in range(1, V):
        Rs.append(ba.so3_exp(rng.standard_normal(3) * 0.03))
        ts.append(np.array([0.15 * v, 0.02 * rng.standard_normal(), 0.02 * rng.standard_normal()]))
    X = np.stack([rng.uniform(-1.5, 1.5, P), rng.uniform(-1, 1, P), rng.uniform(3, 5, P)])
    uv = np.stack([ba.project(Rs[v], ts[v], X, f_true, f_true, W / 2, H / 2)[0] for v in range(V)])
    uv = (uv + rng.normal(0, noise, uv.shape)).astype(np.float32)
    return uv, W, H, f_true, Rs, ts, X


@pytest.mark.parametrize("V,P,noise", [(4, 60, 0.0), (4, 60, 0.3), (8, 120, 0.3)])
def test_bootstrap_matches_oracle(V, P, noise):
    gs = gpu()
    uv, W, H, f_true, Rs, ts, X = _bootstrap_problem(20 + V + P, V, P, noise)
    f, poses, Xg, tr = gs.ba_bootstrap(torch.tensor(uv, device="cuda"), W, H, iters=200, trace=True)
    torch.cuda.synchronize()
    trace = []
    ref = ba.bootstrap_ba(uv.astype(np.float64), W, H, iters=200, trace=trace)
    tg = tr.cpu().numpy()
    # The same Levenberg-Marquardt path: every damping decision equal and the costs to 1e-7 relative
    # (the FP64 solve of the damped normal equations -- Schur reduction here, a dense solve in the
    # oracle -- is ill-conditioned at the start), up to the first iteration where the two runs take
    # different decisions.  They may part only where the decision is a tie at the costs' accuracy
    # (the candidate cost within 1e-6 of the current one, so that rounding decides it), or once the
    # cost has converged (below 1e-9 of the start); then they must still end at the same cost (with
    # noise the bootstrapping problem is nearly flat along the focal / depth direction).
    same = 0
    for it in range(200):
        if tg[it, 2] != trace[it]["lam"]:
            break
        assert abs(tg[it, 0] - trace[it]["cost"]) <= 1e-7 * trace[it]["cost"], it
        assert abs(tg[it, 1] - trace[it]["cost_new"]) <= 1e-7 * max(trace[it]["cost_new"], 1e-300), it
        same += 1
    if same < 200:
        # the decision that parted them was taken at iteration same - 1 (lambda differs at same)
        k = same - 1
        c, cn = trace[k]["cost"], trace[k]["cost_new"]
        tie = abs(cn - c) <= 1e-6 * c
        converged = c <= 1e-9 * trace[0]["cost"]
        assert k >= 0 and (tie or converged), (same, c, cn)
    fg = float(f.item())
    cost_g = ba.bootstrap_cost(fg, poses.cpu().numpy(), Xg.cpu().numpy(), uv.astype(np.float64), W, H)
    cost_o = ba.bootstrap_cost(ref["f"], np.stack([np.concatenate([ref["R"][v].reshape(9), ref["t"][v]])
                                                   for v in range(V)]), ref["X"], uv.astype(np.float64), W, H)
    if same == 200:
        assert abs(cost_g - cost_o) <= 1e-6 * cost_o + 1e-12, (cost_g, cost_o)
    else:  # parted at a tie in a nearly flat valley: equally good ends, the same focal length to 2 %
        assert abs(cost_g - cost_o) <= 0.05 * cost_o + 1e-9, (cost_g, cost_o)
        assert abs(fg - ref["f"]) <= 0.02 * ref["f"], (fg, ref["f"])
    if same == 200:  # one path throughout: the same solution
        assert abs(fg - ref["f"]) <= 1e-6 * ref["f"]
        P_ = poses.cpu().numpy()
        for v in range(V):
            assert np.abs(P_[v, :9] - ref["R"][v].reshape(9)).max() < 1e-7
            assert np.abs(P_[v, 9:] - ref["t"][v]).max() < 1e-7
        assert np.abs(Xg.cpu().numpy() - ref["X"]).max() < 1e-6 * np.abs(ref["X"]).max()
    print(f"bootstrap V={V} P={P} noise={noise}: same path for {same} iterations; f {fg:.4f} "
          f"(oracle {ref['f']:.4f}, true {f_true}); cost {cost_g:.6g} vs {cost_o:.6g}")


def test_bootstrap_largest_problem_recovers_truth():
    gs = gpu()
    V, P = 8, 1024
    uv, W, H, f_true, Rs, ts, X = _bootstrap_problem(99, V, P, 0.0)
    f, poses, Xg, _ = gs.ba_bootstrap(torch.tensor(uv, device="cuda"), W, H, iters=200)
    torch.cuda.synchronize()
    fg = float(f.item())
    P_ = poses.cpu().numpy()
    r, _ = ba.ba_residuals(fg, [P_[v, :9].reshape(3, 3) for v in range(V)], [P_[v, 9:] for v in range(V)],
                           Xg.cpu().numpy(), uv.astype(np.float64), W / 2, H / 2)
    rms = np.sqrt((r * r).mean())
    s = np.linalg.norm(P_[1, 9:]) / np.linalg.norm(ts[1])
    assert rms < 1e-2 and abs(fg - f_true) < 1.0, (rms, fg)
    for v in range(1, V):
        assert np.allclose(P_[v, 9:] / s, ts[v], atol=5e-3)
    print(f"bootstrap 8 x 1024: rms {rms:.2e} px, f {fg:.3f}")
