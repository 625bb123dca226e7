"""Pins of the FP64 rasterizer oracle against facts that do not come from it.

* SH basis: orthonormality over the sphere (exact product quadrature).
* Quaternion rotation: equals the Hamilton product q v q*.
* One Gaussian on the optical axis: image, depth, alpha and the gradients with
  respect to opacity, scales, depth, mean and colour have closed forms.
* Compositing invariants: weights telescope (sum w + T = 1), white-on-white
  stays white, equal depths give depth = z * alpha, order of the input does
  not matter, transparent scenes give the background, T never drops below the
  cutoff, a Gaussian hidden behind a saturated pixel changes nothing.
* Finite differences (FP64, central, h = 1e-6) of every parameter and of the
  camera twist on small scenes whose pixels are away from every decision
  threshold.
* Pose gauge identity: a left twist of the camera equals moving every
  Gaussian by the inverse motion, so the pose gradient must equal a sum of
  Gaussian gradients (degree-0 colour, no view dependence).
"""
import math

import numpy as np
import pytest

from paper_2506_05558_amd import synth


def _cam(orc, view, **kw):
    return orc.Camera.from_view(view, **kw)


def _g(orc, scene):
    return orc.Gaussians.from_scene(scene)


# --------------------------------------------------------------------------
def test_sh_orthonormal(oracle_lib):
    orc = oracle_lib
    x, w = np.polynomial.legendre.leggauss(12)  # exact for degree <= 23 in cos(theta)
    nphi = 24
    phi = 2 * math.pi * np.arange(nphi) / nphi
    dirs, wts = [], []
    for ct, wt in zip(x, w):
        st = math.sqrt(1 - ct * ct)
        for ph in phi:
            dirs.append([st * math.cos(ph), st * math.sin(ph), ct])
            wts.append(wt * 2 * math.pi / nphi)
    Y = orc.sh_basis(3, np.array(dirs))
    G = (Y * np.array(wts)[:, None]).T @ Y
    assert np.abs(G - np.eye(16)).max() < 1e-12


def test_sh_known_values(oracle_lib):
    # Y_0 = 1/(2 sqrt(pi)); Y_(1,0) along +z = sqrt(3/(4 pi)); Y_(2,0) at +z = sqrt(5/(4 pi))
    Y = oracle_lib.sh_basis(3, np.array([[0.0, 0.0, 1.0]]))[0]
    assert abs(Y[0] - 0.5 / math.sqrt(math.pi)) < 1e-15
    assert abs(Y[2] - math.sqrt(3 / (4 * math.pi))) < 1e-15
    assert abs(Y[6] - math.sqrt(5 / (4 * math.pi))) < 1e-15
    assert abs(Y[12] - math.sqrt(7 / (4 * math.pi))) < 1e-15


def _hamilton(a, b):
    w1, v1 = a[0], np.asarray(a[1:])
    w2, v2 = b[0], np.asarray(b[1:])
    return np.concatenate([[w1 * w2 - v1 @ v2], w1 * v2 + w2 * v1 + np.cross(v1, v2)])


def test_quat_rotation_matches_hamilton(oracle_lib):
    rng = np.random.default_rng(3)
    for _ in range(20):
        q = rng.standard_normal(4)
        R = oracle_lib.quat_to_rot(q)
        qn = q / np.linalg.norm(q)
        v = rng.standard_normal(3)
        rv = _hamilton(_hamilton(qn, np.concatenate([[0.0], v])), qn * np.array([1, -1, -1, -1]))[1:]
        assert np.allclose(R @ v, rv, atol=1e-13)
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-13)
        assert abs(np.linalg.det(R) - 1) < 1e-13


# --------------------------------------------------------------------------
def _one_gaussian(z=3.0, s=(0.02, 0.03, 0.05), logit=0.3, rgb=(0.8, 0.4, 0.2), size=32, f=40.0):
    view = synth.View(size, size, f, f, size / 2.0, size / 2.0)
    sc = synth.Scene(np.array([[0.0], [0.0], [z]], np.float32), np.log(np.array(s, np.float32))[:, None],
                     np.array([[1.0], [0.0], [0.0], [0.0]], np.float32), np.array([logit], np.float32),
                     ((np.array(rgb) - 0.5) * 2 * math.sqrt(math.pi)).astype(np.float32)[None, :, None], 0)
    return view, sc


def test_single_gaussian_closed_form(oracle_lib):
    orc = oracle_lib
    view, sc = _one_gaussian()
    bg = (0.1, 0.2, 0.3)
    cam = _cam(orc, view, bg=bg)
    g = _g(orc, sc)
    proj, out = orc.forward(cam, g)
    z, f = float(sc.means[2, 0]), cam.fx
    s = np.exp(g.log_scales[:, 0])
    v1 = f * f * s[0] ** 2 / z ** 2 + 0.3
    v2 = f * f * s[1] ** 2 / z ** 2 + 0.3
    o = 1 / (1 + math.exp(-g.opacity_logits[0]))
    rgb = 0.5 + g.sh[0, :, 0] * 0.5 / math.sqrt(math.pi)
    yy, xx = np.mgrid[0:view.height, 0:view.width]
    dx, dy = xx - view.cx, yy - view.cy
    raw = o * np.exp(-0.5 * (dx * dx / v1 + dy * dy / v2))
    a = np.where(raw >= 1 / 255, np.minimum(raw, 0.99), 0.0)
    for c in range(3):
        assert np.abs(out["image"][c] - (rgb[c] * a + (1 - a) * bg[c])).max() < 1e-13
    assert np.abs(out["depth"] - z * a).max() < 1e-12
    assert np.abs(out["alpha"] - a).max() < 1e-14

    # gradients of L = sum G_img . image + sum G_d depth, by hand
    rng = np.random.default_rng(0)
    GI = rng.standard_normal((3, view.height, view.width))
    GD = rng.standard_normal((view.height, view.width))
    gr = orc.backward(cam, g, proj, g_image=GI, g_depth=GD)
    live = (raw >= 1 / 255) & (raw < 0.99)
    dL_da = np.einsum("chw,c->hw", GI, rgb) - np.einsum("chw,c->hw", GI, np.array(bg)) + GD * z
    e = np.exp(-0.5 * (dx * dx / v1 + dy * dy / v2))
    # opacity logit: da/do = e, do/dlogit = o (1 - o)
    d_logit = np.sum(dL_da * e * live) * o * (1 - o)
    assert abs(gr["opacity_logits"][0] - d_logit) < 1e-10 * max(1, abs(d_logit))
    # log-scale k (k = 0, 1): da/dv_k = a dx^2 / (2 v_k^2), dv_k/dlog s_k = 2 f^2 s_k^2 / z^2
    for k, (v, d2) in enumerate([(v1, dx * dx), (v2, dy * dy)]):
        ref = np.sum(dL_da * raw * live * d2 / (2 * v * v)) * 2 * f * f * s[k] ** 2 / z ** 2
        assert abs(gr["log_scales"][k, 0] - ref) < 1e-9 * max(1, abs(ref))
    assert abs(gr["log_scales"][2, 0]) < 1e-12  # the depth axis does not project
    # mean x: mean2d_x = f x / z + cx, da/dmx = a dx / v1
    ref = np.sum(dL_da * raw * live * dx / v1) * f / z
    assert abs(gr["means"][0, 0] - ref) < 1e-9 * max(1, abs(ref))
    # mean z: v_k depend on z (dv_k/dz = -2 f^2 s_k^2 / z^3), depth = z directly
    dvdz = [-2 * f * f * s[0] ** 2 / z ** 3, -2 * f * f * s[1] ** 2 / z ** 3]
    ref = np.sum(dL_da * raw * live * (dx * dx / (2 * v1 * v1) * dvdz[0] + dy * dy / (2 * v2 * v2) * dvdz[1]))
    ref += np.sum(GD * a)
    assert abs(gr["means"][2, 0] - ref) < 1e-9 * max(1, abs(ref))
    # colour: d image_c / d sh0_c = a / (2 sqrt(pi))
    for c in range(3):
        ref = np.sum(GI[c] * a) * 0.5 / math.sqrt(math.pi)
        assert abs(gr["sh"][0, c, 0] - ref) < 1e-10 * max(1, abs(ref))
    # translation of the camera along z moves the Gaussian's depth the same way
    assert abs(gr["t"][2] - gr["means"][2, 0]) < 1e-10 * max(1, abs(ref))


def test_mip_filter_single_gaussian_closed_form(oracle_lib):
    # screen-space filter of variance eps: v_k = raw_k + eps and the opacity
    # scaled by rho = sqrt(raw_1 raw_2 / (v_1 v_2)) for an axis-aligned splat
    orc = oracle_lib
    view, sc = _one_gaussian(s=(0.01, 0.015, 0.05), logit=1.5)
    eps = 0.1
    cam = _cam(orc, view, eps2d=eps, mip_filter=1)
    g = _g(orc, sc)
    proj, out = orc.forward(cam, g)
    z, f = float(sc.means[2, 0]), cam.fx
    s = np.exp(g.log_scales[:, 0])
    r1, r2 = f * f * s[0] ** 2 / z ** 2, f * f * s[1] ** 2 / z ** 2
    v1, v2 = r1 + eps, r2 + eps
    rho = math.sqrt(r1 * r2 / (v1 * v2))
    o = 1 / (1 + math.exp(-g.opacity_logits[0]))
    assert abs(proj["opacity"][0] - o * rho) < 1e-15
    yy, xx = np.mgrid[0:view.height, 0:view.width]
    dx, dy = xx - view.cx, yy - view.cy
    e = np.exp(-0.5 * (dx * dx / v1 + dy * dy / v2))
    raw = o * rho * e
    a = np.where(raw >= 1 / 255, np.minimum(raw, 0.99), 0.0)
    assert np.abs(out["alpha"] - a).max() < 1e-14
    rng = np.random.default_rng(1)
    GA = rng.standard_normal((view.height, view.width))
    gr = orc.backward(cam, g, proj, g_alpha=GA)
    live = (raw >= 1 / 255) & (raw < 0.99)
    # d alpha / d logit = e rho o (1 - o)
    ref = np.sum(GA * live * e) * rho * o * (1 - o)
    assert abs(gr["opacity_logits"][0] - ref) < 1e-10 * max(1, abs(ref))
    # log-scale k: raw_k = f^2 s_k^2 / z^2 moves v_k and rho; d raw_k / d log s_k = 2 raw_k,
    # d rho / d raw_k = rho (1 / raw_k - 1 / v_k) / 2, d alpha / d v_k = alpha d^2 / (2 v_k^2)
    for k, (rk, vk, d2) in enumerate([(r1, v1, dx * dx), (r2, v2, dy * dy)]):
        dv = np.sum(GA * live * raw * d2 / (2 * vk * vk))
        drho = np.sum(GA * live * o * e) * rho * (1 / rk - 1 / vk) / 2
        ref = (dv + drho) * 2 * rk
        assert abs(gr["log_scales"][k, 0] - ref) < 1e-9 * max(1, abs(ref)), k


def test_mip_filter_preserves_the_splat_integral(oracle_lib):
    # the filter keeps o 2 pi sqrt(det Sigma2): the compensated opacity times
    # sqrt(det) equals the unfiltered one's, whatever the filter variance
    orc = oracle_lib
    view, sc, _ = synth.tiny_scene(2, n=300, size=64)
    g = _g(orc, sc)
    p0 = orc.project(_cam(orc, view, eps2d=0.0), g)
    for eps in (0.1, 0.3, 2.0):
        p1 = orc.project(_cam(orc, view, eps2d=eps, mip_filter=1), g)
        both = (p0["visible"] > 0) & (p1["visible"] > 0)
        assert both.sum() > 100
        det = lambda c: c[0] * c[2] - c[1] * c[1]
        lhs = p1["opacity"][both] * np.sqrt(det(p1["cov2d"])[both])
        rhs = p0["opacity"][both] * np.sqrt(det(p0["cov2d"])[both])
        assert np.allclose(lhs, rhs, rtol=1e-9, atol=0)
        assert (p1["opacity"][both] < p0["opacity"][both]).all()
    # with eps = 0 the filter changes nothing
    p2 = orc.project(_cam(orc, view, eps2d=0.0, mip_filter=1), g)
    assert np.array_equal(p2["opacity"], p0["opacity"])


def test_single_gaussian_alpha_clamp(oracle_lib):
    orc = oracle_lib
    view, sc = _one_gaussian(logit=8.0, s=(0.1, 0.1, 0.1))
    cam = _cam(orc, view)
    g = _g(orc, sc)
    proj, out = orc.forward(cam, g)
    assert abs(out["alpha"].max() - 0.99) < 1e-15
    # where the clamp is active the opacity logit receives no gradient
    GI = np.zeros((3, view.height, view.width))
    c = int(view.cx)
    GI[0, c, c] = 1.0
    gr = orc.backward(cam, g, proj, g_image=GI)
    assert gr["opacity_logits"][0] == 0.0
    assert gr["log_scales"][0, 0] == 0.0


# --------------------------------------------------------------------------
def test_compositing_invariants(oracle_lib):
    orc = oracle_lib
    view, sc, _ = synth.tiny_scene(1)
    cam = _cam(orc, view)
    g = _g(orc, sc)
    proj, out = orc.forward(cam, g)
    a, T = out["alpha"], out["final_t"]
    assert (a >= 0).all() and (a < 1).all()
    assert np.abs(a + T - 1).max() < 1e-15
    assert (T >= 1e-4).all()
    assert (out["image"] >= -1e-15).all() and (out["image"] <= a[None] + 1e-12).all()
    assert out["n_contrib"].max() > 3

    # white Gaussians on a white background: weights telescope to exactly one
    gw = _g(orc, sc)
    gw.sh[:] = math.sqrt(math.pi)  # colour exactly 0.5 + sqrt(pi) / (2 sqrt(pi)) = 1 in FP64
    camw = _cam(orc, view, bg=(1.0, 1.0, 1.0))
    _, outw = orc.forward(camw, gw)
    assert np.abs(outw["image"] - 1.0).max() < 1e-12

    # all at one depth (identity pose): depth = z * alpha
    flat = synth.Scene(np.concatenate([sc.means[:2], np.full_like(sc.means[2:], 4.0)]), sc.log_scales, sc.quats,
                       sc.opacity_logits, sc.sh, 0)
    _, outf = orc.forward(cam, _g(orc, flat))
    assert np.abs(outf["depth"] - 4.0 * outf["alpha"]).max() < 1e-12

    # input order does not matter when depths are distinct
    perm = np.random.default_rng(0).permutation(sc.n)
    sp = synth.Scene(sc.means[:, perm], sc.log_scales[:, perm], sc.quats[:, perm], sc.opacity_logits[perm],
                     sc.sh[:, :, perm], 0)
    _, outp = orc.forward(cam, _g(orc, sp))
    assert np.abs(outp["image"] - out["image"]).max() < 1e-14

    # fully transparent scene renders the background
    clear = synth.Scene(sc.means, sc.log_scales, sc.quats, np.full_like(sc.opacity_logits, -20.0), sc.sh, 0)
    camb = _cam(orc, view, bg=(0.25, 0.5, 0.75))
    projc, outc = orc.forward(camb, _g(orc, clear))
    assert projc["visible"].sum() == 0
    assert np.abs(outc["image"] - np.array([0.25, 0.5, 0.75])[:, None, None]).max() == 0.0


def test_hidden_gaussian_changes_nothing(oracle_lib):
    orc = oracle_lib
    # a wall of opaque Gaussians saturates the centre; one more far behind is invisible there
    n = 60
    rng = np.random.default_rng(5)
    means = np.stack([rng.uniform(-0.05, 0.05, n), rng.uniform(-0.05, 0.05, n), rng.uniform(2.0, 2.2, n)])
    sc = synth.Scene(means.astype(np.float32), np.full((3, n), -1.5, np.float32),
                     np.tile(np.array([[1.0], [0], [0], [0]], np.float32), (1, n)), np.full(n, 6.0, np.float32),
                     np.zeros((1, 3, n), np.float32), 0)
    view = synth.View(16, 16, 20.0, 20.0, 8.0, 8.0)
    cam = _cam(orc, view)
    _, out = orc.forward(cam, _g(orc, sc))
    extra = synth.Scene(np.concatenate([sc.means, np.array([[0.0], [0.0], [5.0]], np.float32)], 1),
                        np.concatenate([sc.log_scales, np.full((3, 1), -1.0, np.float32)], 1),
                        np.concatenate([sc.quats, np.array([[1.0], [0], [0], [0]], np.float32)], 1),
                        np.concatenate([sc.opacity_logits, [3.0]]).astype(np.float32),
                        np.concatenate([sc.sh, np.full((1, 3, 1), 1.0, np.float32)], 2), 0)
    _, out2 = orc.forward(cam, _g(orc, extra))
    sat = out["n_support"] > out["n_contrib"]  # the pixel stopped at the cutoff
    assert sat.sum() > 10
    assert np.array_equal(out["image"][:, sat], out2["image"][:, sat])


# --------------------------------------------------------------------------
def _loss_and_grads(orc, cam, g, G):
    proj, out = orc.forward(cam, g, nthreads=1)
    L = float(np.sum(G["image"] * out["image"]) + np.sum(G["depth"] * out["depth"]) +
              np.sum(G["alpha"] * out["alpha"]))
    return L, proj, out


def _fd_scene_ok(orc, cam, g):
    _, out = orc.forward(cam, g, flag_rel=1e-3, nthreads=1)
    return (out["flags"] == 0).all()


@pytest.mark.parametrize("deg,seed,mip", [(0, 11, 0), (3, 12, 0), (3, 14, 1)])
def test_finite_differences_params(oracle_lib, deg, seed, mip):
    orc = oracle_lib
    for s in range(seed, seed + 50):
        view, sc = synth.small_scene(s, sh_degree=deg)
        cam = _cam(orc, view, bg=(0.2, 0.1, 0.05), mip_filter=mip, eps2d=0.1 if mip else 0.3)
        g = _g(orc, sc)
        if _fd_scene_ok(orc, cam, g):
            break
    else:
        pytest.fail("no threshold-free scene found")
    rng = np.random.default_rng(seed)
    G = dict(image=rng.standard_normal((3, view.height, view.width)),
             depth=rng.standard_normal((view.height, view.width)) * 0.1,
             alpha=rng.standard_normal((view.height, view.width)))
    _, proj, _ = _loss_and_grads(orc, cam, g, G)
    an = orc.backward(cam, g, proj, G["image"], G["depth"], G["alpha"], nthreads=1)
    h = 1e-6
    for name in ["means", "log_scales", "quats", "opacity_logits", "sh"]:
        arr = getattr(g, name)
        fd = np.zeros_like(arr)
        it = np.nditer(arr, flags=["multi_index"])
        for _ in it:
            idx = it.multi_index
            keep = arr[idx]
            arr[idx] = keep + h
            Lp = _loss_and_grads(orc, cam, g, G)[0]
            arr[idx] = keep - h
            Lm = _loss_and_grads(orc, cam, g, G)[0]
            arr[idx] = keep
            fd[idx] = (Lp - Lm) / (2 * h)
        err = np.linalg.norm(fd - an[name]) / max(np.linalg.norm(an[name]), 1e-12)
        assert err < 2e-6, (name, err)
        assert np.linalg.norm(an[name]) > 0 or name == "quats"


def _expm_hat(w):
    th = np.linalg.norm(w)
    if th == 0:
        return np.eye(3)
    K = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]]) / th
    return np.eye(3) + math.sin(th) * K + (1 - math.cos(th)) * K @ K


def test_finite_differences_pose(oracle_lib):
    orc = oracle_lib
    for s in range(30, 80):
        view, sc = synth.small_scene(s, sh_degree=0)
        R, t = synth.random_pose(np.random.default_rng(s), 4.0, 0.05)
        view.R, view.t = R, t
        cam = _cam(orc, view)
        g = _g(orc, sc)
        if _fd_scene_ok(orc, cam, g):
            break
    rng = np.random.default_rng(1)
    G = dict(image=rng.standard_normal((3, view.height, view.width)),
             depth=rng.standard_normal((view.height, view.width)) * 0.1,
             alpha=rng.standard_normal((view.height, view.width)))
    _, proj, _ = _loss_and_grads(orc, cam, g, G)
    an = orc.backward(cam, g, proj, G["image"], G["depth"], G["alpha"], nthreads=1)
    h = 1e-6
    R0, t0 = cam.R.copy(), cam.t.copy()
    fd = np.zeros(6)
    for j in range(6):
        xi = np.zeros(6)
        vals = []
        for sgn in (1, -1):
            xi[:] = 0
            xi[j] = sgn * h
            E = _expm_hat(xi[3:])
            cam.R, cam.t = E @ R0, E @ t0 + xi[:3]
            vals.append(_loss_and_grads(orc, cam, g, G)[0])
        fd[j] = (vals[0] - vals[1]) / (2 * h)
    cam.R, cam.t = R0, t0
    assert np.linalg.norm(fd - an["twist"]) < 2e-6 * np.linalg.norm(an["twist"])
    # dL/dR and dL/dt against raw-entry differences (R as a general matrix)
    fdR = np.zeros(9)
    for k in range(9):
        Rp = R0.reshape(9).copy()
        Rp[k] += h
        cam.R = Rp.reshape(3, 3)
        Lp = _loss_and_grads(orc, cam, g, G)[0]
        Rp[k] -= 2 * h
        cam.R = Rp.reshape(3, 3)
        Lm = _loss_and_grads(orc, cam, g, G)[0]
        fdR[k] = (Lp - Lm) / (2 * h)
    cam.R = R0
    assert np.linalg.norm(fdR - an["R"].reshape(9)) < 2e-6 * np.linalg.norm(an["R"])


def test_pose_gauge_identity(oracle_lib):
    orc = oracle_lib
    view, sc, target = synth.tiny_scene(2)
    R, t = synth.random_pose(np.random.default_rng(2), 6.0, 0.1)
    view.R, view.t = R, t
    cam = _cam(orc, view)
    U, _, Vt = np.linalg.svd(cam.R)
    cam.R = U @ Vt  # exactly orthogonal in FP64 (the identity needs R^-1 = R^T)
    g = _g(orc, sc)
    g.quats /= np.linalg.norm(g.quats, axis=0, keepdims=True)  # exactly unit in FP64
    proj, out = orc.forward(cam, g)
    gi = np.sign(out["image"] - target) / out["image"].size
    gr = orc.backward(cam, g, proj, g_image=gi, g_depth=np.full(out["depth"].shape, 1e-3))
    Rm = cam.R
    vis = proj["visible"] > 0
    gm = gr["means"][:, vis]
    gq = gr["quats"][:, vis]
    mu = g.means[:, vis]
    q = g.quats[:, vis]
    p = Rm @ mu + cam.t[:, None]
    Rg = Rm @ gm
    rho = Rg.sum(1)
    w, v = q[0], q[1:]
    gw, gv = gq[0], gq[1:]
    d_omega = 0.5 * (w * gv - gw * v + np.cross(v.T, gv.T).T)
    phi = np.cross(p.T, Rg.T).sum(0) + (Rm @ d_omega).sum(1)
    ref = np.concatenate([rho, phi])
    assert np.linalg.norm(ref - gr["twist"]) < 1e-9 * np.linalg.norm(ref)


def test_depth_tie_flag(oracle_lib):
    """The tie flag fires exactly when binary32 depths tie and the index order
    runs against the FP64 depth order."""
    orc = oracle_lib
    view = synth.View(8, 8, 10.0, 10.0, 4.0, 4.0)
    z0 = 3.0
    z1 = float(np.nextafter(np.float64(z0), 4.0))  # same binary32 rounding, larger in FP64
    for zs, expect in [((z1, z0), True), ((z0, z1), False), ((z0, z0 + 1e-3), False)]:
        means = np.array([[0.0, 0.0], [0.0, 0.0], list(zs)])
        g = orc.Gaussians(means, np.full((3, 2), -2.0), np.tile([[1.0], [0], [0], [0]], (1, 2)),
                          np.full(2, 0.0), np.zeros((1, 3, 2)), 0)
        _, out = orc.forward(orc.Camera.from_view(view), g)
        assert bool(out["flags"][4, 4] & 8) == expect, zs


def test_support_box_is_the_ellipse_bounding_box(oracle_lib):
    """hx, hy bound every pixel offset with alpha >= alpha_min and are attained
    on the boundary ellipse d^T Sigma2^-1 d = 2 ln(o / alpha_min)."""
    orc = oracle_lib
    view, sc, _ = synth.tiny_scene(4)
    cam = _cam(orc, view)
    proj = orc.project(cam, _g(orc, sc))
    th = np.linspace(0, 2 * np.pi, 20001)
    for i in np.nonzero(proj["visible"])[0][:50]:
        a, b, c = proj["cov2d"][:, i]
        qmax = 2 * np.log(proj["opacity"][i] * 255.0)
        L = np.linalg.cholesky(np.array([[a, b], [b, c]]))
        d = L @ np.stack([np.cos(th), np.sin(th)]) * np.sqrt(qmax)
        assert abs(np.abs(d[0]).max() - proj["half"][0, i]) < 1e-6 * proj["half"][0, i]
        assert abs(np.abs(d[1]).max() - proj["half"][1, i]) < 1e-6 * proj["half"][1, i]
        assert proj["half"][:, i].max() <= proj["radius"][i] * (1 + 1e-12)
