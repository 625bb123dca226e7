"""The 3D smoothing filter of multi-scale training through the C ABI against
the oracle (oracle/multiscale.py apply_filter3d / filter3d_vjp around the
FP64 rasterizer oracle): the sampling-rate update over several cameras, and
the image and every gradient (log-scales and logits through the filter's
chain rule) with and without the screen-space filter."""
import numpy as np
import pytest
import torch

from oracle import multiscale as ms
from oracle import raster as orc
from paper_2506_05558_amd import synth
from tests import gpu_common as gc
from tests.test_gpu_raster import FLAG_REL, _check_grads, _check_image

pytestmark = pytest.mark.gpu


def test_sampling_rate_update_matches_oracle():
    gs = gc.gpu()
    views = synth.trajectory(41, 11, 320, 240)  # 11 cameras: two launches of eight
    scene = synth.window_scene(41, views, 4000, 0)
    means = torch.tensor(scene.means, device="cuda")
    n = scene.n
    nu = torch.zeros(n, dtype=torch.float32, device="cuda")
    f3 = torch.empty(n, dtype=torch.float32, device="cuda")
    cams = [gc.gpu_camera(v) for v in views]
    gs.filter3d_update(means, cams[:4], nu)  # a window first, then the rest (keyframes arriving)
    gs.filter3d_update(means, cams[4:], nu, f3)
    ref = np.zeros(n)
    for v in views:
        R = np.asarray(v.R, np.float32).astype(np.float64)
        t = np.asarray(v.t, np.float32).astype(np.float64)
        rate = ms.sampling_rate(scene.means, R, t, float(np.float32(v.fx)), float(np.float32(v.fy)),
                                float(np.float32(v.cx)), float(np.float32(v.cy)), v.width, v.height,
                                guard=float(np.float32(1.15)))
        ref = np.maximum(ref, rate)
    got = nu.cpu().numpy().astype(np.float64)
    assert np.array_equal(got > 0, ref > 0)
    assert np.allclose(got, ref, rtol=1e-7, atol=0)
    var = ms.filter_variance(got)
    assert np.allclose(f3.cpu().numpy(), var, rtol=1e-6, atol=0)
    print(f"sampling rates: {int((ref > 0).sum())} of {n} seen, filter variance up to {var.max():.3g}")


def _case(name, view, scene, params_kw, seed, scale=30.0):
    gs = gc.gpu()
    cam = gc.gpu_camera(view)
    g = gc.gpu_gauss(scene)
    # the filter of this camera alone, made larger than Mip-Splatting's so that it matters at 128 px
    R = np.asarray(view.R, np.float32).astype(np.float64)
    t = np.asarray(view.t, np.float32).astype(np.float64)
    rate = ms.sampling_rate(scene.means, R, t, float(np.float32(view.fx)), float(np.float32(view.fy)),
                            float(np.float32(view.cx)), float(np.float32(view.cy)), view.width, view.height)
    v = (ms.filter_variance(rate) * scale).astype(np.float32)
    g.filter3d = torch.tensor(v, device="cuda")
    params = gs.Params(**params_kw)
    proj = gs.project(cam, g, params)
    binned = gs.BinSorter(0)(cam, proj)
    frame = gs.render_fwd(cam, proj, binned, params)
    torch.cuda.synchronize()
    ls2, a2 = ms.apply_filter3d(scene.log_scales, scene.opacity_logits, v.astype(np.float64))
    ocam = orc.Camera.from_view(view, **params_kw)
    og = orc.Gaussians(scene.means, ls2, scene.quats, a2, scene.sh, scene.sh_degree)
    op = orc.project(ocam, og)
    vis = op["visible"] > 0
    assert (vis != (proj.radius.cpu().numpy()[0] > 0)).mean() < 1e-3
    rec = proj.rec.cpu().numpy()
    both = vis & (proj.radius.cpu().numpy()[0] > 0)
    assert np.abs(rec[both, 7] - op["opacity"][both]).max() <= 1e-5
    ref = orc.render(ocam, op, flag_rel=FLAG_REL)
    _check_image(name, frame, ref)
    gi, gd, ga = gc.flagged_upstream((view.height, view.width), ref["flags"], seed)
    d_pose = torch.zeros(12, dtype=torch.float64, device="cuda")
    d_twist = torch.zeros(6, dtype=torch.float64, device="cuda")
    grads = gs.render_bwd(cam, g, proj, binned, frame, torch.tensor(gi, device="cuda"), torch.tensor(gd, device="cuda"),
                          torch.tensor(ga, device="cuda"), dL_dpose=d_pose, dL_dtwist=d_twist, params=params)
    torch.cuda.synchronize()
    rg = orc.backward(ocam, og, op, gi, gd, ga)
    rg["log_scales"], rg["opacity_logits"] = ms.filter3d_vjp(scene.log_scales, scene.opacity_logits, v,
                                                             rg["log_scales"], rg["opacity_logits"])
    _check_grads(name, grads, d_pose, d_twist, rg)
    print(f"{name}: mean filter variance {v.mean():.3g}, opacity factor down to "
          f"{np.exp((scene.log_scales - ls2).sum(0)).min():.3f}")


def test_filter3d_parity_dilation():
    view, scene, _ = synth.tiny_scene(43)
    _case("filter3d", view, scene, dict(), seed=5)


def test_filter3d_parity_with_screen_space_filter():
    view, scene, _ = synth.tiny_scene(44)
    _case("filter3d+mip", view, scene, dict(eps2d=0.1, mip_filter=1), seed=6)


def test_filter3d_zero_is_the_unfiltered_path():
    gs = gc.gpu()
    view, scene, _ = synth.tiny_scene(45)
    cam = gc.gpu_camera(view)
    g = gc.gpu_gauss(scene)
    p0 = gs.project(cam, g)
    g.filter3d = torch.zeros(scene.n, dtype=torch.float32, device="cuda")
    p1 = gs.project(cam, g)
    assert torch.equal(p0.rec, p1.rec) and torch.equal(p0.radius, p1.radius)
