"""GPU parity of the multi-scale training helpers (section 4.3) against the
oracle in oracle/multiscale.py and oracle/optim.py: per-Gaussian Adam rates
and their decay, the coarse-to-fine box filter (every level, ragged sizes,
both load paths, the full 1920x1080 frame), a full forward + adjoint at the
coarse camera, the screen-space (Mip-Splatting) filter with opacity
compensation through projection, compositing and both adjoints, and opacity
culling (bit-exact keep lists, gathers, and an image that culling below
alpha_min leaves bit-identical)."""
import numpy as np
import pytest
import torch

from oracle import multiscale as ms
from oracle import optim
from oracle import raster as orc
from paper_2506_05558_amd import synth

from . import gpu_common as gc
from .test_gpu_raster import FLAG_REL, _check_binning, _check_grads, _check_image, _full_case

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("planes,n,sparse", [(3, 1000, True), (4, 1001, True), (45, 4096, False), (2, 70_001, True)])
def test_adam_per_gaussian_rates(planes, n, sparse):
    # n % 4 == 0 takes the 16-byte path, otherwise the scalar one
    gs = gc.gpu()
    rng = np.random.default_rng(planes + n)
    shape = (planes, n)
    p, g = rng.standard_normal(shape).astype(np.float32), rng.standard_normal(shape).astype(np.float32)
    m, v = (rng.standard_normal(shape) * 0.1).astype(np.float32), (rng.random(shape) * 0.1).astype(np.float32)
    s = (rng.random(n) * 2).astype(np.float32)
    vis = (rng.random(n) < 0.6).astype(np.int32) if sparse else None
    dp, dg, dm, dv, ds = (torch.tensor(x, device="cuda") for x in (p, g, m, v, s))
    gs.adam_step(dp, dg, dm, dv, 1e-3, 3, eps=1e-8, visible=None if vis is None else torch.tensor(vis, device="cuda"),
                 n_stride=n, lr_scale=ds)
    rp, rm, rv = optim.adam(p, g, m, v, 1e-3, 3, eps=1e-8, visible=vis, n_stride=n, lr_scale=s)
    assert np.abs(dp.cpu().numpy() - rp).max() <= 2e-6
    assert np.abs(dm.cpu().numpy() - rm).max() <= 1e-6 and np.abs(dv.cpu().numpy() - rv).max() <= 1e-6
    if sparse:
        hidden = vis == 0
        assert np.array_equal(dp.cpu().numpy()[:, hidden], p[:, hidden])


def test_lr_decay_over_sparse_steps():
    gs = gc.gpu()
    rng = np.random.default_rng(7)
    n, decay = 100_003, 0.995
    s = np.ones(n)
    ds = torch.ones(n, device="cuda")
    for _ in range(30):
        vis = (rng.random(n) < 0.5).astype(np.int32)
        gs.lr_decay(ds, decay, torch.tensor(vis, device="cuda"))
        s = optim.lr_decay(s, decay, vis)
    gs.lr_decay(ds, decay)  # no mask: every Gaussian
    s = optim.lr_decay(s, decay)
    # FP32 products, one rounding per step: relative error <= 31 * 2^-24
    assert np.abs(ds.cpu().numpy() / s - 1).max() <= 31 * 2.0 ** -24


@pytest.mark.parametrize("c,h,w", [(3, 37, 53), (3, 64, 96), (1, 17, 16), (3, 1080, 1920)])
def test_downsample_every_level(c, h, w):
    gs = gc.gpu()
    rng = np.random.default_rng(h * w)
    img = rng.random((c, h, w)).astype(np.float32)
    d = torch.tensor(img, device="cuda")
    for level in range(5):
        if (w >> level) < 1 or (h >> level) < 1:
            continue
        out = gs.downsample(d, level).cpu().numpy()
        ref = ms.downsample(img, level)
        assert out.shape == ref.shape
        # a FP32 sum of 4^level values in [0, 1): error <= 4^level ulp(1) relative to the mean's scale
        assert np.abs(out - ref).max() <= (4 ** level) * 2.0 ** -24 + 1e-7, level
        if level == 0:
            assert np.array_equal(out, img)


def test_coarse_camera_forward_and_adjoint():
    # the newest image's first iterations: forward and adjoint at the 2^2 and
    # 2^1 coarse cameras match the oracle on the same camera
    gs = gc.gpu()
    view, scene, _ = synth.tiny_scene(11, n=3000, size=160)
    for level in (1, 2):
        w, h, fx, fy, cx, cy = ms.camera_level(view.width, view.height, view.fx, view.fy, view.cx, view.cy, level)
        cv = synth.View(w, h, np.float32(fx), np.float32(fy), np.float32(cx), np.float32(cy), view.R, view.t)
        c = gs.camera_level(gc.gpu_camera(view), level)
        assert (c.width, c.height) == (w, h) and c.fx == np.float32(fx) and c.cx == np.float32(cx)
        _full_case(f"coarse{level}", cv, scene, seed=level)


@pytest.mark.parametrize("n", [0, 1, 1000, 300_001, 2_500_000])
def test_prune_keep_list_bit_exact(n):
    gs = gc.gpu()
    rng = np.random.default_rng(n + 1)
    t = 0.005
    lg = rng.uniform(-9, 3, n).astype(np.float32)
    thr = ms.opacity_threshold_logit(t)
    if n > 10:  # values on and next to the threshold
        lg[:5] = [thr, np.nextafter(thr, np.float32(-np.inf)), np.nextafter(thr, np.float32(np.inf)), -20, 20]
    dl = torch.tensor(lg, device="cuda")
    keep = gs.prune_opacity(dl, t)
    ref = ms.prune_keep(lg, t)
    assert np.array_equal(keep.cpu().numpy(), ref)
    if n > 10:
        assert keep.cpu().numpy()[:2].tolist() == [0, 2]


def test_prune_all_or_nothing_and_gather():
    gs = gc.gpu()
    n = 5000
    assert gs.prune_opacity(torch.full((n,), 5.0, device="cuda")).numel() == n
    assert gs.prune_opacity(torch.full((n,), -9.0, device="cuda")).numel() == 0
    rng = np.random.default_rng(3)
    src = rng.standard_normal((16, 3, n)).astype(np.float32)
    idx = np.sort(rng.choice(n, 1234, replace=False)).astype(np.int32)
    out = gs.gather_planes(torch.tensor(src, device="cuda"), torch.tensor(idx, device="cuda"))
    assert np.array_equal(out.cpu().numpy(), ms.gather_planes(src.reshape(48, n), idx).reshape(16, 3, 1234))


def test_culling_below_alpha_min_leaves_the_image_bit_identical():
    # a Gaussian with opacity < 0.003 < alpha_min = 1/255 never reaches a
    # pixel, and culling keeps the survivors' order, so the tile lists and
    # the image are unchanged
    gs = gc.gpu()
    view, scene, _ = synth.tiny_scene(12, n=4000, size=128)
    rng = np.random.default_rng(4)
    lg = scene.opacity_logits.copy()
    lg[rng.random(lg.size) < 0.3] = -7.0  # opacity 9e-4
    scene.opacity_logits = lg.astype(np.float32)
    cam = gc.gpu_camera(view)
    g = gc.gpu_gauss(scene)
    _, _, full = gc.run_forward(cam, g)
    keep = gs.prune_opacity(g.opacity_logits, 0.003)
    assert np.array_equal(keep.cpu().numpy(), ms.prune_keep(scene.opacity_logits, 0.003))
    g2 = gs.prune_gaussians(g, keep)
    assert g2.n == keep.numel() < g.n
    _, _, cut = gc.run_forward(cam, g2)
    assert torch.equal(full.image, cut.image) and torch.equal(full.depth, cut.depth)
    assert torch.equal(full.final_t, cut.final_t)


def _mip_case(name, view, scene, seed, eps=0.1):
    gs = gc.gpu()
    params = gs.Params(eps2d=eps, mip_filter=1)
    cam = gc.gpu_camera(view)
    g = gc.gpu_gauss(scene)
    proj = gs.project(cam, g, params)
    binned = gs.BinSorter(0)(cam, proj)
    frame = gs.render_fwd(cam, proj, binned, params)
    torch.cuda.synchronize()
    ocam = orc.Camera.from_view(view, eps2d=eps, mip_filter=1)
    og = orc.Gaussians.from_scene(scene)
    op = orc.project(ocam, og)
    rec = proj.rec.cpu().numpy()
    vis = op["visible"] > 0
    assert np.array_equal(vis, proj.radius.cpu().numpy()[0] > 0)
    # the compensated opacity, and the support box it sets
    assert np.abs(rec[vis, 7] - op["opacity"][vis]).max() <= 1e-6
    assert np.abs(rec[vis, 12:14] - op["half"].T[vis]).max() <= 1e-6 * (1 + np.abs(op["half"]).max())
    _check_binning(view, proj, binned)
    ref = orc.render(ocam, op, flag_rel=FLAG_REL)
    _check_image(name, frame, ref)
    gi, gd, ga = gc.flagged_upstream((view.height, view.width), ref["flags"], seed)
    d_pose = torch.zeros(12, dtype=torch.float64, device="cuda")
    d_twist = torch.zeros(6, dtype=torch.float64, device="cuda")
    grads = gs.render_bwd(cam, g, proj, binned, frame, torch.tensor(gi, device="cuda"),
                          torch.tensor(gd, device="cuda"), torch.tensor(ga, device="cuda"), dL_dpose=d_pose,
                          dL_dtwist=d_twist, params=params)
    torch.cuda.synchronize()
    _check_grads(name, grads, d_pose, d_twist, orc.backward(ocam, og, op, gi, gd, ga))


def test_mip_filter_full_parity():
    view, scene, _ = synth.tiny_scene(13)
    _mip_case("mip", view, scene, seed=3)


def test_mip_filter_at_the_coarse_camera():
    # the filter's purpose: the coarse levels of coarse-to-fine training
    view, scene, _ = synth.tiny_scene(14, n=3000, size=160)
    w, h, fx, fy, cx, cy = ms.camera_level(view.width, view.height, view.fx, view.fy, view.cx, view.cy, 2)
    cv = synth.View(w, h, np.float32(fx), np.float32(fy), np.float32(cx), np.float32(cy), view.R, view.t)
    _mip_case("mip-coarse2", cv, scene, seed=4)


def test_mip_filter_window_views_match_single_view():
    # the multi-view projection and adjoint take the same filter per view
    gs = gc.gpu()
    params = gs.Params(eps2d=0.1, mip_filter=1)
    views = synth.trajectory(5, 3, 96, 64)
    scene = synth.window_scene(5, views, 800, 1)
    g = gc.gpu_gauss(scene)
    cams = [gc.gpu_camera(v) for v in views]
    wv = [gs.View(c, gs.alloc_projected(g.n), None, torch.empty(g.n, dtype=torch.int32, device="cuda"))
          for c in cams]
    gs.project_views(wv, g, params)
    for c, v in zip(cams, wv):
        one = gs.project(c, g, params)
        assert torch.equal(one.rec, v.proj.rec) and torch.equal(one.radius, v.proj.radius)
