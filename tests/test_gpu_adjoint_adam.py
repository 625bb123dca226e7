"""The window's projection adjoint with the sparse Adam step applied by its
last pass (gs_project_bwd_views_adam).

* Bit for bit equal to the store-form adjoint followed by gs_adam_step on
  each parameter group (visible set, per-Gaussian rates) and gs_lr_decay:
  one batch of views, more than eight views (the last batch's pass adds to
  the earlier batches' stored SH gradients), without per-Gaussian rates,
  and with no view at all (nothing is updated).
* Against the FP64 oracle on a 3-view window: the oracle's gradients summed
  over the views, then its Adam step and rate decay on the oracle's own
  visible set (positive tile count in some view), compared through the
  moments (the gradient each recovers), the parameter step and the rates.
"""
import numpy as np
import pytest
import torch

from oracle import binning, optim
from oracle import raster as orc
from tests import gpu_common as gc
from tests.test_gpu_adjoint_store import _window as store_window
from tests.test_gpu_raster import FLAG_REL
from tests.test_gpu_raster import _window as raster_window

pytestmark = pytest.mark.gpu

GROUPS = (("means", "lr_means"), ("log_scales", "lr_log_scales"), ("quats", "lr_quats"),
          ("opacity_logits", "lr_opacity"))
DECAY = 0.99


def _opt(gs, step):
    return gs.AdamGroups(lr_means=1.6e-2, lr_log_scales=5e-3, lr_quats=1e-2, lr_opacity=2e-2, lr_sh_dc=7.5e-3,
                         lr_sh_rest=6e-3, step=step, lr_decay=DECAY)


def _clone(gs, g):
    return gs.Gaussians(*[t.clone() for t in g.tensors()])


def _moments(gs, g, seed, m_scale=1e-3, v_scale=1e-6):
    rng = np.random.default_rng(seed)
    dev = lambda a: torch.tensor(a.astype(np.float32), device="cuda")
    m1 = gs.Gaussians(*[dev(rng.standard_normal(tuple(t.shape)) * m_scale) for t in g.tensors()])
    m2 = gs.Gaussians(*[dev(rng.random(tuple(t.shape)) * v_scale) for t in g.tensors()])
    return m1, m2, dev(rng.uniform(0.5, 1.0, g.n))


def _unfused(gs, vs, g, m1, m2, rates, opt, params):
    grads = g.zeros_like()
    vis = torch.zeros(g.n, dtype=torch.int32, device="cuda")
    gs.project_bwd_views(vs, g, grads, params, store=True, visible=vis)
    for name, lr in GROUPS:
        gs.adam_step(getattr(g, name), getattr(grads, name), getattr(m1, name), getattr(m2, name), getattr(opt, lr),
                     opt.step, visible=vis, n_stride=g.n, lr_scale=rates)
    gs.adam_step(g.sh[0], grads.sh[0], m1.sh[0], m2.sh[0], opt.lr_sh_dc, opt.step, visible=vis, n_stride=g.n,
                 lr_scale=rates)
    if g.sh.shape[0] > 1:
        gs.adam_step(g.sh[1:], grads.sh[1:], m1.sh[1:], m2.sh[1:], opt.lr_sh_rest, opt.step, visible=vis,
                     n_stride=g.n, lr_scale=rates)
    if rates is not None:
        gs.lr_decay(rates, opt.lr_decay, vis)
    return vis


@pytest.mark.parametrize("n_views,with_rates", [(3, True), (11, True), (3, False), (0, True)])
def test_fused_equals_store_then_adam(n_views, with_rates):
    gs = gc.gpu()
    g, vs, params = store_window(gs, max(n_views, 1), 90 + n_views)
    vs = vs[:n_views]
    opt = _opt(gs, 7)
    m1, m2, rates = _moments(gs, g, 5 + n_views)
    if not with_rates:
        rates = None
    # unfused: store-form adjoint, six Adam launches, rate decay
    gA, m1A, m2A = _clone(gs, g), _clone(gs, m1), _clone(gs, m2)
    rA = None if rates is None else rates.clone()
    visA = _unfused(gs, vs, gA, m1A, m2A, rA, opt, params)
    poses_A = [vw.dL_dpose.clone() for vw in vs]
    for vw in vs:
        vw.dL_dpose.zero_()
    # fused, with stale scratch and a stale visible set
    gB, m1B, m2B = _clone(gs, g), _clone(gs, m1), _clone(gs, m2)
    rB = None if rates is None else rates.clone()
    scratch = gs.Gaussians(*[torch.full_like(t, 123.0) for t in g.tensors()])
    visB = torch.full((g.n,), 7, dtype=torch.int32, device="cuda")
    gs.project_bwd_views_adam(vs, gB, scratch, m1B, m2B, opt, visB, lr_scale=rB, params=params)
    torch.cuda.synchronize()
    assert torch.equal(visA, visB)
    for name, a, b in zip(("g", "m1", "m2"), (gA, m1A, m2A), (gB, m1B, m2B)):
        for k, (x, y) in enumerate(zip(a.tensors(), b.tensors())):
            assert torch.equal(x, y), f"{name} plane group {k} differs"
    if rates is not None:
        assert torch.equal(rA, rB)
    for vw, p in zip(vs, poses_A):
        assert torch.equal(vw.dL_dpose, p)
    seen = int(visB.sum())
    if n_views == 0:
        assert seen == 0
        for x, y in zip(gB.tensors(), g.tensors()):
            assert torch.equal(x, y)
        if rates is not None:
            assert torch.equal(rB, rates)
    else:
        assert 0 < seen < g.n
        hidden = visB == 0
        for x, y in zip(gB.tensors(), g.tensors()):  # the sparse step leaves the others as they were
            assert torch.equal(x[..., hidden], y[..., hidden])
            assert not torch.equal(x[..., ~hidden], y[..., ~hidden])


def _oracle_visible(views, scene):
    """Positive tile count in some view, from the oracle's own projection."""
    vis = np.zeros(scene.n, bool)
    for v in views:
        ocam, og = gc.oracle_inputs(v, scene)
        op = orc.project(ocam, og)
        on = op["visible"] > 0
        rx = np.where(on, np.ceil(op["half"][0] * (1 + 1e-4) + 1e-3), 0).astype(np.int64)
        ry = np.where(on, np.ceil(op["half"][1] * (1 + 1e-4) + 1e-3), 0).astype(np.int64)
        cnt = binning.tile_rects(op["mean2d"][0], op["mean2d"][1], rx, ry, v.width, v.height, 16)[4]
        vis |= on & (cnt > 0)
    return vis


def test_fused_step_matches_oracle():
    """3 views of 160x120, 4,500 SH-3 Gaussians, step 7: the oracle's FP64
    gradients summed over the views, its Adam step per group and its rate
    decay, against the fused call."""
    gs = gc.gpu()
    views, scene = raster_window(3, 160, 120, 1500, 31)
    g = gc.gpu_gauss(scene)
    n = scene.n
    keys = ("means", "log_scales", "quats", "opacity_logits", "sh")
    total, ups = None, []
    for k, v in enumerate(views):
        ocam, og = gc.oracle_inputs(v, scene)
        op = orc.project(ocam, og)
        ref = orc.render(ocam, op, flag_rel=FLAG_REL)
        up = gc.flagged_upstream((v.height, v.width), ref["flags"], 40 + k)
        ups.append(up)
        rg = orc.backward(ocam, og, op, *up)
        total = {key: rg[key] if total is None else total[key] + rg[key] for key in keys}
    vis_o = _oracle_visible(views, scene)
    # moments at the scale s of each plane's gradients (m0 ~ s / 10,
    # v0 ~ s^2 / 10^4): the new moments and the step then depend on the
    # gradient more than on the moments' rounding, and the step (a few
    # times the rate) stays well above the parameters' rounding
    rng = np.random.default_rng(17)
    m0, v0 = {}, {}
    for key in keys:
        gref = np.asarray(total[key], np.float64)
        s = float(np.sqrt(np.mean(gref[..., vis_o] ** 2))) + 1e-30
        m0[key] = (rng.standard_normal(gref.shape) * 0.1 * s).astype(np.float32)
        v0[key] = ((rng.random(gref.shape) + 0.5) * 1e-4 * s * s).astype(np.float32)
    rates0 = rng.uniform(0.5, 1.0, n).astype(np.float32)
    opt = _opt(gs, 7)
    dev = lambda a: torch.tensor(a, device="cuda")
    # device side: views through the multi-view path, then the fused call
    vs = []
    for k, v in enumerate(views):
        cam = gc.gpu_camera(v)
        vs.append(gs.View(cam, gs.alloc_projected(n), first_slot=torch.empty(n, dtype=torch.int32, device="cuda"),
                          dL_dpose=torch.zeros(12, dtype=torch.float64, device="cuda")))
    gs.project_views(vs, g)
    for k, vw in enumerate(vs):
        b = gs.BinSorter(0)(vw.cam, vw.proj, first_slot=vw.first_slot)
        fr = gs.render_fwd(vw.cam, vw.proj, b)
        vw.pair_grad = torch.empty((max(b.n_instances, 1), 12), dtype=torch.float32, device="cuda")
        gi, gd, ga = (dev(a) for a in ups[k])
        gs.render_bwd_pairs(vw.cam, vw.proj, b, fr, gi, vw.pair_grad, gd, ga)
    p0 = {key: getattr(g, key).cpu().numpy().astype(np.float64) for key in keys}
    m1 = gs.Gaussians(*[dev(m0[key]) for key in keys])
    m2 = gs.Gaussians(*[dev(v0[key]) for key in keys])
    rates = dev(rates0)
    vis = torch.zeros(n, dtype=torch.int32, device="cuda")
    gs.project_bwd_views_adam(vs, g, g.zeros_like(), m1, m2, opt, vis, lr_scale=rates)
    torch.cuda.synchronize()
    assert np.array_equal(vis.cpu().numpy() != 0, vis_o)
    lrs = {"means": opt.lr_means, "log_scales": opt.lr_log_scales, "quats": opt.lr_quats,
           "opacity_logits": opt.lr_opacity}
    b1, b2 = opt.beta1, opt.beta2
    for key in keys:
        gref = np.asarray(total[key], np.float64)
        if key == "sh":  # degree 0 and the higher degrees take their own rates
            parts = [(np.s_[0:1], opt.lr_sh_dc), (np.s_[1:], opt.lr_sh_rest)]
        else:
            parts = [(np.s_[...], lrs[key])]
        for sl, lr in parts:
            gp = gref[sl]
            pn, mn, vn = optim.adam(p0[key][sl], gp, m0[key][sl], v0[key][sl], lr, opt.step, b1, b2, opt.eps,
                                    visible=vis_o.astype(np.int32), n_stride=n, lr_scale=rates0)
            got_p = getattr(g, key).cpu().numpy()[sl].astype(np.float64)
            got_m = getattr(m1, key).cpu().numpy()[sl].astype(np.float64)
            got_v = getattr(m2, key).cpu().numpy()[sl].astype(np.float64)
            on, off = (np.s_[..., vis_o], np.s_[..., ~vis_o])
            # the Gaussians the step skipped keep their values exactly
            assert np.array_equal(got_p[off], p0[key][sl][off])
            assert np.array_equal(got_m[off], m0[key][sl][off].astype(np.float64))
            assert np.array_equal(got_v[off], v0[key][sl][off].astype(np.float64))
            # the gradient each moment recovers, and the parameter step
            name = f"{key}[{sl}]"
            gc.assert_grad_close(f"{name} grad from m1", (got_m[on] - b1 * m0[key][sl][on]) / (1 - b1), gp[on])
            gc.assert_grad_close(f"{name} grad^2 from m2", (got_v[on] - b2 * v0[key][sl][on].astype(np.float64)) /
                                 (1 - b2), gp[on] ** 2, rel=2e-3)
            # the step: L2 over the set at the gradients' tolerance; per element the new FP32
            # parameter within 1e-3 of the step (its rounding, and the gradients' tolerance
            # where the step hardly depends on g), plus what the gradients' per-element
            # tolerance (assert_grad_close's) moves the oracle's step -- its own Adam at
            # g +- that tolerance; where b1 m0 and (1 - b1) g nearly cancel the step is far more
            # sensitive than g -- plus two units in the parameter's last place (a smaller step
            # cannot be resolved)
            dp_ref = pn[on] - p0[key][sl][on]
            dp_got = got_p[on] - p0[key][sl][on]
            e = np.linalg.norm(dp_got - dp_ref) / np.linalg.norm(dp_ref)
            assert e <= 1e-3, f"{name} step: relative L2 error {e:.3e}"
            eg = 1e-3 * (np.abs(gp) + 1e-3 * np.abs(gp[on]).max())
            moved = [optim.adam(p0[key][sl], gp + sgn * eg, m0[key][sl], v0[key][sl], lr, opt.step, b1, b2, opt.eps,
                                visible=vis_o.astype(np.int32), n_stride=n, lr_scale=rates0)[0][on] for sgn in (1, -1)]
            tol = (1e-3 * np.abs(dp_ref) + np.maximum(np.abs(moved[0] - pn[on]), np.abs(moved[1] - pn[on])) +
                   2 * np.spacing(np.abs(pn[on]).astype(np.float32)).astype(np.float64))
            bad = np.abs(got_p[on] - pn[on]) > tol
            print(f"{name} step: rel L2 {e:.2e}, {bad.sum()} of {bad.size} outside")
            assert not bad.any(), f"{name} step: {bad.sum()} of {bad.size} elements outside tolerance"
    r_ref = optim.lr_decay(rates0, DECAY, vis_o.astype(np.int32))
    assert np.abs(rates.cpu().numpy() - r_ref).max() <= 1e-6
