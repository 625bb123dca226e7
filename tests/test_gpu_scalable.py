"""The scalable construction's bookkeeping (section 4.4) on the GPU: an
anchor's offload to pinned host memory and its reload are bit-identical
round trips; a sliding-window step at a camera from which most of the
active set looks sub-pixel stores the pre-update set (parameters, both Adam
moments, rates, keyframes) in the anchor unchanged, and the new active set
carries the kept Gaussians' optimiser state (gathered with the kept
indices) with merged entries reset (moments 0, rate 1) -- all checked
against numpy indexing of the host copies and the oracle's merge plan; no
anchor is created from a near camera; the nearest anchors and their blend
weight follow the oracle."""
import numpy as np
import pytest
import torch

from oracle import anchors as an
from paper_2506_05558_amd import synth

from .gpu_common import gpu

pytestmark = pytest.mark.gpu


def _active(seed, n_per_view=20_000, deg=1):
    gs = gpu()
    from paper_2506_05558_amd import scalable
    views = synth.trajectory(seed, 2, 640, 360)
    scene = synth.window_scene(seed, views, n_per_view, deg)
    g = gs.Gaussians.from_arrays(scene.arrays())
    rng = np.random.default_rng(seed)
    a = scalable.ActiveSet(g, *[gs.Gaussians(*[torch.tensor(rng.standard_normal(t.shape).astype(np.float32),
                                                            device="cuda") for t in g.tensors()]) for _ in range(2)],
                           torch.tensor(rng.random(g.n).astype(np.float32), device="cuda"), [3, 4, 5])
    return views, scene, a


def test_offload_reload_round_trip():
    from paper_2506_05558_amd import scalable
    views, scene, act = _active(1, 5_000, 3)
    mgr = scalable.AnchorManager(f=views[0].fx)
    before = [t.clone() for t in act.tensors()]
    anchor = mgr.offload(act, [1.0, 2.0, 3.0])
    anchor.wait()
    back = mgr.load(anchor)
    torch.cuda.synchronize()
    for a, b in zip(back.tensors(), before):
        assert a.shape == b.shape and torch.equal(a, b)
    assert back.keyframes == [3, 4, 5] and anchor.n == act.n


def test_sliding_window_step():
    gs = gpu()
    from paper_2506_05558_amd import scalable
    views, scene, act = _active(2)
    # the synthetic Gaussians are seeded at about a pixel from their view, so
    # the test uses tau = 0.5 px: no anchor from the first keyframe itself,
    # one from a camera 15 units behind it
    mgr = scalable.AnchorManager(f=views[0].fx, tau=0.5, seed=17)
    host_before = [t.cpu().numpy() for t in act.tensors()]
    R, t = views[0].R, views[0].t
    near = np.concatenate([R.reshape(9), t]).astype(np.float32)
    _, _, fire_near = an.trigger(scene.means, scene.log_scales, R, t, views[0].fx, tau=0.5)
    assert not fire_near
    same, anchor = mgr.step(act, near, an.camera_centre(R, t))
    assert anchor is None and same is act and not mgr.anchors
    tf = t + np.array([0.0, 0.0, 15.0])
    far = np.concatenate([R.reshape(9), tf]).astype(np.float32)
    # the oracle takes the pose the library receives (binary32)
    flags_ref, count_ref, fire = an.trigger(scene.means, scene.log_scales, far[:9].reshape(3, 3).astype(np.float64),
                                            far[9:].astype(np.float64), views[0].fx, tau=0.5)
    assert fire
    new, anchor = mgr.step(act, far, an.camera_centre(R, tf))
    torch.cuda.synchronize()
    assert anchor is not None and len(mgr.anchors) == 1
    # the anchor holds the pre-update set, bit for bit
    back = mgr.load(anchor)
    for a, b in zip(back.tensors(), host_before):
        assert np.array_equal(a.cpu().numpy(), b)
    assert back.keyframes == [3, 4, 5] and new.keyframes == []
    # the new active set: the oracle's plan, optimiser state gathered and reset
    p = dict(means=scene.means, log_scales=scene.log_scales, quats=scene.quats, opacity_logits=scene.opacity_logits,
             sh=scene.sh)
    cls, nbr, own, keep = an.merge_plan(p, flags_ref, 3, 17)
    assert new.n == keep.size
    merged_pos = np.zeros(keep.size, bool)
    for s in set(own[own >= 0].tolist()):
        merged_pos[np.searchsorted(keep, s)] = True
    m_host = host_before[5:15]
    for k, tnew in enumerate([*new.m1.tensors(), *new.m2.tensors()]):
        want = m_host[k][..., keep].copy()
        want[..., merged_pos] = 0.0
        assert np.array_equal(tnew.cpu().numpy(), want), k
    want_rates = host_before[15][keep].copy()
    want_rates[merged_pos] = 1.0
    assert np.array_equal(new.rates.cpu().numpy(), want_rates)
    kept = ~merged_pos
    for k, tnew in enumerate(new.g.tensors()):
        assert np.array_equal(tnew.cpu().numpy()[..., kept], host_before[k][..., keep][..., kept]), k
    print(f"window step: {act.n} -> {new.n} Gaussians, {merged_pos.sum()} merged, anchor {anchor.host.numel()} B")


def test_nearest_anchors_and_weight():
    from paper_2506_05558_amd import scalable
    views, scene, act = _active(3, 2_000, 0)
    mgr = scalable.AnchorManager(f=views[0].fx)
    for loc in ([0.0, 0.0, 0.0], [10.0, 0.0, 0.0], [0.0, 30.0, 0.0]):
        mgr.offload(act, loc)
    for a in mgr.anchors:
        a.wait()
    for centre in ([1.0, 0.0, 0.0], [4.8, 0.1, 0.0], [5.0, 0.0, 0.0], [9.0, 1.0, 0.0]):
        i1, i2, w = mgr.nearest(centre)
        d = [np.linalg.norm(np.array(a.location) - np.array(centre)) for a in mgr.anchors]
        o = np.argsort(d, kind="stable")
        assert (i1, i2) == (int(o[0]), int(o[1]))
        assert abs(w - an.blend_weight(d[o[0]], d[o[1]], 0.1)) <= 1e-6
