"""Metrics and non-finite handling through the C ABI: gs_psnr against the
oracle's PSNR (and its closed form), gs_count_nonfinite against a planted
count, the projection's cull of Gaussians whose projection is not finite
(the image and every other gradient are unchanged, bit for bit), and the
GS_CHECK_FINITE debug mode's GS_ERR_NONFINITE."""
import math
import os

import numpy as np
import pytest
import torch

from oracle import optim
from paper_2506_05558_amd import synth
from tests import gpu_common as gc

pytestmark = pytest.mark.gpu


def test_psnr_matches_oracle_and_closed_form():
    gs = gc.gpu()
    rng = np.random.default_rng(11)
    for shape in [(3, 17, 23), (3, 1080, 1920), (5,)]:
        img = rng.random(shape).astype(np.float32)
        tgt = rng.random(shape).astype(np.float32)
        out = gs.psnr(torch.tensor(img, device="cuda"), torch.tensor(tgt, device="cuda")).cpu().numpy()
        ref, mse = optim.psnr_images(img, tgt)
        assert abs(out[1] - mse) <= 1e-12 * mse and abs(out[0] - ref) <= 1e-10
    # a constant offset: PSNR = 20 log10(peak / |c|) up to the binary32 inputs
    tgt = rng.random((3, 64, 64)).astype(np.float32)
    img = (tgt.astype(np.float64) + 0.125).astype(np.float32)
    out = gs.psnr(torch.tensor(img, device="cuda"), torch.tensor(tgt, device="cuda"), peak=2.0).cpu().numpy()
    ref, _ = optim.psnr_images(img, tgt, 2.0)
    assert abs(out[0] - ref) <= 1e-10 and abs(out[0] - 20 * math.log10(2.0 / 0.125)) < 1e-3
    same = torch.tensor(tgt, device="cuda")
    assert gs.psnr(same, same).cpu().numpy()[0] == np.inf


def test_count_nonfinite_counts_planted_values():
    gs = gc.gpu()
    x = torch.randn(1_000_003, device="cuda")
    assert gs.count_nonfinite(x) == 0
    idx = torch.tensor([0, 17, 65, 4097, 1_000_002], device="cuda")
    x[idx[:2]] = float("nan")
    x[idx[2:4]] = float("inf")
    x[idx[4]] = float("-inf")
    assert gs.count_nonfinite(x) == 5
    assert gs.count_nonfinite(x[:0].contiguous()) == 0


def _with_bad(scene):
    """The scene followed by Gaussians whose projection is not finite."""
    n = scene.n
    a = {k: v.copy() for k, v in scene.arrays().items()}
    cases = [("means", 0, np.nan), ("means", 2, np.inf), ("log_scales", 1, np.nan), ("log_scales", 0, np.inf),
             ("quats", 3, np.nan), ("quats", None, 0.0), ("opacity_logits", None, np.nan),
             ("opacity_logits", None, -np.inf)]
    k = len(cases)
    src = np.arange(k) % n  # copies of well-placed Gaussians, then spoiled
    for key in a:
        arr = a[key]
        a[key] = np.concatenate([arr, arr[..., src]], axis=-1)
    for c, (field, row, value) in enumerate(cases):
        j = n + c
        if field == "opacity_logits":
            a[field][j] = value
        elif row is None:
            a[field][:, j] = value
        else:
            a[field][row, j] = value
    return a, k


def _run(gs, cam, g, gimg):
    proj = gs.project(cam, g)
    binned = gs.BinSorter(0)(cam, proj)
    frame = gs.render_fwd(cam, proj, binned)
    d_pose = torch.zeros(12, dtype=torch.float64, device="cuda")
    grads = gs.render_bwd(cam, g, proj, binned, frame, gimg, dL_dpose=d_pose)
    torch.cuda.synchronize()
    return proj, binned, frame, grads, d_pose


def test_nonfinite_gaussians_are_culled():
    gs = gc.gpu()
    view, scene, target = synth.tiny_scene(21)
    cam = gc.gpu_camera(view)
    good = gc.gpu_gauss(scene)
    arrays, k = _with_bad(scene)
    spoiled = gs.Gaussians.from_arrays(arrays)
    gimg = torch.tensor(np.random.default_rng(3).standard_normal((3, view.height, view.width)).astype(np.float32),
                        device="cuda")
    p0, b0, f0, g0, d0 = _run(gs, cam, good, gimg)
    p1, b1, f1, g1, d1 = _run(gs, cam, spoiled, gimg)
    n = scene.n
    assert int(p1.tiles_touched[n:].abs().sum()) == 0 and int(p1.radius[:, n:].abs().sum()) == 0
    assert b1.n_instances == b0.n_instances
    for a, b in zip([f1.image, f1.depth, f1.alpha, f1.n_contrib], [f0.image, f0.depth, f0.alpha, f0.n_contrib]):
        assert torch.equal(a, b)
    for a, b in zip(g1.tensors(), g0.tensors()):
        assert torch.equal(a[..., :n], b)
        assert int(torch.count_nonzero(a[..., n:])) == 0
    assert torch.allclose(d1, d0, rtol=1e-12, atol=0.0)
    print(f"{k} spoiled Gaussians culled; {b0.n_instances} pairs unchanged")


def test_check_finite_mode_reports_nonfinite():
    gs = gc.gpu()
    view, scene, _ = synth.tiny_scene(22)
    cam = gc.gpu_camera(view)
    g = gc.gpu_gauss(scene)
    old = os.environ.get("GS_CHECK_FINITE")
    try:
        os.environ["GS_CHECK_FINITE"] = "1"
        proj = gs.project(cam, g)  # clean inputs pass
        binned = gs.BinSorter(0)(cam, proj)
        frame = gs.render_fwd(cam, proj, binned)
        gimg = torch.zeros((3, view.height, view.width), device="cuda")
        gs.render_bwd(cam, g, proj, binned, frame, gimg)
        bad = gs.Gaussians(*[t.clone() for t in g.tensors()])
        bad.sh[0, 1, 5] = float("nan")
        with pytest.raises(gs.GsError) as e:
            gs.project(cam, bad)
        assert e.value.status == gs.GS_ERR_NONFINITE and "sh" in str(e.value) and " 1 non-finite" in str(e.value)
        bad = gs.Gaussians(*[t.clone() for t in g.tensors()])
        bad.means[2, :3] = float("inf")
        with pytest.raises(gs.GsError) as e:
            gs.project(cam, bad)
        assert e.value.status == gs.GS_ERR_NONFINITE and "means" in str(e.value)
        gimg[1, 3, 4] = float("nan")
        with pytest.raises(gs.GsError) as e:
            gs.render_bwd(cam, g, proj, binned, frame, gimg)
        assert e.value.status == gs.GS_ERR_NONFINITE and "dL_dimage" in str(e.value)
        # off again: the same call goes through
        os.environ["GS_CHECK_FINITE"] = "0"
        gs.render_bwd(cam, g, proj, binned, frame, gimg)
        torch.cuda.synchronize()
    finally:
        if old is None:
            os.environ.pop("GS_CHECK_FINITE", None)
        else:
            os.environ["GS_CHECK_FINITE"] = old
