"""gs_render_fwd_l1_noalloc (fixed library scratch, no workspace) against
gs_render_fwd_l1 (caller workspace) through the C ABI: two calls in a row on
one GPU, the second on a smaller image, each equal bit for bit to the
workspace form on the same inputs (the same kernels, so every output and
both loss sums agree exactly), and an image beyond the fixed scratch is
refused with an error."""
import numpy as np
import pytest
import torch

from paper_2506_05558_amd import synth
from tests import gpu_common as gc

pytestmark = pytest.mark.gpu


def _frame(gs, H, W):
    f = lambda *s, dt=torch.float32: torch.full(s, -7.0, dtype=dt, device="cuda") if dt == torch.float32 \
        else torch.full(s, -7, dtype=dt, device="cuda")
    return gs.Frame(f(3, H, W), f(H, W), f(H, W), f(H, W), f(H, W, dt=torch.int32))


def _case(gs, view, scene, seed):
    params = gs.Params(eps2d=0.1, mip_filter=1)
    cam = gc.gpu_camera(view)
    g = gc.gpu_gauss(scene)
    proj = gs.project(cam, g, params)
    binned = gs.BinSorter(0)(cam, proj)
    H, W = view.height, view.width
    tgt = torch.tensor(np.random.default_rng(seed).random((3, H, W)).astype(np.float32), device="cuda")
    scale = 1.0 / (3 * H * W)
    ref, ref_g, ref_s = _frame(gs, H, W), torch.empty((3, H, W), device="cuda"), torch.empty(2, dtype=torch.float64,
                                                                                             device="cuda")
    gs.render_fwd_l1(cam, proj, binned, tgt, scale, ref_g, ref_s, params=params, out=ref)
    out, got_g, got_s = _frame(gs, H, W), torch.full((3, H, W), 5.0, device="cuda"), torch.full(
        (2,), 5.0, dtype=torch.float64, device="cuda")
    gs.render_fwd_l1_noalloc(cam, proj, binned, tgt, scale, got_g, got_s, out, params)
    torch.cuda.synchronize()
    for a, b in zip([out.image, out.depth, out.alpha, out.final_t, out.n_contrib, got_g, got_s],
                    [ref.image, ref.depth, ref.alpha, ref.final_t, ref.n_contrib, ref_g, ref_s]):
        assert torch.equal(a, b)
    # the loss sums also match their definition on the rendered image
    d = (ref.image.double() - tgt.double())
    assert abs(float(got_s[0]) - float(d.abs().sum())) <= 1e-9 * float(d.abs().sum())
    print(f"noalloc {W}x{H}: {binned.n_instances} pairs, L1 sum {float(got_s[0]):.6f}")


def test_noalloc_forward_l1_matches_workspace_form_twice():
    gs = gc.gpu()
    view, scene = synth.single_view(3, width=1296, height=840, n=200_000)
    _case(gs, view, scene, 1)
    small, sscene, _ = synth.tiny_scene(4)
    _case(gs, small, sscene, 2)


def test_noalloc_refuses_images_beyond_the_scratch():
    gs = gc.gpu()
    view, scene, _ = synth.tiny_scene(5)
    cam = gc.gpu_camera(view)
    g = gc.gpu_gauss(scene)
    proj = gs.project(cam, g)
    binned = gs.BinSorter(0)(cam, proj)
    big = gs.Camera(4112, 4096, cam.fx, cam.fy, cam.cx, cam.cy, cam.pose)  # 257 x 256 tiles > 65,536
    H, W = 4096, 4112
    buf = lambda *s: torch.empty(s, dtype=torch.float32, device="cuda")
    out = gs.Frame(buf(3, H, W), buf(H, W), buf(H, W), buf(H, W), torch.empty((H, W), dtype=torch.int32,
                                                                               device="cuda"))
    with pytest.raises(gs.GsError) as e:
        gs.render_fwd_l1_noalloc(big, proj, binned, buf(3, H, W), 1.0, buf(3, H, W),
                                 torch.empty(2, dtype=torch.float64, device="cuda"), out)
    assert e.value.status == gs.GS_ERR_INVALID_ARG and "scratch" in str(e.value)
