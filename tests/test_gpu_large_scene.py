"""The large-scene residency through the library: cells copied between the
pinned host store and the device page pool and back (a round trip is bit
for bit), the unused columns of the pages culled, the resident pool
rendering what the whole scene renders from a window view, and a 2560x1440
crop of the resident pool against the FP64 oracle; then a few keyframes of
joint optimisation over a residency that changes along the trajectory."""
import numpy as np
import pytest
import torch

from oracle import raster as orc
from paper_2506_05558_amd import gsmi, large_scene as L, synth
from tests import gpu_common as gc

pytestmark = pytest.mark.gpu


def _small(frames=12, per_frame=20_000, cells=24, window=3, iters=3):
    cfg = L.Config(frames=frames, per_frame=per_frame, cells=cells, kmeans_iters=10, window=window, iters=iters,
                   spawn_k=20_000)
    return L.LargeScene(cfg, log=print)


def _resident_columns(ls):
    op = ls.pool.g.opacity_logits.cpu().numpy()
    return np.nonzero(op > L.CULLED_LOGIT)[0]


def test_residency_round_trip_and_cull():
    ls = _small()
    res, pool, st = ls.res, ls.pool, ls.store
    need = res.needed([ls.cams[i] for i in ls.window(5)])
    res.update(need)
    torch.cuda.synchronize()
    cols = _resident_columns(ls)
    assert cols.size == sum(int(st.count[j]) for j in need)
    # each resident cell's rows on the device equal its host block
    for j in list(need)[:4]:
        blk = st.host[st.off[j]:st.off[j + 1]].view(st.R, int(st.count[j]))
        dev = torch.cat([pool.buf[:, p * L.PAGE:(p + 1) * L.PAGE] for p in res.pages[j]], dim=1)
        assert torch.equal(dev[:, :blk.shape[1]].cpu(), blk)
    # change the device copy of one cell, evict it (write-back), reload it
    j = sorted(need)[0]
    p0 = res.pages[j][0]
    pool.buf[:, p0 * L.PAGE:p0 * L.PAGE + 5] += 1.0
    expect = torch.cat([pool.buf[:, p * L.PAGE:(p + 1) * L.PAGE] for p in res.pages[j]], dim=1)[:, :int(st.count[j])]
    expect = expect.cpu()
    res.update(need - {j})
    torch.cuda.synchronize()
    assert j not in res.pages
    assert float(pool.g.opacity_logits[p0 * L.PAGE:(p0 + 1) * L.PAGE].max()) == L.CULLED_LOGIT
    blk = st.host[st.off[j]:st.off[j + 1]].view(st.R, int(st.count[j]))
    assert torch.equal(blk, expect)
    res.update(need)
    torch.cuda.synchronize()
    dev = torch.cat([pool.buf[:, p * L.PAGE:(p + 1) * L.PAGE] for p in res.pages[j]], dim=1)[:, :int(st.count[j])]
    assert torch.equal(dev.cpu(), expect)
    assert _resident_columns(ls).size == sum(int(st.count[c]) for c in need)


def test_resident_pool_renders_the_whole_scene():
    ls = _small()
    f = 7
    win = ls.window(f)
    ls.res.update(ls.res.needed([ls.cams[i] for i in win]))
    # the whole optimised scene (every cell) on the device, in store order
    st = ls.store
    whole = torch.cat([st.host[st.off[j]:st.off[j + 1]].view(st.R, int(st.count[j]))[:L.param_rows(3)]
                       for j in range(st.k)], dim=1).cuda()
    g_all = L._gauss_view(whole.contiguous(), 3)
    for i in win:
        cam = ls.cams[i]
        p = gsmi.project(cam, ls.pool.g, ls.params)
        img_pool = gsmi.render_fwd(cam, p, gsmi.BinSorter()(cam, p), ls.params).image.clone()
        q = gsmi.project(cam, g_all, ls.params)
        img_all = gsmi.render_fwd(cam, q, gsmi.BinSorter()(cam, q), ls.params).image
        diff = (img_pool - img_all).abs()
        # the same Gaussians in another order: equal unless two depths tie
        assert float(diff.max()) <= 1e-4 and float((diff > 1e-6).float().mean()) < 1e-4, float(diff.max())


def test_resident_pool_crop_against_oracle():
    ls = _small(frames=8, per_frame=30_000, cells=16)
    f = 6
    ls.res.update(ls.res.needed([ls.cams[i] for i in ls.window(f)]))
    cam = ls.cams[f]
    pr = gsmi.project(cam, ls.pool.g, ls.params)
    fr = gsmi.render_fwd(cam, pr, gsmi.BinSorter()(cam, pr), ls.params)
    torch.cuda.synchronize()
    cols = _resident_columns(ls)
    arr = {k: v.detach().cpu().numpy()[..., cols] for k, v in zip(
        ["means", "log_scales", "quats", "opacity_logits", "sh"], ls.pool.g.tensors())}
    og = orc.Gaussians(arr["means"], arr["log_scales"], arr["quats"], arr["opacity_logits"], arr["sh"], 3)
    pose = cam.pose.cpu().numpy().astype(np.float64)
    ocam = orc.Camera(pose[:9].reshape(3, 3), pose[9:], float(np.float32(cam.fx)), float(np.float32(cam.fy)),
                      float(np.float32(cam.cx)), float(np.float32(cam.cy)), cam.width, cam.height,
                      eps2d=0.1, mip_filter=1)
    op = orc.project(ocam, og)
    for crop in [(1264, 704, 32, 32), (0, 0, 24, 24)]:
        ref = orc.render(ocam, op, crop=crop, flag_rel=1e-5)
        ok = ref["flags"] == 0
        assert 1 - ok.mean() < 0.01
        x0, y0, w, h = crop
        img = fr.image.cpu().numpy()[:, y0:y0 + h, x0:x0 + w]
        err = np.abs(img - ref["image"])[:, ok].max(initial=0)
        print(f"crop {crop[:2]}: image error {err:.2e} over {int(ok.sum())} pixels")
        assert err <= 1e-4


def test_keyframes_with_changing_residency():
    ls = _small(frames=10, window=3, iters=3)
    psnr = []
    for f in range(10):
        win = ls.keyframe(f, ls.cfg.iters)
        torch.cuda.synchronize()
        ls.check_lists(win)
        psnr.append(ls.psnr(win))
        assert np.isfinite(psnr[-1])
    assert ls.res.loads >= len(ls.res.pages) > 0
    assert ls.res.loads - ls.res.evictions == len(ls.res.pages)
    assert ls.n_spawned[-1] > 0
    # everything written back is finite and the host store holds every Gaussian once
    st = ls.store
    assert int(st.count.sum()) == ls.n_scene
    print(f"keyframes: PSNR {psnr[0]:.2f} -> {psnr[-1]:.2f}, loads {ls.res.loads}, evictions {ls.res.evictions}")
