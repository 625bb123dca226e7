"""GPU parity of the joint-optimisation helpers (section 4.3) against the
float64 oracle in oracle/optim.py: the L1 loss, its sums and gradient; Adam,
dense and sparse (a Gaussian the step did not process keeps its parameter
and moments), over several parameter planes and ragged lengths; the 6D pose
map and its adjoint; the visibility mask; the fill kernel."""
import numpy as np
import pytest
import torch

from oracle import optim

from .gpu_common import gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("count", [1, 255, 257, 3 * 1920 * 1080])
def test_loss_l1(count):
    gs = gpu()
    rng = np.random.default_rng(count)
    a = rng.random(count).astype(np.float32)
    b = rng.random(count).astype(np.float32)
    b[: count // 7] = a[: count // 7]  # exact zeros: sign(0) = 0
    grad = torch.empty(count, device="cuda")
    sums = gs.loss_l1(torch.tensor(a, device="cuda"), torch.tensor(b, device="cuda"), 0.25, grad)
    s1, s2, g = optim.l1_loss(a, b, 0.25)
    got = sums.cpu().numpy()
    # the kernel forms I - I* in binary32 (one rounding, relative 2^-24) and sums in binary64
    assert abs(got[0] - s1) <= 1e-7 * max(s1, 1) and abs(got[1] - s2) <= 2e-7 * max(s2, 1)
    assert np.array_equal(grad.cpu().numpy(), g.astype(np.float32))


@pytest.mark.parametrize("planes,n,sparse", [(1, 1000, False), (3, 1001, True), (45, 4097, True), (4, 70_000, True)])
def test_adam(planes, n, sparse):
    gs = gpu()
    rng = np.random.default_rng(planes * n)
    shape = (planes, n)
    p, g = rng.standard_normal(shape).astype(np.float32), rng.standard_normal(shape).astype(np.float32)
    m, v = (rng.standard_normal(shape) * 0.1).astype(np.float32), (rng.random(shape) * 0.1).astype(np.float32)
    vis = (rng.random(n) < 0.6).astype(np.int32) if sparse else None
    dp, dg, dm, dv = (torch.tensor(x, device="cuda") for x in (p, g, m, v))
    gs.adam_step(dp, dg, dm, dv, 1e-3, 7, eps=1e-8, visible=None if vis is None else torch.tensor(vis, device="cuda"),
                 n_stride=n if sparse else 0)
    rp, rm, rv = optim.adam(p, g, m, v, 1e-3, 7, eps=1e-8, visible=vis, n_stride=n)
    assert np.abs(dp.cpu().numpy() - rp).max() <= 1e-6
    assert np.abs(dm.cpu().numpy() - rm).max() <= 1e-6 and np.abs(dv.cpu().numpy() - rv).max() <= 1e-6
    if sparse:
        hidden = vis == 0
        assert np.array_equal(dp.cpu().numpy()[:, hidden], p[:, hidden])
        assert np.array_equal(dm.cpu().numpy()[:, hidden], m[:, hidden])


def test_pose_6d_and_adjoint():
    gs = gpu()
    rng = np.random.default_rng(9)
    x = rng.standard_normal((8, 9)).astype(np.float32)
    pose = torch.empty((8, 12), device="cuda")
    gs.pose_from_6d(torch.tensor(x, device="cuda"), pose)
    assert np.abs(pose.cpu().numpy() - optim.pose_from_6d(x)).max() <= 1e-6
    dpose = rng.standard_normal((8, 12))
    dx = torch.zeros((8, 9), device="cuda")
    gs.pose_6d_bwd(torch.tensor(x, device="cuda"), torch.tensor(dpose, device="cuda"), dx)
    ref = optim.pose_6d_vjp(x.astype(np.float64), dpose)
    assert np.abs(dx.cpu().numpy() - ref).max() <= 1e-5 * (1 + np.abs(ref).max())


def test_mark_visible_and_zero():
    gs = gpu()
    rng = np.random.default_rng(3)
    tiles = rng.integers(-1, 3, 1000).astype(np.int32)
    proj = gs.alloc_projected(1000)
    proj.tiles_touched.copy_(torch.tensor(tiles))
    mask = torch.zeros(1000, dtype=torch.int32, device="cuda")
    mask[:5] = 1
    gs.mark_visible(proj, mask)
    want = (tiles > 0).astype(np.int32)
    want[:5] = 1
    assert np.array_equal(mask.cpu().numpy(), want)
    buf = torch.full((1234,), 7, dtype=torch.uint8, device="cuda")
    gs.zero_(buf[1:1000])  # odd offset and length: the byte path
    b = buf.cpu().numpy()
    assert b[0] == 7 and (b[1:1000] == 0).all() and (b[1000:] == 7).all()
    w = torch.full((777,), 3.0, device="cuda")
    gs.zero_(w)
    assert (w.cpu().numpy() == 0).all()
