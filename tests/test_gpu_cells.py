"""Spatial cells of the large scene through the C ABI against the oracle
(oracle/cells.py): the nearest-centroid assignment bit for bit (ties to the
lower centroid included), one Lloyd step from the same centroids, a whole
k-means run, the stable cell order and offsets, the bounding spheres, and
the frustum test; then the 6M-Gaussian scene of the large-scene workload
(200 keyframes at 2560x1440) on sampled means."""
import numpy as np
import pytest
import torch

from oracle import cells as oc
from paper_2506_05558_amd import synth
from tests import gpu_common as gc

pytestmark = pytest.mark.gpu


def _blobs(seed, n, k):
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-20, 20, (k, 3))
    lab = rng.integers(0, k, n)
    pts = centres[lab].T + rng.normal(0, 2.0, (3, n))
    return pts.astype(np.float32)


def test_assign_bit_exact_with_ties():
    gs = gc.gpu()
    rng = np.random.default_rng(0)
    means = _blobs(1, 100_003, 37)
    cent = rng.uniform(-20, 20, (37, 3))
    # exact ties: a mean midway between centroids 5 and 30 (representable)
    cent[5] = [1.0, 2.0, 3.0]
    cent[30] = [3.0, 2.0, 3.0]
    means[:, 7] = [2.0, 2.0, 3.0]
    cent[30], cent[5] = cent[5].copy(), cent[30].copy()  # the tie goes to index 5 either way
    got = gs.cells_assign(torch.tensor(means, device="cuda"), torch.tensor(cent, device="cuda")).cpu().numpy()
    ref = oc.assign(means, cent)
    assert np.array_equal(got, ref)
    assert got[7] == 5


def test_one_lloyd_step_and_whole_run():
    gs = gc.gpu()
    means = _blobs(2, 150_000, 24)
    m = torch.tensor(means, device="cuda")
    rng = np.random.default_rng(3)
    c0 = means[:, rng.choice(means.shape[1], 24, replace=False)].T.astype(np.float64)
    cent, labels, order, offsets = gs.cells_kmeans(m, 24, 1, centroids=torch.tensor(c0, device="cuda"))
    ref = oc.update(means, oc.assign(means, c0), c0)
    assert np.allclose(cent.cpu().numpy(), ref, rtol=1e-12, atol=1e-12)
    # the final assignment is the oracle's for the GPU's centroids, bit for bit
    lab = labels.cpu().numpy()
    assert np.array_equal(lab, oc.assign(means, cent.cpu().numpy()))
    assert np.array_equal(order.cpu().numpy(), np.argsort(lab, kind="stable"))
    counts = np.bincount(lab, minlength=24)
    assert np.array_equal(offsets.cpu().numpy(), np.concatenate([[0], np.cumsum(counts)]))
    # 12 iterations from the spread start against the oracle's run
    cent, labels, _, _ = gs.cells_kmeans(m, 24, 12, with_order=False)
    rc, rl = oc.kmeans(means, 24, 12)
    assert np.allclose(cent.cpu().numpy(), rc, rtol=1e-9, atol=1e-9)
    assert (labels.cpu().numpy() != rl).mean() <= 1e-4
    print(f"k-means: {int((labels.cpu().numpy() != rl).sum())} labels differ after 12 iterations")


def test_spheres_and_visibility():
    gs = gc.gpu()
    means = _blobs(4, 80_000, 16)
    rng = np.random.default_rng(5)
    ls = rng.normal(-3, 0.5, (3, means.shape[1])).astype(np.float32)
    m, l = torch.tensor(means, device="cuda"), torch.tensor(ls, device="cuda")
    cent, labels, _, _ = gs.cells_kmeans(m, 16, 5, with_order=False)
    rad = gs.cells_spheres(m, l, labels, cent, margin=3.0).cpu().numpy()
    ref = oc.cell_spheres(means, ls, labels.cpu().numpy(), cent.cpu().numpy(), 3.0)
    assert np.allclose(rad, ref, rtol=1e-14, atol=0)
    # frustum test on random spheres and cameras
    k = 256
    centres = rng.uniform([-30, -30, -30], [30, 30, 30], (k, 3))
    radii = rng.uniform(0.1, 8.0, k)
    disagree = 0
    for s in range(12):
        R, t = synth.random_pose(rng, max_deg=60.0, trans=5.0)
        pose = torch.tensor(np.concatenate([R.reshape(9), t]).astype(np.float32), device="cuda")
        W, H = 2560, 1440
        cam = gs.Camera(W, H, 0.7 * W, 0.7 * W, W / 2, H / 2, pose)
        vis = gs.cells_visible(torch.tensor(centres, device="cuda"), torch.tensor(radii, device="cuda"),
                               cam).cpu().numpy()
        Rf = pose.cpu().numpy()[:9].astype(np.float64).reshape(3, 3)
        tf = pose.cpu().numpy()[9:].astype(np.float64)
        for j in range(k):
            ref = oc.sphere_visible(centres[j], radii[j], Rf, tf, 0.7 * W, 0.7 * W, W / 2, H / 2, W, H)
            disagree += int(bool(vis[j]) != ref)
    assert disagree == 0


def test_large_scene_cells_sampled():
    """The large-scene workload: 6M Gaussians seeded from 200 keyframes of a
    2560x1440 trajectory, 120 cells, 20 Lloyd iterations."""
    gs = gc.gpu()
    views = synth.trajectory(2560, 200, 2560, 1440)
    scene = synth.window_scene(2560, views, 30_000)
    means = scene.means
    m = torch.tensor(means, device="cuda")
    cent, labels, order, offsets = gs.cells_kmeans(m, 120, 20)
    torch.cuda.synchronize()
    c = cent.cpu().numpy()
    lab = labels.cpu().numpy()
    rng = np.random.default_rng(6)
    idx = rng.choice(means.shape[1], 20_000, replace=False)
    assert np.array_equal(lab[idx], oc.assign(means[:, idx], c))
    # one more Lloyd step from these centroids against the oracle's step
    c1, _, _, _ = gs.cells_kmeans(m, 120, 1, centroids=cent.clone(), with_order=False)
    ref = oc.update(means, oc.assign(means, c), c)
    assert np.allclose(c1.cpu().numpy(), ref, rtol=1e-12, atol=1e-12)
    counts = np.diff(offsets.cpu().numpy())
    assert counts.sum() == means.shape[1] and np.array_equal(counts, np.bincount(lab, minlength=120))
    o = order.cpu().numpy()
    assert np.all(np.diff(lab[o]) >= 0)
    print(f"cells: {counts.min()}..{counts.max()} Gaussians (mean {counts.mean():.0f})")
