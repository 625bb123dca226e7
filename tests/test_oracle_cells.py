"""Pins of the cell oracle (oracle/cells.py): k-means against scikit-learn's
Lloyd iterations from the same initial centroids, the centres of
well-separated blobs recovered exactly, the nearest-centroid rule against
brute force with ties to the lower index; sphere visibility against
projected samples of the sphere and known cases."""
import numpy as np

from oracle import cells


def test_kmeans_matches_sklearn_lloyd():
    from sklearn.cluster import KMeans
    rng = np.random.default_rng(0)
    means = rng.standard_normal((3, 3000)).astype(np.float32) * np.array([[4.0], [2.0], [1.0]], np.float32)
    k, iters = 12, 15
    cent, labels = cells.kmeans(means, k, iters)
    init = means[:, cells.init_indices(3000, k)].T.astype(np.float64)
    km = KMeans(n_clusters=k, init=init, n_init=1, max_iter=iters, tol=0.0, algorithm="lloyd")
    km.fit(means.T.astype(np.float64))
    assert np.allclose(cent, km.cluster_centers_, atol=1e-9)
    assert np.array_equal(labels, km.labels_)


def test_blobs_and_ties():
    rng = np.random.default_rng(1)
    centres = np.array([[0.0, 0, 0], [10, 0, 0], [0, 10, 0], [0, 0, 10]])
    pts = np.concatenate([c[:, None] + rng.normal(0, 0.1, (3, 500)) for c in centres], axis=1).astype(np.float32)
    cent, labels = cells.kmeans(pts, 4, 10)
    for c in centres:  # every blob centre within its sample mean's error
        assert np.linalg.norm(cent - c, axis=1).min() < 0.02
    # a point equidistant from two centroids joins the lower one
    lab = cells.assign(np.array([[0.5], [0.0], [0.0]], np.float32), np.array([[0.0, 0, 0], [1.0, 0, 0]]))
    assert lab.tolist() == [0]
    lab = cells.assign(np.array([[0.5], [0.0], [0.0]], np.float32), np.array([[1.0, 0, 0], [0.0, 0, 0]]))
    assert lab.tolist() == [0]


def test_sphere_visibility():
    R, t = np.eye(3), np.zeros(3)
    K = (100.0, 100.0, 50.0, 40.0, 100, 80)
    assert cells.sphere_visible([0, 0, 5], 0.1, R, t, *K)
    assert not cells.sphere_visible([0, 0, -5], 1.0, R, t, *K)
    assert cells.sphere_visible([0, 0, -5], 6.0, R, t, *K)
    # far to the right: x / z = 10 vs the widened half-width 1.3 * 0.5
    assert not cells.sphere_visible([50, 0, 5], 1.0, R, t, *K)
    # against samples: a sphere is visible iff some point of it projects into the widened image
    rng = np.random.default_rng(2)
    for _ in range(300):
        c = rng.uniform([-6, -6, -2], [6, 6, 10])
        r = rng.uniform(0.05, 1.5)
        d = rng.standard_normal((3, 20000))
        pts = c[:, None] + d / np.linalg.norm(d, axis=0) * r * rng.random(20000) ** (1 / 3)
        z = pts[2]
        u = pts[0] / np.maximum(z, 1e-9)
        v = pts[1] / np.maximum(z, 1e-9)
        inside = (z > 0.2) & (u <= 1.3 * 0.5) & (u >= -1.3 * 0.5) & (v <= 1.3 * 0.4) & (v >= -1.3 * 0.4)
        vis = cells.sphere_visible(c, r, R, t, *K)
        if inside.any():
            assert vis  # the test never drops a sphere that reaches into the frustum
