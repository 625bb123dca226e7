"""GPU parity of anchor merging (section 4.4) with oracle/anchors.py, through
the C ABI: the selection, the k nearest neighbours, the owners, the new
indices and the kept list bit for bit (brute-force oracle), and every merged
Gaussian against the oracle's FP64 merge -- mean, covariance (rebuilt from
the stored rotation and log-scales, the part that is unique), opacity and
SH -- with the kept Gaussians equal bit for bit to their sources.  Cases:
random clouds with k = 1, 3 and 8, coincident points (every distance tied),
fewer candidates than k, isolated selected points (the brute-force
fallback), no fine primitive, n = 0, a 20k-Gaussian ray scene flagged by the
size test, and a 2M-Gaussian window scene checked on sampled selected
primitives (brute force each) and by the ownership property."""
import numpy as np
import pytest
import torch

from oracle import anchors as an
from paper_2506_05558_amd import synth

from .gpu_common import gpu

pytestmark = pytest.mark.gpu


def _params(scene):
    return dict(means=scene.means, log_scales=scene.log_scales, quats=scene.quats,
                opacity_logits=scene.opacity_logits, sh=scene.sh)


def _random_scene(rng, n, deg=1, spread=1.0):
    return synth.Scene((rng.standard_normal((3, n)) * spread).astype(np.float32),
                       rng.normal(-3.0, 0.4, (3, n)).astype(np.float32),
                       rng.standard_normal((4, n)).astype(np.float32),
                       rng.standard_normal(n).astype(np.float32),
                       rng.standard_normal(((deg + 1) ** 2, 3, n)).astype(np.float32), deg)


def _run(scene, fine, k, seed):
    gs = gpu()
    g = gs.Gaussians.from_arrays(scene.arrays())
    f = torch.tensor(np.asarray(fine, np.int32), device="cuda")
    plan = gs.anchor_merge_plan(g, f, k, seed)
    out, merged = gs.anchor_merge_apply(g, plan)
    torch.cuda.synchronize()
    return plan, out, merged


def _check(scene, fine, k, seed, name):
    plan, out, merged = _run(scene, fine, k, seed)
    p = _params(scene)
    cls, nbr, own, keep = an.merge_plan(p, fine, k, seed)
    assert np.array_equal(plan.cls.cpu().numpy(), cls), name
    assert np.array_equal(plan.nbr.cpu().numpy(), nbr), name
    assert np.array_equal(plan.owner.cpu().numpy(), own), name
    assert np.array_equal(plan.keep_index.cpu().numpy(), keep), name
    new_index = np.full(cls.size, -1, np.int32)
    new_index[keep] = np.arange(keep.size)
    assert np.array_equal(plan.new_index.cpu().numpy(), new_index), name
    groups = an.merge_groups(p, cls, own)
    got = {key: t.cpu().numpy() for key, t in zip(["means", "log_scales", "quats", "opacity_logits", "sh"],
                                                  out.tensors())}
    mflag = merged.cpu().numpy()
    is_merged = np.zeros(keep.size, bool)
    for s, ref in groups.items():
        j = new_index[s]
        is_merged[j] = True
        scale = 1.0 + np.abs(ref["mean"]).max()
        assert np.abs(got["means"][:, j] - ref["mean"]).max() <= 2e-6 * scale, (name, s)
        cov = an.covariance(got["log_scales"][:, j].astype(np.float64), got["quats"][:, j].astype(np.float64))
        assert np.abs(cov - ref["cov"]).max() <= 1e-5 * np.abs(ref["cov"]).max(), (name, s)
        op = 1.0 / (1.0 + np.exp(-np.float64(got["opacity_logits"][j])))
        assert abs(op - ref["opacity"]) <= 1e-6, (name, s, op, ref["opacity"])
        assert np.abs(got["sh"][:, :, j] - ref["sh"]).max() <= 1e-6 * (1 + np.abs(ref["sh"]).max()), (name, s)
    assert np.array_equal(mflag != 0, is_merged), name
    for key in got:  # every other kept Gaussian is its source, bit for bit
        src = np.asarray(p[key])[..., keep]
        assert np.array_equal(got[key][..., ~is_merged], src[..., ~is_merged]), (name, key)
    print(f"{name}: {int((cls == 1).sum())} selected, {int((own >= 0).sum())} absorbed, {len(groups)} merged, "
          f"{keep.size} kept of {cls.size}")


@pytest.mark.parametrize("k", [1, 3, 8])
def test_merge_random_cloud(k):
    rng = np.random.default_rng(10 + k)
    scene = _random_scene(rng, 3000)
    _check(scene, rng.random(3000) < 0.7, k, 77 + k, f"cloud k={k}")


def test_merge_edge_cases():
    rng = np.random.default_rng(5)
    # coincident points: every distance is 0 and ties go to the lower index
    sc = _random_scene(rng, 64)
    sc.means[:] = np.float32(0.25)
    _check(sc, np.ones(64, bool), 3, 1, "coincident")
    # fewer candidates than k: everything fine, k = 8, 6 Gaussians
    _check(_random_scene(rng, 6), np.ones(6, bool), 8, 3, "few")
    # isolated selected points far from the candidates' cloud (the fallback scans)
    sc = _random_scene(rng, 500, spread=0.1)
    sc.means[:, :40] += np.float32(50.0) * rng.standard_normal((3, 40)).astype(np.float32)
    _check(sc, np.ones(500, bool), 3, 11, "isolated")
    # no fine primitive: nothing selected, everything kept
    _check(_random_scene(rng, 100), np.zeros(100, bool), 3, 2, "none fine")
    # one Gaussian
    _check(_random_scene(rng, 1), np.ones(1, bool), 3, 0, "one")
    gs = gpu()
    empty = gs.Gaussians(*[torch.zeros(s, device="cuda") for s in [(3, 0), (3, 0), (4, 0), (0,), (1, 3, 0)]])
    plan = gs.anchor_merge_plan(empty, torch.zeros(0, dtype=torch.int32, device="cuda"), 3, 0)
    assert plan.keep_index.numel() == 0


def test_merge_ray_scene_size_flags():
    # a 20k-Gaussian ray scene (surfaces in depth), too-fine flags from the
    # size test at a camera 15 units behind the first keyframe
    views = synth.trajectory(3, 2, 640, 360)
    scene = synth.window_scene(3, views, 10_000, 1)
    R, t = views[0].R, views[0].t + np.array([0.0, 0.0, 15.0])
    fine, _, _ = an.small_flags(scene.means, scene.log_scales, R, t, views[0].fx)
    assert 0.0 < fine.mean() < 1.0, fine.mean()
    _check(scene, fine, 3, 4242, "ray scene")


def test_merge_two_million_sampled():
    gs = gpu()
    views = synth.trajectory(2506, 8, 1920, 1080)
    scene = synth.window_scene(2506, views, 250_000, 0)
    R, t = views[-1].R, views[-1].t + np.array([0.0, 0.0, 12.0])
    fine, _, _ = an.small_flags(scene.means, scene.log_scales, R, t, views[0].fx)
    plan, out, merged = _run(scene, fine, 3, 99)
    cls = an.merge_classes(fine, 3, 99)
    assert np.array_equal(plan.cls.cpu().numpy(), cls)
    nbr = plan.nbr.cpu().numpy()
    own = plan.owner.cpu().numpy()
    cand = np.flatnonzero(cls == an.CLS_CAND)
    seeds = np.flatnonzero(cls == an.CLS_SEED)
    m64 = scene.means.astype(np.float64)

    def d2(a, b):  # (dx dx + dy dy) + dz dz, as the oracle's sq_dist
        d = m64[:, b] - m64[:, a]
        return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]

    rng = np.random.default_rng(0)
    for s in rng.choice(seeds, 200, replace=False):  # brute force per sampled selected primitive
        order = np.lexsort((cand, d2(np.full(cand.size, s), cand)))[:3]
        assert np.array_equal(nbr[s], cand[order]), s
    # ownership: each absorbed candidate belongs to its smallest (binary32 d2, index) claim
    S = np.repeat(seeds, 3)
    J = nbr[seeds].ravel()
    ok = J >= 0
    S, J = S[ok], J[ok]
    D = d2(S, J).astype(np.float32)
    order = np.lexsort((S, D, J))
    first = np.ones(order.size, bool)
    first[1:] = J[order][1:] != J[order][:-1]
    want = np.full(cls.size, -1, np.int64)
    want[J[order][first]] = S[order][first]
    assert np.array_equal(own, want)
    keep = plan.keep_index.cpu().numpy()
    assert np.array_equal(keep, np.flatnonzero(own < 0))
    assert out.n == keep.size and int(merged.sum()) == len(set(own[own >= 0].tolist()))
    print(f"2M: {fine.sum()} fine, {seeds.size} selected, {(own >= 0).sum()} absorbed, {keep.size} kept")
