"""GPU parity of the guided-matching depth (through the C ABI) with the FP64
oracle in oracle/depth.py.

Decisions are compared exactly where the oracle does not flag them as
near-ties: the neighbour choice where no two separations, and no segment
end and the image border, come within 1e-3 px; the best candidate where its
correlation leads the runner-up by more than 1e-4 relative.  Where both
agree the inverse depth must match to 1e-3 of a candidate step (plus 2e-6
relative) wherever no fit applies or the parabola is well conditioned.
Cases: 1-4 neighbours, 8-64 channels, 3-33 candidates, ragged tiles,
monocular depths that are 0, negative, infinite or NaN, a neighbour that
sees none of the candidates, and the 1920x1080 frame sampled."""
import numpy as np
import pytest
import torch

from oracle import depth as gd
from paper_2506_05558_amd import synth

from .gpu_common import gpu

pytestmark = pytest.mark.gpu


def _poses(poses):
    return [(p[:9].reshape(3, 3).astype(np.float64), p[9:].astype(np.float64)) for p in poses]


def _flags(K, poses, zmono, n, W, H, out):
    """Pixels whose choice or best candidate sits on a near-tie."""
    d = gd.candidates(np.where(np.isfinite(zmono) & (zmono > 0), zmono, 1.0), n)
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    seps, margin = [], np.full((H, W), np.inf)
    for R, t in poses:
        u0, v0, _ = gd.reproject(K, R, t, xx, yy, d[0])
        u1, v1, _ = gd.reproject(K, R, t, xx, yy, d[-1])
        seps.append(np.hypot(u1 - u0, v1 - v0))
        for u, lim in ((u0, W - 1), (u1, W - 1), (v0, H - 1), (v1, H - 1)):
            margin = np.minimum(margin, np.minimum(np.abs(u), np.abs(u - lim)))
    seps = np.sort(np.stack(seps), axis=0)
    flag = margin < 1e-3
    if len(poses) > 1:
        flag |= (seps[-1] - seps[-2]) < 1e-3
    C = out["corr"]
    srt = np.sort(np.where(np.isfinite(C), C, -1e30), axis=0)
    top, second = srt[-1], srt[-2]
    # a pixel without any candidate (no neighbour, or Z* missing) decides nothing
    flag |= (top > -1e30) & ((top - second) <= 1e-4 * (np.abs(top) + 1e-3))
    return flag


def _run(gs, fi, fjs, poses, zm, K, n):
    dev = "cuda"
    depth, best, choice = gs.guided_depth(torch.tensor(fi, device=dev), [torch.tensor(f, device=dev) for f in fjs],
                                          poses, torch.tensor(zm, device=dev), *K, n_cand=n)
    torch.cuda.synchronize()
    return depth.cpu().numpy(), best.cpu().numpy(), choice.cpu().numpy()


def _check(name, dg, bg, cg, ref, flag, n, max_flagged=0.05):
    ok = ~flag
    assert flag.mean() < max_flagged, (name, flag.mean())
    assert np.array_equal(cg[ok], ref["choice"][ok]), name
    same = ok & (cg == ref["choice"])
    assert np.array_equal(bg[same], ref["best"][same]), name
    assert np.array_equal(np.isnan(dg[same]), np.isnan(ref["depth"][same])), name
    est = same & np.isfinite(ref["depth"])
    d = ref["cand"]
    step = (d[-1] - d[0]) / (n - 1)
    kb, C = ref["best"], ref["corr"]
    cm = np.take_along_axis(C, np.clip(kb - 1, 0, n - 1)[None], 0)[0]
    cb = np.take_along_axis(C, np.clip(kb, 0, n - 1)[None], 0)[0]
    cp = np.take_along_axis(C, np.clip(kb + 1, 0, n - 1)[None], 0)[0]
    with np.errstate(invalid="ignore"):
        end = (kb <= 0) | (kb >= n - 1) | ~np.isfinite(cm) | ~np.isfinite(cp)
        den = np.where(end, -1.0, cm - 2 * cb + cp)
        well = end | (np.abs(den) >= 1e-2 * np.maximum(np.abs(cb), 1e-3))
    cmp = est & well
    inv_g, inv_r = 1.0 / dg[cmp], 1.0 / ref["depth"][cmp]
    tol = 1e-3 * step[cmp] + 2e-6 * inv_r
    assert (np.abs(inv_g - inv_r) <= tol).all(), (name, np.abs(inv_g - inv_r).max())
    print(f"{name}: flagged {flag.mean():.2e}, compared {cmp.mean():.3f}, estimates {est.mean():.3f}")
    return cmp


def _compare(name, gs, fi, fjs, poses, zm, K, n):
    H, W, _ = fi.shape
    dg, bg, cg = _run(gs, fi, fjs, poses, zm, K, n)
    P = _poses(poses)
    ref = gd.guided_depth(fi, fjs, K, P, zm, n)
    _check(name, dg, bg, cg, ref, _flags(K, P, zm, n, W, H, ref), n)
    return ref, dg


# widths set the focal length (0.7 W): the candidate segments must span several pixels, or
# neighbouring candidates sample the same place and their correlations tie
@pytest.mark.parametrize("W,H,C,n,nb,seed", [(160, 96, 32, 32, 2, 1), (70, 13, 8, 3, 1, 2), (301, 41, 16, 33, 3, 3),
                                             (258, 30, 64, 17, 4, 4)])
def test_guided_depth_parity(W, H, C, n, nb, seed):
    gs = gpu()
    fi, fjs, poses, zm, _, K = synth.depth_frames(seed, W, H, C, nb)
    _compare(f"{W}x{H} C{C} n{n} nb{nb}", gs, fi, fjs, poses, zm, K, n)


def test_guided_depth_edge_cases():
    gs = gpu()
    fi, fjs, poses, zm, _, K = synth.depth_frames(5, 80, 24, 16, 2)
    zm[0, :4] = [0.0, -1.0, np.inf, np.nan]
    ref, dg = _compare("edges", gs, fi, fjs, poses, zm, K, 16)
    assert np.isnan(dg[0, :4]).all() and np.isnan(ref["depth"][0, :4]).all()
    # a neighbour whose view of every candidate leaves its image: no estimate anywhere
    away = np.concatenate([np.eye(3).reshape(9), [100.0, 0.0, 0.0]]).astype(np.float32)[None]
    dg, bg, cg = _run(gs, fi, fjs[:1], away, zm, K, 16)
    assert np.isnan(dg).all() and (bg == -1).all() and (cg == -1).all()


def test_guided_depth_full_frame_sampled():
    gs = gpu()
    fi, fjs, poses, zm, zt, K = synth.depth_frames(6, 1920, 1080, 32, 2)
    dg, bg, cg = _run(gs, fi, fjs, poses, zm, K, 32)
    rng = np.random.default_rng(0)
    mask = np.zeros(zm.shape, bool)
    mask[rng.integers(0, 1080, 3000), rng.integers(0, 1920, 3000)] = True
    P = _poses(poses)
    ref = gd.guided_depth(fi, fjs, K, P, zm, 32, mask=mask)
    flag = _flags(K, P, zm, 32, 1920, 1080, ref)
    # compare the sampled pixels only (the rest carry no oracle correlation)
    cmp = _check("1080p sampled", np.where(mask, dg, np.nan), np.where(mask, bg, -1), cg, ref, flag & mask, 32)
    assert cmp.sum() > 2000
