"""GPU parity of the anchor decisions (section 4.4) with oracle/anchors.py:
the per-Gaussian size flags bit-exact away from ties (|f S - tau D| within
1e-12 of tau D), the small-Gaussian count and the 40 % decision equal to the
oracle's, for n = 0, 1, ragged and 2M Gaussians under a posed camera; the
opacity scaling to binary32 rounding of the FP64 definition, w = 0 giving
-inf."""
import numpy as np
import pytest
import torch

from oracle import anchors as an
from paper_2506_05558_amd import synth

from .gpu_common import gpu

pytestmark = pytest.mark.gpu


def _pose(seed):
    R, t = synth.perturb_pose(np.random.default_rng(seed), np.eye(3), np.array([0.3, -0.2, 1.0]), 0.2)
    return np.concatenate([np.asarray(R).reshape(9), t]).astype(np.float32)


@pytest.mark.parametrize("n", [0, 1, 1001, 2_000_000])
def test_anchor_sizes(n):
    gs = gpu()
    rng = np.random.default_rng(n + 3)
    means = rng.uniform(-20, 20, (3, n)).astype(np.float32)
    log_scales = rng.normal(-5.0, 1.5, (3, n)).astype(np.float32)
    pose = _pose(n)
    f = np.float32(1344.0)
    g = gs.Gaussians(torch.tensor(means, device="cuda"), torch.tensor(log_scales, device="cuda"),
                     torch.zeros((4, n), device="cuda"), torch.zeros(n, device="cuda"),
                     torch.zeros((1, 3, n), device="cuda"))
    flags = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    count = gs.anchor_sizes(g, pose, float(f), flags=flags[:n] if n else None)
    torch.cuda.synchronize()
    R, t = pose[:9].reshape(3, 3).astype(np.float64), pose[9:].astype(np.float64)
    ref, fS, tD = an.small_flags(means, log_scales, R, t, float(f))
    tie = np.abs(fS - tD) <= 1e-12 * tD
    got = flags[:n].cpu().numpy() != 0
    assert np.array_equal(got[~tie], ref[~tie])
    assert int(count.item()) == int(got.sum())
    if not tie.any():
        assert int(count.item()) == int(ref.sum())
        assert (count.item() > 0.4 * n) == an.trigger(means, log_scales, R, t, float(f))[2]
    if n > 1000:
        assert 0.05 < ref.mean() < 0.95  # the workload has both kinds


def test_scale_opacity():
    gs = gpu()
    rng = np.random.default_rng(8)
    lg = rng.normal(0, 3, 100_003).astype(np.float32)
    d = torch.tensor(lg, device="cuda")
    for w in (1.0, 0.7, 0.05):
        out = gs.scale_opacity(d, w).cpu().numpy()
        ref = an.scale_opacity_logits(lg, np.float32(w)).astype(np.float32)
        assert np.abs(out - ref).max() <= 1e-6 * (1 + np.abs(ref).max())
    out = gs.scale_opacity(d, 0.0).cpu().numpy()
    assert np.isneginf(out).all()
    # in place
    x = d.clone()
    gs.scale_opacity(x, 0.5, out=x)
    assert np.abs(x.cpu().numpy() - an.scale_opacity_logits(lg, 0.5).astype(np.float32)).max() < 1e-5
