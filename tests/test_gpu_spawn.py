"""GPU parity of the spawn step (section 4.2, Eq. 1-3) against the oracle.

P_L and P_s are compared bit for bit with the oracle's fixed-order binary32
reference (every spawn decision is an integer function of them), the
selected pixel sets are compared exactly for both selection modes, and the
rule's parameters within float32 rounding of the float64 oracle.  Inputs:
the synthetic spawn frames of `synth.spawn_frame` at 1920x1080 and at ragged
sizes, sigma 1 and the extremes of the supported range."""
import numpy as np
import pytest
import torch

from oracle import spawn
from paper_2506_05558_amd import synth

from .gpu_common import gpu

pytestmark = pytest.mark.gpu


def _camera(W, H, seed=0):
    gs = gpu()
    rng = np.random.default_rng(seed)
    R = np.linalg.qr(rng.standard_normal((3, 3)))[0]
    R *= np.sign(np.linalg.det(R))
    t = rng.standard_normal(3)
    pose = np.concatenate([R.reshape(9), t]).astype(np.float32)
    f = 0.9 * W
    return gs.Camera(W, H, f, 1.05 * f, W / 2 - 0.3, H / 2 + 0.2, torch.tensor(pose, device="cuda")), pose


def _dev(a):
    return torch.tensor(a, device="cuda")


def _bits(a):
    return np.asarray(a, np.float32).view(np.uint32)


@pytest.mark.parametrize("W,H,sigma,first", [(1920, 1080, 1.0, False), (1920, 1080, 1.0, True),
                                             (37, 23, 1.0, False), (5, 3, 2.0, False), (100, 61, 0.6, False)])
def test_probability_bitwise(W, H, sigma, first):
    gs = gpu()
    img, ren, _ = synth.spawn_frame(11, W, H, n_rects=8 if W < 200 else 60)
    cam, _ = _camera(W, H)
    sp = gs.SpawnParams(sigma=sigma)
    pl, ps = gs.spawn_probability(cam, _dev(img), None if first else _dev(ren), sp)
    torch.cuda.synchronize()
    PL, PS = spawn.probability_f32(img, None if first else ren, float(np.float32(sigma)))
    assert np.array_equal(_bits(pl.cpu().numpy()), _bits(PL))
    assert np.array_equal(_bits(ps.cpu().numpy()), _bits(PS))
    if not first:
        assert (PS < PL).any()  # the rendered structure was penalised


def test_probability_of_a_perfect_render_is_zero():
    gs = gpu()
    img, _, _ = synth.spawn_frame(3, 300, 200)
    cam, _ = _camera(300, 200)
    x = _dev(img)
    _, ps = gs.spawn_probability(cam, x, x.clone())
    assert ps.abs().max().item() == 0.0


@pytest.mark.parametrize("W,H,seed", [(1920, 1080, 5), (333, 77, 2**64 - 3), (16, 16, 0)])
def test_bernoulli_selection_exact(W, H, seed):
    gs = gpu()
    img, ren, _ = synth.spawn_frame(21, W, H, n_rects=40 if W > 100 else 4)
    cam, _ = _camera(W, H)
    sp = gs.SpawnParams(seed=seed)
    _, ps = gs.spawn_probability(cam, _dev(img), _dev(ren), sp)
    pix = gs.spawn_select(cam, ps, sp)
    torch.cuda.synchronize()
    PL, PS = spawn.probability_f32(img, ren)
    ref = np.flatnonzero(spawn.mask_bernoulli(spawn.quantize(PS), seed))
    got = pix.cpu().numpy()
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("K", [0, 1, 5000, 40000, 10**7])
def test_fixed_k_selection_exact(K):
    gs = gpu()
    W, H = 640, 360
    img, ren, _ = synth.spawn_frame(31, W, H)
    cam, _ = _camera(W, H)
    sp = gs.SpawnParams(mode=gs.SPAWN_FIXED_K, k=K, seed=99)
    _, ps = gs.spawn_probability(cam, _dev(img), _dev(ren), sp)
    pix = gs.spawn_select(cam, ps, sp)
    torch.cuda.synchronize()
    _, PS = spawn.probability_f32(img, ren)
    off = spawn.splitmix64(99) >> 40
    q = spawn.quantize(PS)
    if K <= 40000:
        ref = np.flatnonzero(spawn.mask_fixed_k(q, K, off))
        assert np.array_equal(pix.cpu().numpy(), ref)
    else:
        # more thresholds than the oracle's loop visits in seconds: every pixel of
        # mass >= S/K holds a threshold, and no empty pixel is selected
        got = np.zeros(q.size, bool)
        got[pix.cpu().numpy()] = True
        S = int(q.sum())
        assert got[q.reshape(-1) * K >= S].all() and not got[q.reshape(-1) == 0].any()
    assert len(pix) <= K


def test_selection_edge_cases():
    gs = gpu()
    W, H = 64, 48
    cam, _ = _camera(W, H)
    flat = torch.full((3, H, W), 0.4, device="cuda")
    _, ps = gs.spawn_probability(cam, flat, None)
    # a constant image has no structure: the float32 taps sum to zero up to rounding,
    # far below the 2^-24 quantum of the decisions
    assert ps.abs().max().item() < 2.0 ** -24
    for sp in (gs.SpawnParams(), gs.SpawnParams(mode=gs.SPAWN_FIXED_K, k=100)):
        assert gs.spawn_select(cam, ps, sp).numel() == 0
    ones = torch.ones((H, W), device="cuda")  # P_s = 1: every pixel spawns under Bernoulli
    assert torch.equal(gs.spawn_select(cam, ones, gs.SpawnParams()).cpu(), torch.arange(W * H, dtype=torch.int32))
    with pytest.raises(gs.GsError) as e:
        gs.spawn_select(cam, ones, gs.SpawnParams(), capacity=10)
    assert e.value.status == gs.GS_ERR_CAPACITY


def test_rule_attributes():
    gs = gpu()
    W, H = 1920, 1080
    img, ren, depth = synth.spawn_frame(41, W, H)
    cam, pose = _camera(W, H, seed=4)
    sp = gs.SpawnParams(seed=7)
    pl, ps = gs.spawn_probability(cam, _dev(img), _dev(ren), sp)
    pix = gs.spawn_select(cam, ps, sp)
    n = len(pix)
    assert n > 1000
    # the expected attributes take P_L and the selected pixels from the oracle
    # (both are bit-exact there, which the selection tests check on their own)
    PL_ref, PS_ref = spawn.probability_f32(img, ren)
    pix_ref = np.flatnonzero(spawn.mask_bernoulli(spawn.quantize(PS_ref), 7))
    assert np.array_equal(pix.cpu().numpy(), pix_ref)
    for deg in (0, 3):
        off = 17
        nb = (deg + 1) ** 2
        out = gs.Gaussians(torch.full((3, n + off), 7.0, device="cuda"), torch.full((3, n + off), 7.0, device="cuda"),
                           torch.full((4, n + off), 7.0, device="cuda"), torch.full((n + off,), 7.0, device="cuda"),
                           torch.full((nb, 3, n + off), 7.0, device="cuda"))
        gs.spawn_rule(cam, _dev(img), _dev(depth), pl, pix, out, offset=off, sp=sp)
        torch.cuda.synchronize()
        R, t = pose[:9].reshape(3, 3).astype(np.float64), pose[9:].astype(np.float64)
        f32 = lambda x: float(np.float32(x))
        ref = spawn.rule_attributes(pix_ref, PL_ref, img, depth, R, t, f32(cam.fx), f32(cam.fy),
                                    f32(cam.cx), f32(cam.cy), opacity=f32(0.1), min_prob=f32(1e-4))
        m = out.means.cpu().numpy().astype(np.float64)
        assert (m[:, :off] == 7.0).all()  # entries before the offset untouched
        scale = np.abs(ref["means"]).max() + 1.0
        assert np.abs(m[:, off:] - ref["means"]).max() < 4e-6 * scale
        assert np.abs(out.log_scales.cpu().numpy()[:, off:] - ref["log_scales"]).max() < 2e-5
        assert np.abs(out.quats.cpu().numpy()[:, off:] - ref["quats"]).max() < 2e-6
        assert np.abs(out.opacity_logits.cpu().numpy()[off:] - ref["opacity_logits"]).max() < 1e-5
        sh = out.sh.cpu().numpy()
        assert np.abs(sh[0, :, off:] - ref["sh0"]).max() < 2e-6
        if deg:
            assert (sh[1:, :, off:] == 0).all()
