"""GPU parity of the spawn MLP against the oracle (oracle/mlp.py).

Features exactly as defined (RGB patch values bit-equal, log depth ratios
to float32 rounding); the BF16 matrix-core forward against the oracle's
BF16-emulating forward at 1e-2 of the output scale; the fused spawn path
(rule + residuals gathered in-kernel) against the oracle rule plus the
oracle network; the FP32 training step's loss and gradient against the
float64 definition (1e-3 relative, per tensor and per element) and five
Adam steps against the oracle's Adam.  Batches cover one sample, ragged
tails of the 16-sample MFMA groups and 64-sample training chunks, and the
100k-sample size of a full 1080p spawn."""
import numpy as np
import pytest
import torch

from oracle import mlp, spawn
from paper_2506_05558_amd import synth

from .gpu_common import gpu

pytestmark = pytest.mark.gpu


def _camera(W, H):
    gs = gpu()
    pose = np.concatenate([np.eye(3).reshape(9), [0.1, -0.2, 0.3]]).astype(np.float32)
    return gs.Camera(W, H, 0.7 * W, 0.7 * W, W / 2, H / 2, torch.tensor(pose, device="cuda"))


def _frame(W=320, H=200, seed=1):
    img, ren, depth = synth.spawn_frame(seed, W, H, n_rects=20)
    return img, ren, depth


def _pixels(W, H, n, seed):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(W * H, n, replace=False)).astype(np.int32)


def _grad_close(g, ref, tol=1e-3):
    g, ref = np.asarray(g, np.float64), np.asarray(ref, np.float64)
    assert np.linalg.norm(g - ref) <= tol * np.linalg.norm(ref)
    assert (np.abs(g - ref) <= tol * (np.abs(ref) + 1e-3 * np.abs(ref).max())).all()


def test_features_match_definition():
    gs = gpu()
    W, H = 320, 200
    img, _, depth = _frame(W, H)
    pix = np.concatenate([[0, W - 1, W * H - 1, (H - 1) * W, 3 * W + 3], _pixels(W, H, 300, 2)]).astype(np.int32)
    f = gs.mlp_features(_camera(W, H), torch.tensor(img, device="cuda"), torch.tensor(depth, device="cuda"),
                        torch.tensor(pix, device="cuda")).cpu().numpy()
    ref = mlp.features(img, depth, pix)
    assert np.array_equal(f[:, :147], ref[:, :147].astype(np.float32))  # gathered colours: exact
    assert np.abs(f[:, 147:] - ref[:, 147:]).max() < 4e-6  # float32 log of a ratio in [1/20, 20]


@pytest.mark.parametrize("count", [1, 15, 16, 17, 1000])
def test_forward_bf16(count):
    gs = gpu()
    rng = np.random.default_rng(count)
    theta = synth.mlp_init(3, last_scale=1.0)
    theta[mlp.n_params() - 7:] = rng.standard_normal(7) * 0.1  # nonzero output bias
    X = rng.standard_normal((count, 196)).astype(np.float32)
    packed = gs.mlp_pack_bf16(torch.tensor(theta, device="cuda"))
    y = gs.mlp_forward_bf16(packed, torch.tensor(X, device="cuda")).cpu().numpy()
    ref = mlp.forward_bf16(theta.astype(np.float64), X.astype(np.float64))
    scale = np.abs(ref).max()
    assert np.abs(y - ref).max() <= 1e-2 * scale
    # and within BF16 rounding of the exact network
    ref64, _ = mlp.forward_f64(theta.astype(np.float64), X.astype(np.float64))
    assert np.abs(y - ref64).max() <= 5e-2 * scale


def test_forward_bf16_100k_sampled():
    gs = gpu()
    count = 100_000
    rng = np.random.default_rng(7)
    theta = synth.mlp_init(4, last_scale=1.0)
    X = rng.standard_normal((count, 196)).astype(np.float32)
    y = gs.mlp_forward_bf16(gs.mlp_pack_bf16(torch.tensor(theta, device="cuda")),
                            torch.tensor(X, device="cuda")).cpu().numpy()
    rows = np.concatenate([rng.choice(count, 500, replace=False), [0, count - 1]])
    ref = mlp.forward_bf16(theta.astype(np.float64), X[rows].astype(np.float64))
    assert np.abs(y[rows] - ref).max() <= 1e-2 * np.abs(ref).max()


def test_spawn_mlp_fused_equals_rule_plus_network():
    gs = gpu()
    W, H = 640, 360
    img, ren, depth = synth.spawn_frame(5, W, H)
    cam = _camera(W, H)
    sp = gs.SpawnParams(mode=gs.SPAWN_FIXED_K, k=3000, seed=3)
    dimg, ddep = torch.tensor(img, device="cuda"), torch.tensor(depth, device="cuda")
    theta = synth.mlp_init(9, last_scale=1.0)
    packed = gs.mlp_pack_bf16(torch.tensor(theta, device="cuda"))
    cap = 3100
    out = gs.Gaussians(*[torch.zeros(s, device="cuda") for s in ((3, cap), (3, cap), (4, cap), (cap,), (16, 3, cap))])
    n = gs.spawn_init(cam, dimg, ddep, out, offset=5, rendered=torch.tensor(ren, device="cuda"), sp=sp,
                      mlp_packed=packed)
    torch.cuda.synchronize()
    assert 0 < n <= 3000
    PL, PS = spawn.probability_f32(img, ren)
    pix = np.flatnonzero(spawn.mask_fixed_k(spawn.quantize(PS), 3000, spawn.splitmix64(3) >> 40))
    assert len(pix) == n
    R = np.eye(3)
    t = np.array([0.1, -0.2, 0.3], np.float32).astype(np.float64)
    f32 = lambda x: float(np.float32(x))
    rule = spawn.rule_attributes(pix, PL, img, depth, R, t, f32(cam.fx), f32(cam.fy), f32(cam.cx), f32(cam.cy),
                                 opacity=f32(0.1), min_prob=f32(1e-4))
    y = mlp.forward_bf16(theta.astype(np.float64), mlp.features(img, depth, pix))
    sl = slice(5, 5 + n)
    tol = 1e-2 * np.abs(y).max()
    assert np.abs(out.log_scales.cpu().numpy()[:, sl] - (rule["log_scales"] + y[:, :3].T)).max() < tol + 2e-5
    assert np.abs(out.opacity_logits.cpu().numpy()[sl] - (rule["opacity_logits"] + y[:, 3])).max() < tol + 1e-5
    dc = 2 * np.sqrt(np.pi)
    assert np.abs(out.sh.cpu().numpy()[0, :, sl] - (rule["sh0"] + dc * y[:, 4:].T)).max() < dc * tol + 2e-6
    assert np.abs(out.means.cpu().numpy()[:, sl] - rule["means"]).max() < 1e-4
    # without the network the same call gives the rule alone
    out2 = gs.Gaussians(*[torch.zeros_like(x) for x in out.tensors()])
    assert gs.spawn_init(cam, dimg, ddep, out2, offset=5, rendered=torch.tensor(ren, device="cuda"), sp=sp) == n
    assert np.abs(out2.log_scales.cpu().numpy()[:, sl] - rule["log_scales"]).max() < 2e-5


@pytest.mark.parametrize("batch", [1, 63, 64, 65, 1000])
def test_train_step_gradient(batch):
    gs = gpu()
    rng = np.random.default_rng(batch)
    theta = synth.mlp_init(11, last_scale=1.0)
    X = rng.standard_normal((batch, 196)).astype(np.float32)
    T = rng.standard_normal((batch, 7)).astype(np.float32)
    tr = gs.MlpTrainer(torch.tensor(theta, device="cuda"))
    grad = torch.empty(mlp.n_params(), device="cuda")
    loss = tr.step(torch.tensor(X, device="cuda"), torch.tensor(T, device="cuda"), lr=0.0, grad=grad)
    torch.cuda.synchronize()
    Y, cache = mlp.forward_f64(theta.astype(np.float64), X.astype(np.float64))
    L, dY = mlp.mse(Y, T)
    g_ref = mlp.backward_f64(theta.astype(np.float64), cache, dY)
    assert abs(loss.item() - L) <= 1e-5 * L
    g = grad.cpu().numpy()
    o = 0
    for part in mlp.unpack(np.arange(mlp.n_params())):  # per tensor: W1, b1, W2, b2, W3, b3
        sl = slice(o, o + part.size)
        _grad_close(g[sl], g_ref[sl])
        o += part.size
    assert np.array_equal(tr.theta.cpu().numpy(), theta)  # lr = 0 leaves the parameters


def test_train_adam_steps_match_oracle():
    gs = gpu()
    rng = np.random.default_rng(21)
    theta = synth.mlp_init(12, last_scale=1.0)
    X = rng.standard_normal((300, 196)).astype(np.float32)
    T = rng.standard_normal((300, 7)).astype(np.float32)
    tr = gs.MlpTrainer(torch.tensor(theta, device="cuda"), lr=1e-3)
    dX, dT = torch.tensor(X, device="cuda"), torch.tensor(T, device="cuda")
    th = theta.astype(np.float64)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    losses = []
    for step in range(1, 6):
        losses.append(tr.step(dX, dT).item())
        Y, cache = mlp.forward_f64(th, X.astype(np.float64))
        L, dY = mlp.mse(Y, T)
        assert abs(losses[-1] - L) <= 1e-5 * L
        th, m, v = mlp.adam(th, mlp.backward_f64(th, cache, dY), m, v, 1e-3, step)
    got = tr.theta.cpu().numpy().astype(np.float64)
    assert np.abs(got - th).max() < 2e-5  # 5 steps of at most lr = 1e-3 each
    assert losses[-1] < losses[0]
