"""Pins of the spawn and spawn-network oracles.

Spawn (section 4.2): LoG taps sum to zero and match the analytic Laplacian
of a Gaussian; a constant image gives zero response; a step edge gives two
equal-magnitude peaks on either side with a sign change between them (the
paper's LoG step-response figure); rendering equal to the input gives
P_s = 0 everywhere; the first frame gives P_s = P_L; the FP32 reference is
within FP32 rounding of the FP64 definition; the scale rule's closed form;
the mean nearest-neighbour distance of a 2D Poisson process is 1/(2 sqrt(l))
(Monte Carlo, independent of the formula); unprojected means project back to
their pixel and depth; SplitMix64 against its published first output;
systematic sampling draws exactly K thresholds and never selects an empty
pixel; Bernoulli draws are uniform.
Network: GELU known values; finite differences of the float64 backward;
torch float64 autograd on the same weights; bf16 rounding known values.
"""
import math

import numpy as np
import pytest

from oracle import mlp, spawn


def test_log_kernel():
    k = spawn.log_kernel_f64(1.0)
    assert k.shape == (9, 9)
    assert abs(k.sum()) < 1e-15
    # analytic LoG (before the zero-sum shift) at the centre is -1/(pi sigma^4)
    raw_centre = -2.0 / (2 * math.pi)
    shift = k[4, 4] - raw_centre
    assert abs(k[0, 4] - shift - (16 - 2) * math.exp(-8) / (2 * math.pi)) < 1e-15


def test_log_step_edge_two_peaks():
    W = 40
    img = np.zeros((3, 8, W))
    img[:, :, W // 2:] = 1.0
    L = spawn.log_response_f64(img)[0, 4]
    left, right = L[W // 2 - 1], L[W // 2]
    assert left > 0 > right  # sign change across the edge
    assert abs(abs(left) - abs(right)) < 1e-12  # equal magnitude on either side
    # mirror symmetry about the edge, peaks within 2 px of it (the continuous peak is sigma away)
    for k in range(W // 2):
        assert abs(abs(L[W // 2 - 1 - k]) - abs(L[W // 2 + k])) < 1e-12
    assert W // 2 - 1 - np.argmax(np.abs(L[: W // 2])) <= 1
    PL, _, _ = spawn.prob_f64(img)
    assert PL.max() <= 1.0 and PL[4, 2] == 0.0


def test_constant_and_penalty_properties():
    rng = np.random.default_rng(0)
    img = rng.random((3, 24, 30))
    assert np.abs(spawn.log_response_f64(np.full((3, 10, 10), 0.7))).max() < 1e-14
    PL, Pt, Ps = spawn.prob_f64(img, img)
    assert np.abs(Ps).max() == 0.0
    PL, Pt, Ps = spawn.prob_f64(img)
    assert (Pt == 0).all() and np.array_equal(Ps, PL)
    assert ((PL >= 0) & (PL <= 1)).all()
    # the binary32 reference is the same quantity within FP32 rounding
    PL32, Ps32 = spawn.probability_f32(img, img * 0.5)
    PLd, _, Psd = spawn.prob_f64(img, img * 0.5)
    assert np.abs(PL32 - PLd).max() < 1e-5 and np.abs(Ps32 - Psd).max() < 1e-5


def test_clark_evans_mean_nn_distance():
    """Mean nearest-neighbour distance of a Poisson process of intensity l is
    1/(2 sqrt(l)): simulate on a torus."""
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(1)
    L = 200.0
    for lam in (0.05, 0.3):
        n = rng.poisson(lam * L * L)
        pts = rng.uniform(0, L, (n, 2))
        tree = cKDTree(pts, boxsize=L)
        d, _ = tree.query(pts, k=2)
        assert abs(d[:, 1].mean() - 1.0 / (2 * math.sqrt(lam))) < 0.02 / math.sqrt(lam)


def test_rule_attributes_geometry():
    rng = np.random.default_rng(2)
    H, W = 12, 16
    img = rng.random((3, H, W))
    depth = rng.uniform(2, 5, (H, W))
    PL = rng.uniform(0.01, 1, (H, W))
    R = np.linalg.qr(rng.standard_normal((3, 3)))[0]
    R *= np.sign(np.linalg.det(R))
    t = rng.standard_normal(3)
    fx, fy, cx, cy = 20.0, 22.0, 8.3, 5.7
    pix = np.array([0, 5, 77, H * W - 1])
    a = spawn.rule_attributes(pix, PL, img, depth, R, t, fx, fy, cx, cy)
    p = R @ a["means"] + t[:, None]
    v, u = pix // W, pix % W
    assert np.allclose(p[2], depth.reshape(-1)[pix])
    assert np.allclose(fx * p[0] / p[2] + cx, u) and np.allclose(fy * p[1] / p[2] + cy, v)
    s = np.exp(a["log_scales"])
    assert np.allclose(s, depth.reshape(-1)[pix] / (2 * math.sqrt(fx * fy) * np.sqrt(PL.reshape(-1)[pix])))
    assert np.allclose(0.5 + a["sh0"] / (2 * math.sqrt(math.pi)), img.reshape(3, -1)[:, pix])
    from oracle import raster
    assert np.allclose(raster.quat_to_rot(a["quats"][:, 0]), R.T)


def test_splitmix64_published_value():
    # first output of SplitMix64 started from state 0
    assert spawn.splitmix64(0) == 0xE220A8397B1DCDAF


def test_uniform_draws_are_uniform():
    u = spawn.uniform24(12345, 20000)
    # the array form is the scalar generator, including the wrap of seed + p past 2^64
    for p in (0, 1, 777, 19999):
        assert u[p] == spawn.splitmix64(12345 + p) >> 40
    w = spawn.uniform24((1 << 64) - 2, 5)
    assert [int(x) for x in w] == [spawn.splitmix64(((1 << 64) - 2 + p) % (1 << 64)) >> 40 for p in range(5)]
    assert u.min() >= 0 and u.max() < (1 << 24)
    hist = np.bincount(u >> 20, minlength=16)
    assert (np.abs(hist - 1250) < 200).all()


def test_fixed_k_sampling():
    rng = np.random.default_rng(3)
    q = rng.integers(0, 1 << 24, 500)
    q[rng.random(500) < 0.4] = 0
    for k, off in [(50, 0), (50, 12345), (137, (1 << 24) - 1), (2000, 5)]:
        sel = spawn.mask_fixed_k(q, k, off)
        # independent count per pixel: thresholds t_j in [a, a + q) <=> j in [ceil((aK-U)/S), ceil((bK-U)/S))
        S = int(q.sum())
        U = (S >> 24) * off + (((S & 0xFFFFFF) * off) >> 24)
        a = np.concatenate([[0], np.cumsum(q)[:-1]])
        cnt = []
        for ai, qi in zip(a.tolist(), q.tolist()):
            lo = -((U - ai * k) // S)  # ceil((a K - U) / S)
            hi = -((U - (ai + qi) * k) // S)
            cnt.append(max(0, min(k, hi) - max(0, lo)))
        cnt = np.array(cnt)
        assert cnt.sum() == k  # exactly K thresholds
        assert np.array_equal(sel, cnt > 0)  # duplicates collapse to one spawn
        assert not (sel & (q == 0)).any()
    # masses far above S/K give exactly one spawn per selected heavy pixel
    q2 = np.zeros(100, np.int64)
    q2[[3, 40, 77]] = 1 << 24
    assert np.array_equal(np.nonzero(spawn.mask_fixed_k(q2, 3, 7))[0], [3, 40, 77])


def test_bernoulli_rate():
    q = np.full(40000, 1 << 22)  # probability 1/4
    m = spawn.mask_bernoulli(q, 99)
    assert abs(m.mean() - 0.25) < 0.01


# ----------------------------------------------------------------- network
def test_gelu_known_values():
    assert mlp.gelu(0.0) == 0.0
    assert abs(mlp.gelu(1.0) - 0.8413447460685429) < 1e-15
    assert abs(mlp.gelu(-1.0) + 0.15865525393145707) < 1e-15


def test_mlp_backward_finite_differences():
    rng = np.random.default_rng(4)
    theta = rng.standard_normal(mlp.n_params()) * 0.1
    X = rng.standard_normal((5, 196))
    dY = rng.standard_normal((5, 7))
    Y, cache = mlp.forward_f64(theta, X)
    g = mlp.backward_f64(theta, cache, dY)
    h = 1e-6
    for idx in rng.choice(theta.size, 40, replace=False):
        tp = theta.copy()
        tp[idx] += h
        tm = theta.copy()
        tm[idx] -= h
        fd = ((mlp.forward_f64(tp, X)[0] - mlp.forward_f64(tm, X)[0]) * dY).sum() / (2 * h)
        assert abs(fd - g[idx]) < 1e-7 * max(1.0, abs(g[idx]))


def test_mlp_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    theta = rng.standard_normal(mlp.n_params()) * 0.1
    X = rng.standard_normal((6, 196))
    T = rng.standard_normal((6, 7))
    W1, b1, W2, b2, W3, b3 = [torch.tensor(a, requires_grad=True) for a in mlp.unpack(theta)]
    x = torch.tensor(X)
    y = torch.nn.functional.gelu(torch.nn.functional.gelu(x @ W1.T + b1) @ W2.T + b2) @ W3.T + b3
    loss = ((y - torch.tensor(T)) ** 2).mean()
    loss.backward()
    Y, cache = mlp.forward_f64(theta, X)
    L, dY = mlp.mse(Y, T)
    g = mlp.backward_f64(theta, cache, dY)
    ref = np.concatenate([a.grad.numpy().ravel() for a in (W1, b1, W2, b2, W3, b3)])
    assert abs(L - loss.item()) < 1e-12 and np.abs(g - ref).max() < 1e-12


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -7, -2.5, 3.14159265])
    out = mlp.bf16_round(vals)
    assert out[0] == 1.0 and out[1] == 1.0  # tie to even (down)
    assert out[2] == 1.0 + 2 ** -6  # tie to even (up)
    assert out[3] == 1.0 + 2 ** -7 and out[4] == -2.5
    assert abs(out[5] - 3.140625) < 1e-12


def test_features_layout():
    rng = np.random.default_rng(6)
    img = rng.random((3, 10, 12))
    depth = rng.uniform(1, 2, (10, 12))
    f = mlp.features(img, depth, [5 * 12 + 6, 0])
    # centre of the RGB patch is the pixel's colour, channel-last
    assert np.allclose(f[0, (3 * 7 + 3) * 3:(3 * 7 + 3) * 3 + 3], img[:, 5, 6])
    assert f[0, 147 + 24] == 0.0 and f[1, 147 + 24] == 0.0  # log(D / D_centre) at the centre
    # corner pixel: replicated border
    assert np.allclose(f[1, :3], img[:, 0, 0])


def test_mlp_adam_constant_gradient_and_torch():
    # the network's Adam: a constant gradient moves every weight by lr sign(g)
    # per step from zero moments (bias correction at every step; eps = 0),
    # and changing gradients follow torch.optim.Adam (float64) step by step
    import torch
    rng = np.random.default_rng(3)
    th0 = rng.standard_normal(mlp.n_params())
    g = rng.standard_normal(th0.size)
    th, m, v = th0.copy(), np.zeros_like(th0), np.zeros_like(th0)
    for k in range(1, 6):
        th, m, v = mlp.adam(th, g, m, v, lr=1e-3, step=k, eps=0.0)
        assert np.allclose(th, th0 - 1e-3 * k * np.sign(g), rtol=0, atol=1e-13)
    pt = torch.tensor(th0, requires_grad=True)
    opt = torch.optim.Adam([pt], lr=2e-3, betas=(0.9, 0.999), eps=1e-8)
    th, m, v = th0.copy(), np.zeros_like(th0), np.zeros_like(th0)
    for k in range(1, 6):
        gk = rng.standard_normal(th0.size) * 10 ** (k - 3)
        opt.zero_grad()
        pt.grad = torch.tensor(gk)
        opt.step()
        th, m, v = mlp.adam(th, gk, m, v, lr=2e-3, step=k)
        assert np.allclose(th, pt.detach().numpy(), rtol=0, atol=1e-14)


def _exact_net(rng):
    """A network whose every product, sum and activation is exact in
    bfloat16 and float64: inputs in {0, 1} with input 0 always 1, first-layer
    weights in {0, 16} with a 16 on input 0, then 0/1 weights with a 1 on the
    first unit, zero biases.  Every pre-activation is then a multiple of 16 in
    [16, 4096] (at most 8 significant bits), and GELU(z) = z exactly for
    z >= 16 (1 - Phi(16) is far below half an ulp of 1)."""
    X = rng.integers(0, 2, (5, 196)).astype(np.float64)
    X[:, 0] = 1.0
    W1 = rng.choice([0.0, 0.0, 16.0], (64, 196))
    W1[:, 0] = 16.0
    W2 = (rng.random((64, 64)) < 1.0 / 64).astype(np.float64)
    W2[:, 0] = 1.0
    W3 = (rng.random((7, 64)) < 0.05).astype(np.float64)
    W3[:, 1] = 1.0
    z = lambda k: np.zeros(k)
    return (W1, W2, W3), X, lambda W1_: np.concatenate([W1_.ravel(), z(64), W2.ravel(), z(64), W3.ravel(), z(7)])


def test_bf16_forward_exact_network_and_rounding_points():
    # with bfloat16-exact inputs, weights and activations the BF16 forward
    # equals the float64 definition exactly; a weight of 1 + 2^-9 (halfway
    # between two bfloat16 values, ties to even -> 1) is rounded before the
    # product, and a hidden activation that needs more than 8 significant
    # bits is rounded before the next layer
    rng = np.random.default_rng(11)
    (W1, W2, W3), X, pack = _exact_net(rng)
    Y64, cache = mlp.forward_f64(pack(W1), X)
    assert (cache[1] >= 16).all()
    assert np.array_equal(mlp.forward_bf16(pack(W1), X), Y64)
    Wh = W1.copy()
    Wh[:, 1] = 1.0 + 2.0 ** -9  # rounds to 1 in bfloat16
    Wr = W1.copy()
    Wr[:, 1] = 1.0
    Xw = X.copy()
    Xw[:, 1] = 15.0  # z1 = 16 k + 15 w: with w = 1, 31 + 16 (k - 1) needs up to 12 bits
    Y_exact, _ = mlp.forward_f64(pack(Wh), Xw)
    Y_round, _ = mlp.forward_f64(pack(Wr), Xw)
    assert not np.array_equal(Y_exact, Y_round)
    h1 = mlp.bf16_round(Xw @ Wr.T)  # GELU(z) = z here; then the activation is rounded
    h2 = mlp.bf16_round(h1 @ W2.T)
    assert not np.array_equal(h1, Xw @ Wr.T)
    assert np.array_equal(mlp.forward_bf16(pack(Wh), Xw), h2 @ W3.T)
