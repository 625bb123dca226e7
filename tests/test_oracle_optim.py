"""Pins of the optimiser oracle: closed forms of the first Adam step, the
sparse mask, known loss values, the 6D map's orthonormality and fixed points,
and finite differences of its adjoint."""
import math

import numpy as np

from oracle import optim


def test_l1_known_values():
    img = np.array([0.5, 0.25, 1.0, 0.0])
    tgt = np.array([0.0, 0.25, 0.5, 1.0])
    s1, s2, g = optim.l1_loss(img, tgt, 0.5)
    assert s1 == 2.0 and s2 == 0.25 + 0.25 + 1.0
    assert g.tolist() == [0.5, 0.0, 0.5, -0.5]
    assert abs(optim.psnr(0.01) - 20.0) < 1e-12


def test_psnr_images_closed_forms():
    rng = np.random.default_rng(7)
    tgt = rng.random((3, 17, 23))
    # a constant offset c gives MSE = c^2 and PSNR = 20 log10(peak / |c|)
    for c, peak in ((0.1, 1.0), (-0.25, 1.0), (3.0, 255.0)):
        p, mse = optim.psnr_images(tgt + c, tgt, peak)
        assert abs(mse - c * c) <= 1e-12 * c * c
        assert abs(p - 20.0 * math.log10(peak / abs(c))) <= 1e-9
    # half the values off by 0.2, half exact: MSE = 0.02, PSNR = 10 log10(50)
    img = tgt.copy().ravel()
    img[::2] += 0.2
    p, mse = optim.psnr_images(img.reshape(tgt.shape), tgt)
    half = (tgt.size + 1) // 2
    assert abs(mse - 0.04 * half / tgt.size) <= 1e-15
    assert optim.psnr_images(tgt, tgt)[0] == np.inf


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(0)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    p1, m1, v1 = optim.adam(p, g, np.zeros(50), np.zeros(50), lr=0.1, step=1, eps=0.0)
    # bias-corrected first moments are g and g^2: the step is lr * sign(g)
    assert np.allclose(p1, p - 0.1 * np.sign(g), atol=1e-15)
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)


def test_adam_sparse_leaves_hidden_gaussians():
    rng = np.random.default_rng(1)
    n = 10
    p = rng.standard_normal((3, n))
    g = rng.standard_normal((3, n))
    m = rng.standard_normal((3, n)) * 0.1
    v = rng.random((3, n)) * 0.1
    vis = (np.arange(n) % 3 == 0).astype(np.int32)
    p1, m1, v1 = optim.adam(p, g, m, v, 0.01, 5, visible=vis, n_stride=n)
    pd, md, vd = optim.adam(p, g, m, v, 0.01, 5)
    hidden = vis == 0
    assert np.array_equal(p1[:, hidden], p[:, hidden]) and np.array_equal(m1[:, hidden], m[:, hidden])
    assert np.array_equal(p1[:, ~hidden], pd[:, ~hidden]) and np.array_equal(v1[:, ~hidden], vd[:, ~hidden])


def test_adam_per_gaussian_rate_first_step_closed_form():
    # the first bias-corrected step moves every element by its own rate
    # times sign(g): lr * s_j for the elements of Gaussian j
    rng = np.random.default_rng(4)
    n = 12
    p = rng.standard_normal((4, n))
    g = rng.standard_normal((4, n))
    s = rng.random(n) + 0.1
    p1, m1, v1 = optim.adam(p, g, np.zeros((4, n)), np.zeros((4, n)), lr=0.2, step=1, eps=0.0, n_stride=n,
                            lr_scale=s)
    assert np.allclose(p1, p - 0.2 * s[None, :] * np.sign(g), atol=1e-15)
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)
    # a hidden Gaussian keeps p, m, v whatever its rate
    vis = (np.arange(n) % 2).astype(np.int32)
    p2, m2, _ = optim.adam(p, g, np.zeros((4, n)), np.zeros((4, n)), 0.2, 1, eps=0.0, visible=vis, n_stride=n,
                           lr_scale=s)
    assert np.array_equal(p2[:, vis == 0], p[:, vis == 0]) and not m2[:, vis == 0].any()
    assert np.allclose(p2[:, vis == 1], (p - 0.2 * s[None, :] * np.sign(g))[:, vis == 1], atol=1e-15)


def test_lr_decay_counts_processed_steps():
    # after a schedule of sparse steps each factor is decay^(steps that saw it)
    rng = np.random.default_rng(5)
    n, steps, decay = 20, 9, 0.97
    s = np.ones(n)
    seen = np.zeros(n, int)
    for _ in range(steps):
        vis = (rng.random(n) < 0.6).astype(np.int32)
        s = optim.lr_decay(s, decay, vis)
        seen += vis
    assert np.allclose(s, decay ** seen, rtol=1e-14)
    assert np.allclose(optim.lr_decay(np.full(3, 2.0), 0.5), [1.0, 1.0, 1.0])


def test_pose_6d_orthonormal_and_identity():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((5, 9))
    P = optim.pose_from_6d(x)
    for i in range(5):
        R = P[i, :9].reshape(3, 3)
        assert np.allclose(R.T @ R, np.eye(3), atol=1e-14) and abs(np.linalg.det(R) - 1) < 1e-14
        # first column is a1's direction
        assert np.allclose(R[:, 0], x[i, :3] / np.linalg.norm(x[i, :3]))
    ident = optim.pose_from_6d(np.array([[2.0, 0, 0, 0.3, 5.0, 0, 1, 2, 3]]))
    assert np.allclose(ident[0, :9], np.eye(3).reshape(9)) and np.allclose(ident[0, 9:], [1, 2, 3])


def test_pose_6d_vjp_finite_differences():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 9))
    G = rng.standard_normal((2, 12))
    an = optim.pose_6d_vjp(x, G)
    h = 1e-6
    fd = np.zeros_like(x)
    for idx in np.ndindex(*x.shape):
        xp = x.copy()
        xp[idx] += h
        xm = x.copy()
        xm[idx] -= h
        fd[idx] = ((optim.pose_from_6d(xp) - optim.pose_from_6d(xm)) * G).sum() / (2 * h)
    assert np.abs(fd - an).max() < 1e-8 * max(1.0, np.abs(an).max())
    assert math.isfinite(an.sum())


def test_adam_constant_gradient_every_step_closed_form():
    # with a constant gradient from zero moments, m_k = (1 - b1^k) g and
    # v_k = (1 - b2^k) g^2, so the bias-corrected moments are g and g^2 at
    # every step k and each step moves by lr * sign(g): this pins the bias
    # correction at steps 2, 3, ..., not only at the first
    rng = np.random.default_rng(7)
    n = 9
    p0 = rng.standard_normal((2, n))
    g = rng.standard_normal((2, n))
    s = rng.random(n) + 0.5
    p, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    for k in range(1, 8):
        p, m, v = optim.adam(p, g, m, v, lr=0.03, step=k, eps=0.0, n_stride=n, lr_scale=s)
        assert np.allclose(p, p0 - 0.03 * k * s[None, :] * np.sign(g), rtol=0, atol=1e-13)
        assert np.allclose(m, (1 - 0.9 ** k) * g, rtol=0, atol=1e-15)
        assert np.allclose(v, (1 - 0.999 ** k) * g * g, rtol=0, atol=1e-15)


def test_adam_matches_torch_optim_adam_over_steps():
    # library routine: torch.optim.Adam (CPU, float64, the same bias-corrected
    # update p -= lr m_hat / (sqrt(v_hat) + eps)) over seven steps with
    # changing gradients; the sparse form on a visible set equals it there
    import torch
    rng = np.random.default_rng(8)
    n = 40
    p0 = rng.standard_normal((3, n))
    grads = [rng.standard_normal((3, n)) * (1 + k) for k in range(7)]
    pt = torch.tensor(p0, requires_grad=True)
    opt = torch.optim.Adam([pt], lr=0.01, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    vis = np.ones(n, np.int32)
    for k, gk in enumerate(grads, start=1):
        opt.zero_grad()
        pt.grad = torch.tensor(gk)
        opt.step()
        p, m, v = optim.adam(p, gk, m, v, lr=0.01, step=k, eps=1e-8, visible=vis, n_stride=n)
        assert np.allclose(p, pt.detach().numpy(), rtol=0, atol=1e-14)
    st = opt.state[pt]
    # torch forms the moments by lerp (m + (1 - b1)(g - m)): equal up to FP64 rounding
    assert np.allclose(m, st["exp_avg"].numpy(), rtol=1e-12, atol=1e-15)
    assert np.allclose(v, st["exp_avg_sq"].numpy(), rtol=1e-12, atol=1e-15)
