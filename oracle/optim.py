"""FP64 oracle of the joint-optimisation helpers (test infrastructure only).

* L1 photometric loss: sum |I - I*|, sum (I - I*)^2, gradient c sign(I - I*).
* Adam (bias-corrected) and its sparse form, which leaves every parameter of
  a Gaussian the step did not process untouched (section 4.3 uses the
  sparse Adam of the fast 3DGS optimiser).
* Per-Gaussian learning rates (section 4.3 and the joint-optimisation
  appendix): each Gaussian's rate starts at a fixed value when it is
  introduced and is multiplied by a decay ratio every time a sparse Adam
  step processes it, so the factor of a Gaussian is decay^k after k steps
  that saw it.
* The continuous 6D rotation representation of the camera poses
  (section 4.3): R's columns by Gram-Schmidt of the two 3-vectors; its
  adjoint is taken with PyTorch CPU autograd in float64.
"""
from __future__ import annotations

import numpy as np


def l1_loss(image, target, grad_scale):
    d = np.asarray(image, np.float64) - np.asarray(target, np.float64)
    return np.abs(d).sum(), (d * d).sum(), grad_scale * np.sign(d)


def psnr(mse):
    return 10.0 * np.log10(1.0 / mse)


def psnr_images(image, target, peak=1.0):
    """(PSNR in dB, MSE) of an image against its target: 10 log10(peak^2 /
    MSE), +inf for equal images (the novel-view metric of section 5)."""
    d = np.asarray(image, np.float64) - np.asarray(target, np.float64)
    mse = (d * d).sum() / d.size
    return (10.0 * np.log10(peak * peak / mse) if mse > 0 else np.inf), mse


def adam(p, g, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-15, visible=None, n_stride=None, lr_scale=None):
    """One Adam step; lr_scale [n_stride] multiplies the rate of element e
    by lr_scale[e % n_stride] (the per-Gaussian rate)."""
    p, g, m, v = (np.array(a, np.float64) for a in (p, g, m, v))
    m_new = beta1 * m + (1 - beta1) * g
    v_new = beta2 * v + (1 - beta2) * g * g
    mh = m_new / (1 - beta1 ** step)
    vh = v_new / (1 - beta2 ** step)
    rate = lr
    if lr_scale is not None:
        flat = np.arange(p.size) % n_stride
        rate = lr * np.asarray(lr_scale, np.float64).reshape(-1)[flat].reshape(p.shape)
    p_new = p - rate * mh / (np.sqrt(vh) + eps)
    if visible is not None:
        flat = np.arange(p.size) % n_stride
        keep = np.asarray(visible).reshape(-1)[flat].reshape(p.shape) != 0
        p_new = np.where(keep, p_new, p)
        m_new = np.where(keep, m_new, m)
        v_new = np.where(keep, v_new, v)
    return p_new, m_new, v_new


def lr_decay(lr_scale, decay, visible=None):
    """The per-Gaussian rates after one sparse step: the Gaussians it
    processed (visible != 0, or all without a mask) are multiplied by decay."""
    s = np.array(lr_scale, np.float64)
    if visible is None:
        return s * decay
    return np.where(np.asarray(visible) != 0, s * decay, s)


def pose_from_6d(x):
    """x (V, 9) = (a1, a2, t) -> pose (V, 12) = (R row-major, t)."""
    x = np.asarray(x, np.float64)
    out = np.zeros((x.shape[0], 12))
    for i, xi in enumerate(x):
        a1, a2 = xi[:3], xi[3:6]
        b1 = a1 / np.linalg.norm(a1)
        u2 = a2 - (b1 @ a2) * b1
        b2 = u2 / np.linalg.norm(u2)
        b3 = np.cross(b1, b2)
        out[i, :9] = np.stack([b1, b2, b3], axis=1).reshape(9)
        out[i, 9:] = xi[6:]
    return out


def pose_6d_vjp(x, d_pose):
    import torch
    xt = torch.tensor(np.asarray(x, np.float64), requires_grad=True)
    a1, a2 = xt[:, 0:3], xt[:, 3:6]
    b1 = a1 / a1.norm(dim=1, keepdim=True)
    u2 = a2 - (b1 * a2).sum(1, keepdim=True) * b1
    b2 = u2 / u2.norm(dim=1, keepdim=True)
    b3 = torch.cross(b1, b2, dim=1)
    R = torch.stack([b1, b2, b3], dim=2).reshape(-1, 9)
    pose = torch.cat([R, xt[:, 6:]], dim=1)
    pose.backward(torch.tensor(np.asarray(d_pose, np.float64)))
    return xt.grad.numpy()
