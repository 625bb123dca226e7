"""Oracle of the learned spawn-init network (test infrastructure only).

The network predicts, for a spawned primitive, corrections to the paper's
direct sampling rule (section 4.2): from the 7x7 RGB patch around the pixel
(channel-last, row-major) and the 7x7 depth patch as log(D / D_centre),
196 inputs -> 64 GELU -> 64 GELU -> 7 outputs: three log-scale offsets, an
opacity-logit offset and three colour offsets, added to the rule's values.

* `forward_f64` / `backward_f64` -- the definition in float64 (exact erf GELU).
* `forward_bf16` -- the same with inputs, weights and the activations fed to
  each layer rounded to bfloat16 (round to nearest, ties to even) and the
  products accumulated in float64: the precision of BF16 matrix cores with
  FP32 accumulation, within FP32 rounding.
* `mse` and `adam` for the training step.
Weights are (W1 [64][196], b1 [64], W2 [64][64], b2 [64], W3 [7][64], b3 [7]),
the layout of a row-major matrix times a column vector.
"""
from __future__ import annotations

import math

import numpy as np

DIMS = (196, 64, 64, 7)
PATCH = 7


def n_params():
    return sum(DIMS[i + 1] * DIMS[i] + DIMS[i + 1] for i in range(3))


def unpack(theta):
    theta = np.asarray(theta)
    out, o = [], 0
    for i in range(3):
        m, k = DIMS[i + 1], DIMS[i]
        out.append(theta[o:o + m * k].reshape(m, k))
        o += m * k
        out.append(theta[o:o + m])
        o += m
    return out


def gelu(x):
    x = np.asarray(x, np.float64)
    return 0.5 * x * (1.0 + np.vectorize(math.erf)(x / math.sqrt(2.0)))


def gelu_grad(x):
    x = np.asarray(x, np.float64)
    cdf = 0.5 * (1.0 + np.vectorize(math.erf)(x / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)
    return cdf + x * pdf


def forward_f64(theta, X):
    """X [B][196] -> (Y [B][7], cache)."""
    W1, b1, W2, b2, W3, b3 = (np.asarray(a, np.float64) for a in unpack(theta))
    X = np.asarray(X, np.float64)
    z1 = X @ W1.T + b1
    h1 = gelu(z1)
    z2 = h1 @ W2.T + b2
    h2 = gelu(z2)
    Y = h2 @ W3.T + b3
    return Y, (X, z1, h1, z2, h2)


def backward_f64(theta, cache, dY):
    """Gradient of sum(dY * Y) with respect to the packed parameters."""
    W1, b1, W2, b2, W3, b3 = (np.asarray(a, np.float64) for a in unpack(theta))
    X, z1, h1, z2, h2 = cache
    dY = np.asarray(dY, np.float64)
    gW3 = dY.T @ h2
    gb3 = dY.sum(0)
    dz2 = (dY @ W3) * gelu_grad(z2)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(0)
    dz1 = (dz2 @ W2) * gelu_grad(z1)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])


def bf16_round(x):
    """Round float64/float32 values to the nearest bfloat16 (ties to even), as float64."""
    f = np.asarray(x, np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    rounded = ((bits + 0x7FFF + lsb) >> 16) << 16
    return rounded.astype(np.uint32).view(np.float32).astype(np.float64)


def forward_bf16(theta, X):
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    f32 = lambda a: np.asarray(a, np.float32).astype(np.float64)
    z1 = bf16_round(X) @ bf16_round(W1).T + f32(b1)
    h1 = gelu(z1)
    z2 = bf16_round(h1) @ bf16_round(W2).T + f32(b2)
    h2 = gelu(z2)
    return bf16_round(h2) @ bf16_round(W3).T + f32(b3)


def mse(Y, T):
    """Mean over samples and outputs of (Y - T)^2, and its gradient."""
    D = np.asarray(Y, np.float64) - np.asarray(T, np.float64)
    return float((D * D).mean()), 2.0 * D / D.size


def adam(theta, g, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-8):
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def features(img, depth, pixels):
    """The 196 inputs of each pixel: 7x7 RGB (channel-last, row-major) with
    replicated borders, then the 7x7 log(D / D_centre)."""
    img = np.asarray(img, np.float64)
    depth = np.asarray(depth, np.float64)
    H, W = depth.shape
    r = PATCH // 2
    out = np.zeros((len(pixels), 196))
    for n, p in enumerate(pixels):
        v, u = divmod(int(p), W)
        ys = np.clip(np.arange(v - r, v + r + 1), 0, H - 1)
        xs = np.clip(np.arange(u - r, u + r + 1), 0, W - 1)
        rgb = img[:, ys][:, :, xs]  # [3][7][7]
        out[n, :147] = rgb.transpose(1, 2, 0).reshape(-1)
        out[n, 147:] = np.log(depth[ys][:, xs] / depth[v, u]).reshape(-1)
    return out
