"""Shared helpers of the GPU parity tests: move a synthetic scene to the
device, run the HIP path through the C ABI, and run the oracle on the same
inputs.  No expected value comes from the HIP path."""
from __future__ import annotations

import numpy as np
import torch

from oracle import raster as orc


def gpu():
    from paper_2506_05558_amd import gsmi
    return gsmi


def gpu_camera(view, bg=(0.0, 0.0, 0.0)):
    gs = gpu()
    pose = np.concatenate([np.asarray(view.R, np.float32).reshape(9), np.asarray(view.t, np.float32)])
    return gs.Camera(view.width, view.height, float(view.fx), float(view.fy), float(view.cx), float(view.cy),
                     torch.tensor(pose, dtype=torch.float32, device="cuda"), 0.2, tuple(bg))


def gpu_gauss(scene):
    return gpu().Gaussians.from_arrays(scene.arrays())


def oracle_inputs(view, scene, bg=(0.0, 0.0, 0.0)):
    return orc.Camera.from_view(view, bg=bg), orc.Gaussians.from_scene(scene)


def run_forward(cam, g, capacity=0, count_pairs=False):
    gs = gpu()
    proj = gs.project(cam, g)
    sorter = gs.BinSorter(capacity)
    binned = sorter(cam, proj)
    frame = gs.render_fwd(cam, proj, binned, count_pairs=count_pairs)
    torch.cuda.synchronize()
    return proj, binned, frame


def flagged_upstream(shape_hw, flags, seed, depth_scale=0.1, alpha_scale=1.0):
    """Random upstream gradients, zero at the oracle's near-decision pixels so
    that a threshold flip there cannot change any gradient."""
    rng = np.random.default_rng(seed)
    H, W = shape_hw
    keep = (flags == 0).astype(np.float64)
    gi = rng.standard_normal((3, H, W)) * keep[None]
    gd = rng.standard_normal((H, W)) * keep * depth_scale
    ga = rng.standard_normal((H, W)) * keep * alpha_scale
    return gi.astype(np.float32), gd.astype(np.float32), ga.astype(np.float32)


def embed(crop_arr, full_hw, crop):
    x0, y0, cw, ch = crop
    H, W = full_hw
    if crop_arr.ndim == 3:
        out = np.zeros((crop_arr.shape[0], H, W), crop_arr.dtype)
        out[:, y0:y0 + ch, x0:x0 + cw] = crop_arr
    else:
        out = np.zeros((H, W), crop_arr.dtype)
        out[y0:y0 + ch, x0:x0 + cw] = crop_arr
    return out


def rel_err(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def assert_grad_close(name, got, ref, rel=1e-3):
    got = np.asarray(got, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    e = rel_err(got, ref)
    assert e <= rel, f"{name}: relative L2 error {e:.3e} > {rel}"
    scale = np.abs(ref).max() if ref.size else 0.0
    bad = np.abs(got - ref) > rel * (np.abs(ref) + 1e-3 * scale) + 1e-12
    worst = np.max(np.abs(got - ref) / (np.abs(ref) + 1e-3 * scale + 1e-30)) if ref.size else 0.0
    print(f"{name}: rel L2 {e:.2e}, worst scaled element error {worst:.2e}, {bad.sum()} of {bad.size} outside")
    assert bad.sum() == 0, f"{name}: {bad.sum()} of {bad.size} elements outside tolerance"
