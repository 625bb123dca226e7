#!/usr/bin/env python3
"""Benchmark: joint pose + Gaussian optimisation step (section 4.3) on one GPU.

Workload (synthetic stand-in for the paper's 1200-1600 px views with 1-2M
primitives): a window of 8 keyframes at 1920x1080 on a smooth random
trajectory, 2M Gaussians (250k seeded from each keyframe) with SH degree 3
in FP32.  Targets are rendered once from the seeded ground-truth scene; the
optimised model starts from the ground truth perturbed, with the poses of
keyframes 1..7 perturbed by N(0, 0.01) twists (keyframe 0 is held fixed).

One step = for each of the 8 views: 6D pose -> R (once for all views),
project, bin + sort, render forward, L1 loss and its gradient, render
backward (Gaussian and pose gradients); then the 6D pose adjoint and one
sparse Adam update of all Gaussian parameters and the poses.  Every step
runs in libgsmi's HIP kernels; inputs are resident in HBM.

Metric: fwd+bwd megapixels per second over the whole step (8 x 1920 x 1080
pixels per step / step time).  Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

W_IMG, H_IMG, N_VIEWS, PER_VIEW, SH_DEG, SEED = 1920, 1080, 8, 250_000, 3, 2506

# MI355X peaks (published): HBM3E 8 TB/s; FP32 vector 157.3 TFLOP/s with
# packed FP32, which this build does not emit: unpacked VALU issue is
# 256 CU x 64 lanes x 2.4 GHz = 39.3 T lane-ops/s.
PEAK_HBM_GBS = 8000.0
PEAK_VALU_TOPS = 256 * 64 * 2.4e9 / 1e12

# Algorithmic work (lane-operations) per (pixel, Gaussian) pair, from the
# definition.  Only pairs inside the Gaussian's support (alpha >= alpha_min)
# are work every correct implementation must do; pairs a tile list adds
# outside the support are acceleration overhead and are not counted.
#  forward, per support pair up to the stop: dx, dy, 5 ops for the quadratic
#  form, exp, opacity scale, clamp, threshold test = 11; a composited pair
#  adds 1 - alpha, T (1 - alpha), cutoff test, w = alpha T, 3 colour and
#  1 depth accumulations = 8.
#  backward, per composited pair: the same 11 to recompute alpha, plus the
#  adjoint 55 (prefix sums 4, suffix 4, 1/(1-alpha) 2, d alpha 17,
#  colour/depth grads 4, opacity/conic/mean grads 21, T update 2, w 1).
FWD_PAIR, FWD_COMP, BWD_COMP = 11, 8, 66


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-crops", type=int, default=12)
    ap.add_argument("--copy-probe", action="store_true",
                    help="end with one plain 256 MiB device copy, the reference for HBM byte counters")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "one GPU only: sharding the step across GPUs is not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2506_05558_amd import gsmi, synth

    torch.cuda.set_device(0)
    dev = "cuda"
    t0 = time.time()
    views = synth.trajectory(SEED, N_VIEWS, W_IMG, H_IMG)
    gt_scene = synth.window_scene(SEED, views, PER_VIEW, SH_DEG)
    start = synth.perturb_scene(SEED, gt_scene)
    n = gt_scene.n
    print(f"# scene generated in {time.time() - t0:.1f}s: {n} Gaussians", file=sys.stderr, flush=True)

    params = gsmi.Params()
    sorter = gsmi.BinSorter(capacity=12 * PER_VIEW * N_VIEWS)
    H, W = H_IMG, W_IMG

    # ---- targets from the ground truth
    gt = gsmi.Gaussians.from_arrays(gt_scene.arrays())
    targets = []
    for v in views:
        pose = torch.tensor(np.concatenate([v.R.reshape(9), v.t]).astype(np.float32), device=dev)
        cam = gsmi.Camera(W, H, v.fx, v.fy, v.cx, v.cy, pose)
        pr = gsmi.project(cam, gt, params)
        b = sorter(cam, pr)
        targets.append(gsmi.render_fwd(cam, pr, b, params).image.clone())
    del gt, pr, b
    torch.cuda.synchronize()

    # ---- optimised state
    g = gsmi.Gaussians.from_arrays(start.arrays())
    grads = g.zeros_like()
    m1 = g.zeros_like()
    m2 = g.zeros_like()
    rng = np.random.default_rng(SEED)
    x6 = np.zeros((N_VIEWS, 9), np.float32)
    for i, v in enumerate(views):
        R, t = (v.R, v.t) if i == 0 else synth.perturb_pose(rng, v.R, v.t, 0.01)
        x6[i] = np.concatenate([R[:, 0], R[:, 1], t])
    x6 = torch.tensor(x6, device=dev)
    dx6 = torch.zeros_like(x6)
    px_m, px_v = torch.zeros_like(x6), torch.zeros_like(x6)
    poses = torch.zeros((N_VIEWS, 12), dtype=torch.float32, device=dev)
    d_pose = torch.zeros((N_VIEWS, 12), dtype=torch.float64, device=dev)
    visible = torch.zeros(n, dtype=torch.int32, device=dev)
    sums = torch.zeros((N_VIEWS, 2), dtype=torch.float64, device=dev)
    proj = gsmi.alloc_projected(n, dev)
    f = lambda *s, dt=torch.float32: torch.empty(s, dtype=dt, device=dev)
    frame = gsmi.Frame(f(3, H, W), f(H, W), f(H, W), f(H, W), f(H, W, dt=torch.int32))
    g_img = f(3, H, W)
    bwd_ws = torch.empty(gsmi.render_bwd_workspace(n, sorter.capacity), dtype=torch.uint8, device=dev)
    loss_ws = torch.empty(1 << 16, dtype=torch.uint8, device=dev)
    cams = [gsmi.Camera(W, H, v.fx, v.fy, v.cx, v.cy, poses[i]) for i, v in enumerate(views)]
    lr = dict(means=1.6e-4 * 10, log_scales=5e-3, quats=1e-3, opacity_logits=5e-2, sh_dc=2.5e-3, sh_rest=1.25e-4,
              pose=1e-4)
    state = dict(step=0)
    pairs = []

    def step(count_pairs=False):
        state["step"] += 1
        k = state["step"]
        for t in grads.tensors():
            gsmi.zero_(t)
        gsmi.zero_(d_pose)
        gsmi.zero_(dx6)
        gsmi.zero_(visible)
        gsmi.pose_from_6d(x6, poses)
        for i, cam in enumerate(cams):
            gsmi.project(cam, g, params, out=proj)
            b = sorter(cam, proj)
            fr = frame
            if count_pairs:
                fr = gsmi.Frame(frame.image, frame.depth, frame.alpha, frame.final_t, frame.n_contrib,
                                torch.empty((4, H, W), dtype=torch.int32, device=dev))
            gsmi.render_fwd(cam, proj, b, params, out=fr)
            gsmi.loss_l1(fr.image, targets[i], 1.0 / (3 * H * W * N_VIEWS), g_img, sums[i], loss_ws)
            gsmi.render_bwd(cam, g, proj, b, fr, g_img, grads=grads, dL_dpose=d_pose[i], params=params, ws=bwd_ws)
            gsmi.mark_visible(proj, visible)
            if count_pairs:
                st = fr.stats.view(4, -1).to(torch.int64).sum(1).cpu().numpy()
                pairs.append((int(st[0]), int(st[1]), int(st[2]), int(st[3]),
                              int(fr.n_contrib.to(torch.int64).sum()), b.n_instances))
        gsmi.pose_6d_bwd(x6, d_pose, dx6)
        for name in ["means", "log_scales", "quats", "opacity_logits"]:
            gsmi.adam_step(getattr(g, name), getattr(grads, name), getattr(m1, name), getattr(m2, name), lr[name],
                           k, visible=visible, n_stride=n)
        gsmi.adam_step(g.sh[0], grads.sh[0], m1.sh[0], m2.sh[0], lr["sh_dc"], k, visible=visible, n_stride=n)
        gsmi.adam_step(g.sh[1:], grads.sh[1:], m1.sh[1:], m2.sh[1:], lr["sh_rest"], k, visible=visible, n_stride=n)
        gsmi.adam_step(x6[1:], dx6[1:], px_m[1:], px_v[1:], lr["pose"], k, eps=1e-12)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    psnr0 = [10 * math.log10(3 * H * W / float(s)) for s in sums[:, 1].cpu()]

    gsmi.profile_reset()
    gsmi.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    gsmi.profile_enable(False)
    kernels = {}
    for name in ["project", "bin_flags", "bin_compact", "radix_hist", "radix_scatter", "scan", "bin_counts",
                 "bin_duplicate", "bin_ranges", "bin_fill", "render_fwd", "loss_l1", "loss_final", "render_bwd",
                 "project_bwd", "pose_reduce", "adam", "zero", "mark_visible", "pose_6d", "pose_6d_bwd"]:
        ms, cnt = gsmi.profile_read(name)
        if cnt:
            kernels[name] = dict(ms_total=ms, launches=cnt, ms_per_launch=ms / cnt)
    gsmi.profile_reset()
    psnr1 = [10 * math.log10(3 * H * W / float(s)) for s in sums[:, 1].cpu()]

    # one extra step (not timed) with pair counters for the algorithmic work
    step(count_pairs=True)
    torch.cuda.synchronize()
    tile_pairs = sum(p[0] for p in pairs) / N_VIEWS
    evaluated = sum(p[1] for p in pairs) / N_VIEWS
    support = sum(p[2] for p in pairs) / N_VIEWS
    comp = sum(p[3] for p in pairs) / N_VIEWS
    walked = sum(p[4] for p in pairs) / N_VIEWS
    M = sum(p[5] for p in pairs) / N_VIEWS

    ms_step = elapsed * 1e3 / args.steps
    mpix = N_VIEWS * W * H / (ms_step * 1e-3) / 1e6

    def roof(name):
        k = kernels[name]
        t = k["ms_per_launch"] * 1e-3
        if name == "render_fwd":
            ops = support * FWD_PAIR + comp * FWD_COMP
            a = ops / t / 1e12
            return dict(bound="alu", achieved=a, peak=PEAK_VALU_TOPS, unit="Tlane-op/s", frac=a / PEAK_VALU_TOPS,
                        traffic=None)
        if name == "render_bwd":
            ops = comp * BWD_COMP
            a = ops / t / 1e12
            return dict(bound="alu", achieved=a, peak=PEAK_VALU_TOPS, unit="Tlane-op/s", frac=a / PEAK_VALU_TOPS,
                        traffic=None)
        per_launch_bytes = {
            "project": n * (236 + 56),
            "project_bwd": n * (236 + 40 + 2 * 236 + 4),
            "radix_scatter": None,
            "adam": None,
        }.get(name)
        if per_launch_bytes is None:
            return None
        a = per_launch_bytes / t / 1e9
        return dict(bound="hbm", achieved=a, peak=PEAK_HBM_GBS, unit="GB/s", frac=a / PEAK_HBM_GBS, traffic=None)

    dominant = max(kernels, key=lambda k: kernels[k]["ms_total"])
    roofline = roof(dominant)
    if roofline is not None:
        roofline["kernel"] = dominant
        roofline["traffic"] = measured_traffic(dominant)
    others = {k: roof(k) for k in ["render_fwd", "render_bwd", "project", "project_bwd"] if k in kernels}

    out = {
        "metric": "fwd+bwd Mpix/s @1080p 2M Gaussians (joint pose+Gaussian step, 8 keyframes)",
        "value": round(mpix, 2),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "joint pose+Gaussian optimisation step: 8 keyframes x 1920x1080, 2M Gaussians "
                               "(8 x 250k ray-seeded), SH degree 3, L1 loss, sparse Adam",
                   "views": N_VIEWS, "width": W, "height": H, "gaussians": n, "sh_degree": SH_DEG},
        "roofline": roofline,
        "kernel_rooflines": others,
        "kernels_ms_per_step": {k: round(v["ms_total"] / args.steps, 4) for k, v in kernels.items()},
        "pairs_per_view": {"tile_list_to_stop": tile_pairs, "evaluated": evaluated, "support": support,
                           "composited": comp, "tile_list_walked_bwd": walked, "instances": M},
        "psnr_start_end": [round(sum(psnr0) / N_VIEWS, 3), round(sum(psnr1) / N_VIEWS, 3)],
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(views[3], start, args.cpu_crops)
    if args.copy_probe:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
    print(json.dumps(out))


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE /
    WRITE_SIZE counter runs (scaled by a plain copy of known size), or None
    if none were taken or the kernel's source changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get("k_" + kernel)
    if not rec:
        return None
    src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    if hashlib.sha256(src).hexdigest()[:16] != rec["source_sha256_16"]:
        return None
    return rec["bytes_per_launch"]


def cpu_baseline(view, scene, n_crops):
    """The FP64 oracle, as it stands, on a bounded sample of the same view:
    projection and its adjoint over all 2M Gaussians (single thread), and
    forward + backward compositing on n_crops 64x64 crops (threads over
    rows).  The full-view time is the projection passes plus the crop time
    per pixel times the view's pixels."""
    import numpy as np

    from oracle import raster as orc

    threads = min(os.cpu_count() or 1, 64)
    cam = orc.Camera.from_view(view)
    og = orc.Gaussians.from_scene(scene)
    t0 = time.perf_counter()
    op = orc.project(cam, og)
    t_proj = time.perf_counter() - t0
    rng = np.random.default_rng(0)
    t_px = 0.0
    npx = 0
    g2d = np.zeros((og.n, 10))
    for _ in range(n_crops):
        x0 = int(rng.integers(0, view.width - 64))
        y0 = int(rng.integers(0, view.height - 64))
        crop = (x0, y0, 64, 64)
        gi = rng.standard_normal((3, 64, 64)) * 1e-3
        t0 = time.perf_counter()
        orc.render(cam, op, crop=crop, nthreads=threads)
        g2d += orc.render_bwd(cam, op, g_image=gi, crop=crop, nthreads=threads)
        t_px += time.perf_counter() - t0
        npx += 64 * 64
    t0 = time.perf_counter()
    orc.project_bwd(cam, og, g2d)
    t_pbwd = time.perf_counter() - t0
    t_view = t_proj + t_pbwd + t_px / npx * view.width * view.height
    return {"value": round(view.width * view.height / t_view / 1e6, 4), "unit": "Mpix/s", "cores": threads,
            "kind": "oracle",
            "sample": f"one 1920x1080 view of the same 2M-Gaussian scene: FP64 projection + adjoint over all "
                      f"Gaussians ({t_proj + t_pbwd:.2f}s, 1 thread) and fwd+bwd compositing of {n_crops} random "
                      f"64x64 crops ({t_px:.2f}s, {threads} threads), extrapolated per pixel to the full view"}


if __name__ == "__main__":
    main()
