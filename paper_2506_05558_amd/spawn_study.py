"""Steps-to-PSNR of the learned spawn initialisation against the direct rule.

Section 4.2 initialises a spawned primitive directly from the frame (depth,
Clark-Evans scale, pixel colour); the learned variant adds the residuals of a
small MLP that has seen, for many earlier frames, where plain optimisation
took such primitives.  This module runs that comparison on one GPU, every
step in libgsmi's kernels:

1. Frames: `synth.spawn_frame` images (piecewise-constant structure, smooth
   shading and sensor noise) at 1920x1080 with their depth observed with
   1 % multiplicative noise (the paper's monocular depth is not available);
   pinhole camera with f = 0.7 W at the identity pose.  Each frame is a first
   frame: P~ = 0, so P_s = P_L.
2. Spawn: fixed-K selection of K = 100k pixels, direct rule (SH degree 0).
3. Plain optimisation of the spawned set on its frame: L1 loss, Adam with
   3DGS-style rates on means, log-scales, opacity and colour, rotation frozen
   so that the three log-scales keep their camera-aligned meaning.
4. Training pairs: on training seeds, the features of every spawned pixel and
   the residuals (converged - rule) of its primitive after `conv_steps`
   steps: 3 log-scales, opacity logit, colour.
5. The MLP is trained on those pairs with the FP32 training kernels.
6. On held-out seeds, the same optimisation starts from the rule and from the
   rule plus the MLP's residuals; the target PSNR is what the rule reaches
   after 30 steps (the paper's per-keyframe budget, section 4.3), and
   steps-to-PSNR is the first step at which a run reaches it.

Command line: python -m paper_2506_05558_amd.spawn_study --out <json>.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

from . import gsmi, synth

LR = dict(means=1.6e-3, log_scales=5e-3, opacity_logits=5e-2, sh=2.5e-3)
DC = 2.0 * math.sqrt(math.pi)  # colour offset -> DC coefficient


def frame(seed: int, width: int, height: int):
    img, _, depth = synth.spawn_frame(seed, width, height)
    rng = np.random.default_rng(seed + 1_000_003)
    depth = (depth * (1.0 + rng.normal(0.0, 0.01, depth.shape))).astype(np.float32)
    return torch.tensor(img, device="cuda"), torch.tensor(depth, device="cuda")


def camera(width: int, height: int):
    pose = torch.tensor([1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0], dtype=torch.float32, device="cuda")
    f = 0.7 * width
    return gsmi.Camera(width, height, f, f, width / 2.0, height / 2.0, pose)


def spawn(cam, img, depth, k: int, seed: int, packed=None):
    """Spawned Gaussians (SH degree 0) and their pixels."""
    sp = gsmi.SpawnParams(mode=gsmi.SPAWN_FIXED_K, k=k, seed=seed)
    p_l, p_s = gsmi.spawn_probability(cam, img, None, sp)
    pix = gsmi.spawn_select(cam, p_s, sp, capacity=k)
    n = pix.numel()
    z = lambda *s: torch.zeros(s, dtype=torch.float32, device="cuda")
    g = gsmi.Gaussians(z(3, n), z(3, n), z(4, n), z(n), z(1, 3, n))
    gsmi.spawn_rule(cam, img, depth, p_l, pix, g, 0, sp)
    if packed is not None:
        gsmi.spawn_mlp(cam, img, depth, pix, packed, g, 0)
    return g, pix


class Fit:
    """Plain optimisation of one Gaussian set on one view (L1, Adam, rotation
    frozen); `step` returns the PSNR of the state before its update."""

    def __init__(self, cam, target, g, lr=LR):
        self.cam, self.target, self.g, self.lr = cam, target, g, lr
        n = g.n
        H, W = cam.height, cam.width
        self.grads, self.m, self.v = g.zeros_like(), g.zeros_like(), g.zeros_like()
        self.params = gsmi.Params()
        self.sorter = gsmi.BinSorter(capacity=8 * n)
        self.proj = gsmi.alloc_projected(n)
        f = lambda *s, dt=torch.float32: torch.empty(s, dtype=dt, device="cuda")
        self.frame = gsmi.Frame(f(3, H, W), f(H, W), f(H, W), f(H, W), f(H, W, dt=torch.int32))
        self.g_img = f(3, H, W)
        self.sums = torch.zeros(2, dtype=torch.float64, device="cuda")
        self.loss_ws = torch.empty(1 << 16, dtype=torch.uint8, device="cuda")
        self.bwd_ws = None
        self.k = 0
        self.npix = 3 * H * W

    def _forward(self):
        gsmi.project(self.cam, self.g, self.params, out=self.proj)
        b = self.sorter(self.cam, self.proj)
        gsmi.render_fwd(self.cam, self.proj, b, self.params, out=self.frame)
        gsmi.loss_l1(self.frame.image, self.target, 1.0 / self.npix, self.g_img, self.sums, self.loss_ws)
        return b

    def psnr_value(self):
        return 10.0 * math.log10(self.npix / max(float(self.sums[1]), 1e-30))

    def psnr(self):
        self._forward()
        return self.psnr_value()

    def step(self):
        self.k += 1
        for t in self.grads.tensors():
            gsmi.zero_(t)
        b = self._forward()
        need = gsmi.render_bwd_workspace(self.g.n, max(b.n_instances, 1))
        if self.bwd_ws is None or self.bwd_ws.numel() < need:
            self.bwd_ws = torch.empty(int(need * 1.25), dtype=torch.uint8, device="cuda")
        gsmi.render_bwd(self.cam, self.g, self.proj, b, self.frame, self.g_img, grads=self.grads,
                        params=self.params, ws=self.bwd_ws)
        for name in ("means", "log_scales", "opacity_logits", "sh"):
            gsmi.adam_step(getattr(self.g, name), getattr(self.grads, name), getattr(self.m, name),
                           getattr(self.v, name), self.lr[name], self.k)
        return self.psnr_value()


def curve(fit: Fit, steps: int):
    """PSNR after 0 .. steps updates."""
    out = [fit.step() for _ in range(steps)]
    out.append(fit.psnr())
    return out


def residual_targets(g0, g1):
    """(converged - rule) per primitive: 3 log-scales, opacity logit, colour."""
    return torch.cat([(g1.log_scales - g0.log_scales).T, (g1.opacity_logits - g0.opacity_logits)[:, None],
                      ((g1.sh[0] - g0.sh[0]) / DC).T], dim=1).contiguous()


def collect(seeds, width, height, k, conv_steps, log=print):
    X, Y = [], []
    cam = camera(width, height)
    for s in seeds:
        img, depth = frame(s, width, height)
        g, pix = spawn(cam, img, depth, k, s)
        g0 = gsmi.Gaussians(*[t.clone() for t in g.tensors()])
        fit = Fit(cam, img, g)
        c = curve(fit, conv_steps)
        X.append(gsmi.mlp_features(cam, img, depth, pix))
        Y.append(residual_targets(g0, g))
        log(f"# train seed {s}: {pix.numel()} spawned, PSNR {c[0]:.2f} -> {c[30]:.2f} (30) -> {c[-1]:.2f} "
            f"({conv_steps})")
    return torch.cat(X), torch.cat(Y)


def train(X, Y, steps, batch, lr, seed=0, log=print):
    theta = torch.tensor(synth.mlp_init(seed), device="cuda")
    tr = gsmi.MlpTrainer(theta, lr=lr)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    n = X.shape[0]
    nval = max(n // 20, 1)
    perm = torch.randperm(n, device="cuda", generator=gen)
    Xv, Yv = X[perm[:nval]].contiguous(), Y[perm[:nval]].contiguous()
    tr_idx = perm[nval:]
    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(steps):
        # cosine decay of the rate to 5 % of its start
        rate = lr * (0.05 + 0.95 * 0.5 * (1 + math.cos(math.pi * it / steps)))
        idx = tr_idx[torch.randint(0, tr_idx.numel(), (batch,), device="cuda", generator=gen)]
        loss = tr.step(X[idx].contiguous(), Y[idx].contiguous(), lr=rate)
        if it % 500 == 0 or it == steps - 1:
            lt = float(loss)  # the trainer's loss buffer is reused by the next call
            val = float(tr.step(Xv, Yv, lr=0.0))
            losses.append((it, lt, val))
            log(f"# mlp step {it}: train {lt:.5f} held-out {val:.5f}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    base = float(((Yv - Yv.mean(0)) ** 2).mean())  # held-out loss of the best constant
    return tr.theta, dict(losses=losses, seconds=elapsed, held_out_constant_baseline=base)


def time_kernels(cam, img, depth, k, packed, X, batch, reps=20):
    """Kernel time (the library's launch events) of the fused MLP inference
    for the k pixels spawned on a frame, and FP32 training samples per second
    at one step on `batch` samples (three kernels per step)."""
    g, pix = spawn(cam, img, depth, k, 1)
    tr = gsmi.MlpTrainer(torch.tensor(synth.mlp_init(5), device="cuda"))
    Xb = X[:batch].contiguous()
    Yb = torch.zeros((batch, 7), device="cuda")
    for _ in range(3):
        gsmi.spawn_mlp(cam, img, depth, pix, packed, g, 0)
        tr.step(Xb, Yb)
    torch.cuda.synchronize()
    gsmi.profile_reset()
    gsmi.profile_select(["mlp_infer", "mlp_train"])
    gsmi.profile_enable(True)
    for _ in range(reps):
        gsmi.spawn_mlp(cam, img, depth, pix, packed, g, 0)
    for _ in range(reps):
        tr.step(Xb, Yb)
    torch.cuda.synchronize()
    gsmi.profile_enable(False)
    gsmi.profile_select(None)
    infer_ms, n_inf = gsmi.profile_read("mlp_infer")
    train_ms, n_tr = gsmi.profile_read("mlp_train")
    gsmi.profile_reset()
    return dict(mlp_infer_us=round(infer_ms * 1e3 / n_inf, 2), mlp_infer_count=int(pix.numel()),
                mlp_train_us_per_step=round(train_ms * 1e3 / reps, 2), mlp_train_batch=batch,
                mlp_train_samples_per_s=round(batch * reps / (train_ms * 1e-3), 1))


def constant_theta(Y):
    """Parameters of the network that ignores its input and returns the mean
    residual of the training pairs: the best constant correction of the rule."""
    theta = torch.zeros(gsmi.MLP_PARAMS, dtype=torch.float32, device="cuda")
    theta[gsmi.MLP_PARAMS - 7:] = Y.mean(0)
    return theta


def evaluate(arms, seeds, width, height, k, steps, budget=30, log=print):
    """arms: name -> parameters (None = the rule alone).  Steps-to-PSNR of
    each arm against the rule's PSNR after `budget` steps."""
    cam = camera(width, height)
    packed = {a: (None if th is None else gsmi.mlp_pack_bf16(th)) for a, th in arms.items()}
    rows = []
    for s in seeds:
        img, depth = frame(s, width, height)
        curves = {}
        for a in arms:
            g, _ = spawn(cam, img, depth, k, s, packed=packed[a])
            curves[a] = curve(Fit(cam, img, g), steps)
        target = curves["rule"][budget]
        final = curves["rule"][steps]
        row = dict(seed=s, target_psnr=target, final_rule_psnr=final)
        for a, c in curves.items():
            reach = next((i for i, p in enumerate(c) if p >= target), None)
            # ratio of steps: budget / steps to the target; None (infinite) when the run
            # starts at or above the target, budget / steps (a lower bound) if never reached
            ratio = None if reach == 0 else budget / (reach if reach is not None else steps)
            reach_final = next((i for i, p in enumerate(c) if p >= final), None)
            row[a] = dict(steps=reach, reached=reach is not None, ratio=ratio, steps_to_final_rule=reach_final,
                          psnr={i: c[i] for i in (0, 5, 10, 30, steps)})
        rows.append(row)
        log(f"# eval seed {s}: target {target:.2f} dB; steps " +
            ", ".join(f"{a} {row[a]['steps']}" for a in arms) + "; PSNR@5 " +
            ", ".join(f"{a} {row[a]['psnr'][5]:.2f}" for a in arms))
    return rows


def summarise(rows, arm, boot=2000, seed=0):
    r = np.array([np.inf if x[arm]["ratio"] is None else x[arm]["ratio"] for x in rows], np.float64)
    rng = np.random.default_rng(seed)
    meds = np.array([np.median(rng.choice(r, r.size)) for _ in range(boot)])
    fin = lambda v: None if not np.isfinite(v) else round(float(v), 3)
    # "nearest" percentiles: the medians may be infinite, which interpolation turns into NaN
    return dict(median_ratio=fin(np.median(r)), ci95=[fin(np.percentile(meds, 2.5, method="nearest")),
                                                      fin(np.percentile(meds, 97.5, method="nearest"))],
                n=int(r.size), not_reached=int(sum(not x[arm]["reached"] for x in rows)),
                median_steps=float(np.median([np.inf if x[arm]["steps"] is None else x[arm]["steps"] for x in rows])),
                median_steps_to_final_rule=float(np.median([np.inf if x[arm]["steps_to_final_rule"] is None
                                                            else x[arm]["steps_to_final_rule"] for x in rows])),
                mean_psnr_at={k: round(float(np.mean([x[arm]["psnr"][k] for x in rows])), 3)
                              for k in rows[0][arm]["psnr"]})


def parse_range(s):
    a, b = s.split(":")
    return list(range(int(a), int(b)))


def run(width=1920, height=1080, k=100_000, train_seeds="100:140", eval_seeds="200:208", conv_steps=200,
        eval_steps=100, mlp_steps=4000, mlp_batch=4096, mlp_lr=1e-3, log=print):
    """The whole study; returns its report (see the module docstring)."""
    t0 = time.time()
    X, Y = collect(parse_range(train_seeds), width, height, k, conv_steps, log)
    log(f"# {X.shape[0]} pairs in {time.time() - t0:.1f}s; residual means {Y.mean(0).tolist()}")
    theta, tinfo = train(X, Y, mlp_steps, mlp_batch, mlp_lr, log=log)
    arms = dict(rule=None, constant=constant_theta(Y), learned=theta)
    rows = evaluate(arms, parse_range(eval_seeds), width, height, k, eval_steps, log=log)
    cam = camera(width, height)
    img, depth = frame(999, width, height)
    timing = time_kernels(cam, img, depth, k, gsmi.mlp_pack_bf16(theta), X, mlp_batch)
    return dict(config=dict(width=width, height=height, k=k, train_seeds=train_seeds, eval_seeds=eval_seeds,
                            conv_steps=conv_steps, eval_steps=eval_steps, mlp_steps=mlp_steps, mlp_batch=mlp_batch,
                            mlp_lr=mlp_lr, lr=LR),
                pairs=int(X.shape[0]), residual_mean=Y.mean(0).tolist(), residual_std=Y.std(0).tolist(),
                training=tinfo, eval=rows, summary={a: summarise(rows, a) for a in arms}, timing=timing,
                seconds=round(time.time() - t0, 1)), theta


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--width", type=int, default=1920)
    ap.add_argument("--height", type=int, default=1080)
    ap.add_argument("--k", type=int, default=100_000)
    ap.add_argument("--train-seeds", default="100:140")
    ap.add_argument("--eval-seeds", default="200:208")
    ap.add_argument("--conv-steps", type=int, default=200)
    ap.add_argument("--eval-steps", type=int, default=100)
    ap.add_argument("--mlp-steps", type=int, default=4000)
    ap.add_argument("--mlp-batch", type=int, default=4096)
    ap.add_argument("--mlp-lr", type=float, default=1e-3)
    ap.add_argument("--out", default=None)
    ap.add_argument("--theta-out", default=None)
    a = ap.parse_args(argv)
    log = lambda m: print(m, file=sys.stderr, flush=True)
    torch.cuda.set_device(0)
    res, theta = run(a.width, a.height, a.k, a.train_seeds, a.eval_seeds, a.conv_steps, a.eval_steps, a.mlp_steps,
                     a.mlp_batch, a.mlp_lr, log)
    if a.out:
        os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
        with open(a.out, "w") as fh:
            json.dump(res, fh, indent=1)
    if a.theta_out:
        np.save(a.theta_out, theta.cpu().numpy())
    print(json.dumps(dict(summary=res["summary"], timing=res["timing"], pairs=res["pairs"])))


if __name__ == "__main__":
    main()
