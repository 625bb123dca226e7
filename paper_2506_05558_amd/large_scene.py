"""Large-scene workload: a scene that is not kept on the device as a whole
(the scalable construction of section 4.4, at scene scale), optimised
jointly with the poses along a long trajectory (section 4.3) with the
learned spawn initialisation on.

Orchestration of libgsmi's calls only; torch supplies device and pinned
host memory, streams and events.

* Cells: Lloyd's k-means (gs_cells_kmeans) over the means of the whole
  scene, and each cell's bounding sphere (gs_cells_spheres).
* Store: every cell's rows -- its parameters, both Adam moments and its
  per-Gaussian rate factors -- in pinned CPU RAM, one [rows][count] block
  per cell.
* Pool: the device holds pages of PAGE Gaussians; one [rows][pages x PAGE]
  buffer whose row views are the parameters, moments and rates the
  rasterizer and the optimiser see.  A resident cell owns ceil(count /
  PAGE) pages; the columns of a page that no Gaussian uses carry an opacity
  logit that the projection culls.
* Residency: before each keyframe the cells whose spheres meet a frustum of
  the window's views (gs_cells_visible) must be resident.  Cells no longer
  needed are written back to their host blocks and their pages culled; newly
  needed cells are copied in (gs_copy_rows, one call per page); all of it
  on a side stream that first waits for the main stream's last update, and
  the main stream waits for the copies before the keyframe's first
  projection.
* Keyframe: the new frame's spawn step (P~ from the current model's render,
  fixed-K selection, the rule plus the learned residuals), then joint
  iterations over the window (projection of the resident pool into every
  view, per-view sort on a side stream, forward with the L1 loss, adjoint,
  projection adjoint with pose gradients, sparse Adam with per-Gaussian
  rates, pose Adam through the 6D parametrisation; keyframe 0 fixed).
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass
from typing import Dict, List, Optional

import numpy as np
import torch

from . import gsmi, synth

PAGE = 16384
CULLED_LOGIT = -1.0e4  # sigmoid(-1e4) = 0 < alpha_min: the projection culls it


def param_rows(sh_degree: int) -> int:
    return 3 + 3 + 4 + 1 + 3 * (sh_degree + 1) ** 2


def total_rows(sh_degree: int) -> int:
    """Parameters, first and second Adam moments, rate factor."""
    return 3 * param_rows(sh_degree) + 1


def _gauss_view(rows: torch.Tensor, d: int) -> gsmi.Gaussians:
    n = rows.shape[1]
    nb = (d + 1) ** 2
    return gsmi.Gaussians(rows[0:3], rows[3:6], rows[6:10], rows[10], rows[11:11 + 3 * nb].view(nb, 3, n))


class CellStore:
    """Every cell's rows in pinned CPU RAM: block j is [rows][count_j]."""

    def __init__(self, arrays: Dict[str, np.ndarray], order: np.ndarray, offsets: np.ndarray, sh_degree: int):
        self.d = sh_degree
        self.R = total_rows(sh_degree)
        P = param_rows(sh_degree)
        self.k = len(offsets) - 1
        self.count = np.diff(offsets).astype(np.int64)
        self.off = np.concatenate([[0], np.cumsum(self.count * self.R)]).astype(np.int64)
        self.host = torch.empty(int(self.off[-1]), dtype=torch.float32, pin_memory=True)
        n = int(offsets[-1])
        flat = np.concatenate([arrays["means"], arrays["log_scales"], arrays["quats"],
                               arrays["opacity_logits"][None], arrays["sh"].reshape(-1, n)], axis=0)
        assert flat.shape[0] == P
        h = self.host.numpy()
        for j in range(self.k):
            idx = order[offsets[j]:offsets[j + 1]]
            c = int(self.count[j])
            blk = h[self.off[j]:self.off[j + 1]].reshape(self.R, c)
            blk[:P] = flat[:, idx]
            blk[P:3 * P] = 0.0  # Adam moments start at zero
            blk[3 * P] = 1.0  # rate factor of a new Gaussian
        self.bytes = int(self.off[-1]) * 4

    def ptr(self, j: int, col: int = 0) -> int:
        return self.host.data_ptr() + int(self.off[j] + col) * 4


class PagePool:
    """Device pages: one [rows][pages x PAGE] buffer and its row views."""

    def __init__(self, n_pages: int, sh_degree: int, device="cuda"):
        self.d = sh_degree
        self.R = total_rows(sh_degree)
        P = param_rows(sh_degree)
        self.n_pages = n_pages
        self.n = n_pages * PAGE
        self.buf = torch.zeros((self.R, self.n), dtype=torch.float32, device=device)
        self.g = _gauss_view(self.buf[0:P], sh_degree)
        self.m1 = _gauss_view(self.buf[P:2 * P], sh_degree)
        self.m2 = _gauss_view(self.buf[2 * P:3 * P], sh_degree)
        self.rates = self.buf[3 * P]
        gsmi.fill_(self.g.opacity_logits, CULLED_LOGIT)
        self.free = list(range(n_pages))[::-1]

    def opacity_cols(self, page: int, c0: int, c1: int) -> torch.Tensor:
        return self.g.opacity_logits[page * PAGE + c0:page * PAGE + c1]


class Residency:
    """Which cells are on the device, and the copies that change it."""

    def __init__(self, store: CellStore, pool: PagePool, centroids: torch.Tensor, radius: torch.Tensor):
        self.store, self.pool = store, pool
        self.cent, self.radius = centroids, radius
        self.pages: Dict[int, List[int]] = {}
        self.side = torch.cuda.Stream()
        self.ev_main = torch.cuda.Event()
        self.ev_done = torch.cuda.Event()
        self.flags = torch.zeros((64, store.k), dtype=torch.int32, device=pool.buf.device)
        self.h2d_bytes = 0
        self.d2h_bytes = 0
        self.loads = 0
        self.evictions = 0

    def needed(self, cams) -> set:
        """Cells whose sphere meets any of the cameras' frusta (one sync)."""
        assert len(cams) <= self.flags.shape[0]
        for i, cam in enumerate(cams):
            gsmi.cells_visible(self.cent, self.radius, cam, out=self.flags[i])
        f = self.flags[:len(cams)].amax(0).cpu().numpy()
        return set(np.nonzero(f)[0].tolist())

    def pages_for(self, cells) -> int:
        return int(sum(math.ceil(self.store.count[j] / PAGE) for j in cells))

    def _rows(self, j: int, p: int, i: int):
        """(device address, host address, width in bytes) of page i of cell j."""
        c0 = i * PAGE
        cnt = int(min(PAGE, self.store.count[j] - c0))
        dev = self.pool.buf.data_ptr() + p * PAGE * 4
        return dev, self.store.ptr(j, c0), cnt

    def update(self, needed: set):
        """Write back and free the cells not needed, copy in the new ones; the
        main stream waits for it before its next kernel."""
        st, pool, R = self.store, self.pool, self.store.R
        dpitch = pool.n * 4
        self.ev_main.record()
        with torch.cuda.stream(self.side):
            self.side.wait_event(self.ev_main)
            for j in [c for c in self.pages if c not in needed]:
                spitch = int(st.count[j]) * 4
                for i, p in enumerate(self.pages[j]):
                    dev, host, cnt = self._rows(j, p, i)
                    gsmi.copy_rows(host, spitch, dev, dpitch, cnt * 4, R)
                    gsmi.fill_(pool.opacity_cols(p, 0, PAGE), CULLED_LOGIT)
                    self.d2h_bytes += cnt * 4 * R
                    pool.free.append(p)
                del self.pages[j]
                self.evictions += 1
            for j in sorted(needed - set(self.pages)):
                npg = math.ceil(st.count[j] / PAGE)
                if len(pool.free) < npg:
                    raise RuntimeError(f"page pool too small: cell {j} needs {npg} pages, {len(pool.free)} free")
                spitch = int(st.count[j]) * 4
                pages = [pool.free.pop() for _ in range(npg)]
                for i, p in enumerate(pages):
                    dev, host, cnt = self._rows(j, p, i)
                    gsmi.copy_rows(dev, dpitch, host, spitch, cnt * 4, R)
                    if cnt < PAGE:
                        gsmi.fill_(pool.opacity_cols(p, cnt, PAGE), CULLED_LOGIT)
                    self.h2d_bytes += cnt * 4 * R
                self.pages[j] = pages
                self.loads += 1
            self.ev_done.record(self.side)
        torch.cuda.current_stream().wait_event(self.ev_done)

    def resident(self) -> int:
        return int(sum(self.store.count[j] for j in self.pages))


@dataclass
class Config:
    width: int = 2560
    height: int = 1440
    frames: int = 200
    per_frame: int = 30_000  # 6M Gaussians seeded from 200 keyframes
    cells: int = 120
    kmeans_iters: int = 20
    window: int = 4
    iters: int = 10
    sh_degree: int = 3
    spawn_k: int = 100_000
    seed: int = 2560
    lr_decay: float = 0.995


LR = dict(means=1.6e-3, log_scales=5e-3, quats=1e-3, opacity_logits=5e-2, sh_dc=2.5e-3, sh_rest=1.25e-4, pose=1e-4)


def _pose_tensor(v, dev="cuda"):
    return torch.tensor(np.concatenate([v.R.reshape(9), v.t]).astype(np.float32), device=dev)


class LargeScene:
    """The scene, its cells, the store, the pool and the optimiser state."""

    def __init__(self, cfg: Config, log=print, mlp_theta: Optional[torch.Tensor] = None):
        t0 = time.time()
        self.cfg, self.log = cfg, log
        W, H, d = cfg.width, cfg.height, cfg.sh_degree
        self.views = synth.trajectory(cfg.seed, cfg.frames, W, H)
        gt = synth.window_scene(cfg.seed, self.views, cfg.per_frame, d)
        start = synth.perturb_scene(cfg.seed, gt)
        self.n_scene = gt.n
        log(f"# large scene: {gt.n} Gaussians from {cfg.frames} keyframes in {time.time() - t0:.1f}s")
        self.params = gsmi.Params(eps2d=0.1, mip_filter=1)
        # ground truth on the device stands in for the captured images
        self.gt = gsmi.Gaussians.from_arrays(gt.arrays())
        self.gt_sorter = gsmi.BinSorter(capacity=1 << 24)
        # cells over the optimised model's means
        means = torch.tensor(start.means, device="cuda")
        ls = torch.tensor(start.log_scales, device="cuda")
        t1 = time.time()
        self.cent, labels, order, offsets = gsmi.cells_kmeans(means, cfg.cells, cfg.kmeans_iters)
        # the alpha >= 1/255 support reaches sqrt(2 ln 255) = 3.33 of the largest axis scale
        self.radius = gsmi.cells_spheres(means, ls, labels, self.cent, margin=3.5)
        torch.cuda.synchronize()
        self.kmeans_s = time.time() - t1
        order, offsets = order.cpu().numpy(), offsets.cpu().numpy()
        del means, ls, labels
        t1 = time.time()
        self.store = CellStore(start.arrays(), order, offsets, d)
        log(f"# cells: {cfg.cells} (k-means {self.kmeans_s:.2f}s), sizes {int(np.diff(offsets).min())}.."
            f"{int(np.diff(offsets).max())}; host store {self.store.bytes / 2**30:.2f} GiB in {time.time() - t1:.1f}s")
        # poses: keyframe 0 fixed, the others perturbed, 6D parametrisation
        rng = np.random.default_rng(cfg.seed)
        x6 = np.zeros((cfg.frames, 9), np.float32)
        for i, v in enumerate(self.views):
            R, t = (v.R, v.t) if i == 0 else synth.perturb_pose(rng, v.R, v.t, 0.01)
            x6[i] = np.concatenate([R[:, 0], R[:, 1], t])
        self.x6 = torch.tensor(x6, device="cuda")
        self.dx6 = torch.zeros_like(self.x6)
        self.px_m, self.px_v = torch.zeros_like(self.x6), torch.zeros_like(self.x6)
        self.poses = torch.zeros((cfg.frames, 12), dtype=torch.float32, device="cuda")
        self.d_pose = torch.zeros((cfg.frames, 12), dtype=torch.float64, device="cuda")
        gsmi.pose_from_6d(self.x6, self.poses)
        self.cams = [gsmi.Camera(W, H, v.fx, v.fy, v.cx, v.cy, self.poses[i]) for i, v in enumerate(self.views)]
        self.gt_cams = [gsmi.Camera(W, H, v.fx, v.fy, v.cx, v.cy, _pose_tensor(v)) for v in self.views]
        # the pool: sized for the largest window's cells (visibility from the true poses)
        probe = Residency(self.store, PagePool(1, d), self.cent, self.radius)
        need = 0
        for f in range(cfg.frames):
            win = self.window(f)
            need = max(need, probe.pages_for(probe.needed([self.gt_cams[i] for i in win])))
        self.pool = PagePool(int(need * 1.15) + 8, d)
        self.res = Residency(self.store, self.pool, self.cent, self.radius)
        log(f"# page pool: {self.pool.n_pages} pages of {PAGE} ({self.pool.n} Gaussians, "
            f"{self.pool.buf.numel() * 4 / 2**30:.2f} GiB) for at most {need} pages per window")
        self.theta = mlp_theta
        self.packed = gsmi.mlp_pack_bf16(mlp_theta) if mlp_theta is not None else None
        self._alloc_step()

    def window(self, f: int) -> List[int]:
        return list(range(max(0, f - self.cfg.window + 1), f + 1))

    # ------------------------------------------------------------ buffers
    def _alloc_step(self):
        cfg, n, d = self.cfg, self.pool.n, self.cfg.sh_degree
        W, H = cfg.width, cfg.height
        f = lambda *s, dt=torch.float32: torch.empty(s, dtype=dt, device="cuda")
        P = param_rows(d)
        self.gflat = torch.zeros((P, n), dtype=torch.float32, device="cuda")
        self.grads = _gauss_view(self.gflat, d)
        self.visible = torch.zeros(n, dtype=torch.int32, device="cuda")
        self.frame = gsmi.Frame(f(3, H, W), f(H, W), f(H, W), f(H, W), f(H, W, dt=torch.int32))
        self.g_img = f(3, H, W)
        self.sums = torch.zeros((cfg.window, 2), dtype=torch.float64, device="cuda")
        self.fwd_ws = torch.empty(gsmi.render_fwd_l1_workspace(W, H), dtype=torch.uint8, device="cuda")
        self.wviews = [gsmi.View(self.cams[0], gsmi.alloc_projected(n), None,
                                 torch.empty(n, dtype=torch.int32, device="cuda"), None)
                       for _ in range(cfg.window)]
        self.pbwd_ws = torch.empty(gsmi.project_bwd_views_workspace(n, cfg.window), dtype=torch.uint8, device="cuda")
        self.sorters = [gsmi.BinSorter(capacity=0) for _ in range(cfg.window)]
        self.n_pairs = torch.zeros(cfg.window, dtype=torch.int32, device="cuda")
        self.n_pairs_max = torch.zeros(cfg.window, dtype=torch.int32, device="cuda")
        self.side = torch.cuda.Stream()
        self.ev_proj = torch.cuda.Event()
        self.ev_sorted = [torch.cuda.Event() for _ in range(cfg.window)]
        self.targets: Dict[int, torch.Tensor] = {}
        self.depths: Dict[int, torch.Tensor] = {}
        self.spawn_sorter = gsmi.BinSorter(capacity=1 << 23)
        self.probe_sorter = gsmi.BinSorter(capacity=1 << 23)
        self.spawned = gsmi.Gaussians(f(3, cfg.spawn_k), f(3, cfg.spawn_k), f(4, cfg.spawn_k), f(cfg.spawn_k),
                                      f((d + 1) ** 2, 3, cfg.spawn_k))
        gsmi.zero_(self.spawned.sh)
        self.spawn_ws = torch.empty(gsmi.spawn_init_workspace(W, H, cfg.spawn_k), dtype=torch.uint8, device="cuda")
        self.rendered = f(3, H, W)
        self.step_count = 0
        self.n_spawned: List[int] = []

    # ------------------------------------------------------------ targets
    def target(self, i: int) -> torch.Tensor:
        if i not in self.targets:
            cam = self.gt_cams[i]
            pr = gsmi.project(cam, self.gt, self.params)
            b = self.gt_sorter(cam, pr)
            fr = gsmi.render_fwd(cam, pr, b, self.params)
            self.targets[i] = fr.image.clone()
            dn = torch.tensor(np.random.default_rng(self.cfg.seed + i).normal(0, 0.01, fr.depth.shape)
                              .astype(np.float32), device="cuda")
            dep = torch.where(fr.alpha > 1e-3, fr.depth / fr.alpha.clamp_min(1e-3), torch.full_like(fr.depth, 20.0))
            self.depths[i] = (dep * (1 + dn)).contiguous()
        return self.targets[i]

    def drop_targets(self, keep):
        for i in [i for i in self.targets if i not in keep]:
            del self.targets[i]
            del self.depths[i]

    # ------------------------------------------------------------ keyframe
    def spawn(self, f: int):
        """The spawn step on frame f: P~ from the current model's render."""
        cam, pool, cfg = self.cams[f], self.pool, self.cfg
        view = self.wviews[0]
        gsmi.project(cam, pool.g, self.params, out=view.proj)
        b = self.spawn_sorter(cam, view.proj)
        fr = gsmi.Frame(self.rendered, self.frame.depth, self.frame.alpha, self.frame.final_t, self.frame.n_contrib)
        gsmi.render_fwd(cam, view.proj, b, self.params, out=fr)
        sp = gsmi.SpawnParams(mode=gsmi.SPAWN_FIXED_K, k=cfg.spawn_k, seed=cfg.seed + f)
        self.n_spawned.append(gsmi.spawn_init(cam, self.target(f), self.depths[f], self.spawned, 0,
                                              rendered=self.rendered, sp=sp, mlp_packed=self.packed,
                                              ws=self.spawn_ws))

    def size_lists(self, win):
        """One synchronous sort per view: list capacities for the keyframe."""
        gsmi.pose_from_6d(self.x6, self.poses)
        for i, fi in enumerate(win):
            vw = self.wviews[i]
            vw.cam = self.cams[fi]
            gsmi.project(vw.cam, self.pool.g, self.params, out=vw.proj)
            m = self.probe_sorter(vw.cam, vw.proj).n_instances
            cap = int(m * 1.25) + 65536
            if self.sorters[i].capacity < cap:
                self.sorters[i] = gsmi.BinSorter(capacity=cap)
                self.sorters[i].reserve(self.pool.n, vw.cam.tiles_x * vw.cam.tiles_y, "cuda")
            cap = self.sorters[i].capacity
            if vw.pair_grad is None or vw.pair_grad.shape[0] < cap:
                vw.pair_grad = torch.empty((cap, 12), dtype=torch.float32, device="cuda")

    def joint_iteration(self, win):
        cfg, pool = self.cfg, self.pool
        self.step_count += 1
        k = self.step_count
        views = self.wviews[:len(win)]
        gsmi.zero_(self.d_pose)
        gsmi.zero_(self.dx6)
        gsmi.pose_from_6d(self.x6, self.poses)
        for i, fi in enumerate(win):
            views[i].cam = self.cams[fi]
            views[i].dL_dpose = self.d_pose[fi]
        gsmi.project_views(views, pool.g, self.params)
        self.ev_proj.record()
        lists = []
        with torch.cuda.stream(self.side):
            self.side.wait_event(self.ev_proj)
            for i, vw in enumerate(views):
                lists.append(self.sorters[i].sort_async(vw.cam, vw.proj, self.n_pairs[i:i + 1],
                                                        first_slot=vw.first_slot))
                self.ev_sorted[i].record(self.side)
        H, W = cfg.height, cfg.width
        scale = 1.0 / (3 * H * W * len(win))
        for i, vw in enumerate(views):
            torch.cuda.current_stream().wait_event(self.ev_sorted[i])
            b = lists[i]
            gsmi.render_fwd_l1(vw.cam, vw.proj, b, self.target(win[i]), scale, self.g_img, self.sums[i],
                               self.fwd_ws, self.params, out=self.frame)
            gsmi.render_bwd_pairs(vw.cam, vw.proj, b, self.frame, self.g_img, vw.pair_grad, params=self.params)
        # the window's adjoint with the sparse Adam step and the rate decay in its last pass (the
        # geometry pass writes the set the step updates)
        opt = gsmi.AdamGroups(lr_means=LR["means"], lr_log_scales=LR["log_scales"], lr_quats=LR["quats"],
                              lr_opacity=LR["opacity_logits"], lr_sh_dc=LR["sh_dc"], lr_sh_rest=LR["sh_rest"],
                              step=k, lr_decay=cfg.lr_decay)
        gsmi.project_bwd_views_adam(views, pool.g, self.grads, pool.m1, pool.m2, opt, self.visible,
                                    lr_scale=pool.rates, params=self.params, ws=self.pbwd_ws)
        torch.maximum(self.n_pairs_max[:len(win)], self.n_pairs[:len(win)], out=self.n_pairs_max[:len(win)])
        gsmi.pose_6d_bwd(self.x6, self.d_pose, self.dx6)
        # poses of the window except keyframe 0
        lo = max(win[0], 1)
        if lo <= win[-1]:
            gsmi.adam_step(self.x6[lo:win[-1] + 1], self.dx6[lo:win[-1] + 1], self.px_m[lo:win[-1] + 1],
                           self.px_v[lo:win[-1] + 1], LR["pose"], k, eps=1e-12)

    def keyframe(self, f: int, iters: int):
        """Residency, spawn and the joint iterations of keyframe f; returns
        the number of iterations run."""
        win = self.window(f)
        self.drop_targets(set(win))
        for i in win:
            self.target(i)
        need = self.res.needed([self.cams[i] for i in win])
        self.res.update(need)
        self.spawn(f)
        self.size_lists(win)
        gsmi.zero_(self.n_pairs_max)
        for _ in range(iters):
            self.joint_iteration(win)
        return win

    def check_lists(self, win):
        mx = self.n_pairs_max[:len(win)].cpu().numpy()
        cap = np.array([self.sorters[i].capacity for i in range(len(win))])
        if np.any(mx > cap):
            raise RuntimeError(f"pair lists overflowed: {mx.tolist()} > {cap.tolist()}")
        return int(mx.max())

    def psnr(self, win) -> float:
        return float(np.mean([10 * math.log10(3 * self.cfg.height * self.cfg.width / max(float(s), 1e-30))
                              for s in self.sums[:len(win), 1].cpu()]))


# ------------------------------------------------------- steps-to-PSNR study
SPAWN_LR = dict(means=1.6e-3, log_scales=5e-3, opacity_logits=5e-2, sh=2.5e-3)
DC = 2.0 * math.sqrt(math.pi)  # colour offset -> DC coefficient


class UnionFit:
    """Optimisation of a keyframe's spawned primitives composited with the
    current model (frozen): the union is rendered, only the spawned part is
    updated (L1 on the keyframe's image, Adam, rotation frozen so that the
    three log-scales keep their camera-aligned meaning)."""

    def __init__(self, cam, target, model: gsmi.Gaussians, spawned: gsmi.Gaussians, params, lr=SPAWN_LR):
        self.cam, self.target, self.params, self.lr = cam, target, params, lr
        self.n0 = model.n
        self.g = gsmi.Gaussians(*[torch.cat([a, b], dim=-1).contiguous()
                                  for a, b in zip(model.tensors(), spawned.tensors())])
        n = self.g.n
        H, W = cam.height, cam.width
        self.grads, self.m, self.v = self.g.zeros_like(), self.g.zeros_like(), self.g.zeros_like()
        self.sorter = gsmi.BinSorter(capacity=1 << 23)
        self.proj = gsmi.alloc_projected(n)
        f = lambda *s, dt=torch.float32: torch.empty(s, dtype=dt, device="cuda")
        self.frame = gsmi.Frame(f(3, H, W), f(H, W), f(H, W), f(H, W), f(H, W, dt=torch.int32))
        self.g_img = f(3, H, W)
        self.sums = torch.zeros(2, dtype=torch.float64, device="cuda")
        self.loss_ws = torch.empty(1 << 16, dtype=torch.uint8, device="cuda")
        self.visible = torch.zeros(n, dtype=torch.int32, device="cuda")
        self.bwd_ws = None
        self.k = 0
        self.npix = 3 * H * W

    def spawned(self) -> gsmi.Gaussians:
        return gsmi.Gaussians(*[t[..., self.n0:] for t in self.g.tensors()])

    def _forward(self):
        gsmi.project(self.cam, self.g, self.params, out=self.proj)
        b = self.sorter(self.cam, self.proj)
        gsmi.render_fwd(self.cam, self.proj, b, self.params, out=self.frame)
        gsmi.loss_l1(self.frame.image, self.target, 1.0 / self.npix, self.g_img, self.sums, self.loss_ws)
        return b

    def psnr_value(self):
        return 10.0 * math.log10(self.npix / max(float(self.sums[1]), 1e-30))

    def step(self):
        self.k += 1
        gsmi.zero_(self.visible)
        for t in self.grads.tensors():
            gsmi.zero_(t)
        b = self._forward()
        need = gsmi.render_bwd_workspace(self.g.n, max(b.n_instances, 1))
        if self.bwd_ws is None or self.bwd_ws.numel() < need:
            self.bwd_ws = torch.empty(int(need * 1.25), dtype=torch.uint8, device="cuda")
        gsmi.render_bwd(self.cam, self.g, self.proj, b, self.frame, self.g_img, grads=self.grads,
                        params=self.params, ws=self.bwd_ws)
        gsmi.mark_visible(self.proj, self.visible)
        gsmi.zero_(self.visible[:self.n0])  # the model is frozen
        n = self.g.n
        for name in ("means", "log_scales", "opacity_logits", "sh"):
            gsmi.adam_step(getattr(self.g, name), getattr(self.grads, name), getattr(self.m, name),
                           getattr(self.v, name), self.lr[name], self.k, visible=self.visible, n_stride=n)
        return self.psnr_value()

    def curve(self, steps):
        out = [self.step() for _ in range(steps)]
        self._forward()
        out.append(self.psnr_value())
        return out


def spawn_set(ls: LargeScene, f: int, packed=None, k: Optional[int] = None):
    """The keyframe's spawned primitives (rule, or rule + the network's
    residuals), P~ from the current model's render, and their pixels."""
    cam, cfg = ls.cams[f], ls.cfg
    k = k or cfg.spawn_k
    view = ls.wviews[0]
    gsmi.project(cam, ls.pool.g, ls.params, out=view.proj)
    b = ls.spawn_sorter(cam, view.proj)
    fr = gsmi.Frame(ls.rendered, ls.frame.depth, ls.frame.alpha, ls.frame.final_t, ls.frame.n_contrib)
    gsmi.render_fwd(cam, view.proj, b, ls.params, out=fr)
    sp = gsmi.SpawnParams(mode=gsmi.SPAWN_FIXED_K, k=k, seed=cfg.seed + 7 * f)
    img, dep = ls.target(f), ls.depths[f]
    p_l, p_s = gsmi.spawn_probability(cam, img, ls.rendered, sp)
    pix = gsmi.spawn_select(cam, p_s, sp, capacity=k)
    m = pix.numel()
    d = cfg.sh_degree
    z = lambda *s: torch.zeros(s, dtype=torch.float32, device="cuda")
    g = gsmi.Gaussians(z(3, m), z(3, m), z(4, m), z(m), z((d + 1) ** 2, 3, m))
    gsmi.spawn_rule(cam, img, dep, p_l, pix, g, 0, sp)
    if packed is not None:
        gsmi.spawn_mlp(cam, img, dep, pix, packed, g, 0)
    return g, pix


def log_pairs(ls: LargeScene, f: int, conv_steps: int, k: int):
    """Training pairs of keyframe f: features of the spawned pixels and the
    residuals (converged - rule) after conv_steps of UnionFit."""
    g, pix = spawn_set(ls, f, None, k)
    g0 = gsmi.Gaussians(*[t.clone() for t in g.tensors()])
    fit = UnionFit(ls.cams[f], ls.target(f), ls.pool.g, g, ls.params)
    c = fit.curve(conv_steps)
    g1 = fit.spawned()
    y = torch.cat([(g1.log_scales - g0.log_scales).T, (g1.opacity_logits - g0.opacity_logits)[:, None],
                   ((g1.sh[0] - g0.sh[0]) / DC).T], dim=1).contiguous()
    x = gsmi.mlp_features(ls.cams[f], ls.target(f), ls.depths[f], pix)
    return x, y, c


def steps_to_psnr(ls: LargeScene, f: int, arms: Dict[str, Optional[torch.Tensor]], k: int, steps: int = 30,
                  budget: int = 30):
    """Each arm's PSNR curve on keyframe f from the same model state; the
    target is what the rule reaches after `budget` steps."""
    curves = {}
    for a, packed in arms.items():
        g, _ = spawn_set(ls, f, packed, k)
        curves[a] = UnionFit(ls.cams[f], ls.target(f), ls.pool.g, g, ls.params).curve(steps)
    target = curves["rule"][budget]
    row = dict(frame=f, target_psnr=target)
    for a, c in curves.items():
        reach = next((i for i, p in enumerate(c) if p >= target), None)
        row[a] = dict(steps=reach, psnr={i: c[i] for i in (0, 5, 10, steps)})
    return row


def run(cfg: Config = Config(), train_frames=None, eval_frames=None, conv_steps: int = 100, study_k: int = 50_000,
        mlp_steps: int = 3000, log=print):
    """The large-scene workload; returns its report."""
    from . import spawn_study
    half = cfg.frames // 2
    if train_frames is None:  # keyframes 20, 30, ..., 90 of 200
        train_frames = list(range(min(20, cfg.frames // 4), half, max(1, cfg.frames // 20)))
    if eval_frames is None:  # keyframes 110, 130, ..., 190 of 200
        eval_frames = list(range(half + max(1, cfg.frames // 20), cfg.frames, max(1, cfg.frames // 10)))
    ls = LargeScene(cfg, log=log)
    W, H = cfg.width, cfg.height
    X, Y = [], []
    rows = []
    t_kf = []
    pix = 0
    resident_max = 0
    arms = None
    for f in range(cfg.frames):
        if f == half and X:
            # the spawn network from the pairs this run logged; learned spawn-init from here on
            Xc, Yc = torch.cat(X), torch.cat(Y)
            theta, tinfo = spawn_study.train(Xc, Yc, mlp_steps, 4096, 1e-3, log=log)
            ls.packed = gsmi.mlp_pack_bf16(theta)
            arms = dict(rule=None, constant=gsmi.mlp_pack_bf16(spawn_study.constant_theta(Yc)), learned=ls.packed)
            log(f"# spawn network trained on {Xc.shape[0]} pairs from {len(X)} keyframes")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        win = ls.keyframe(f, cfg.iters)
        torch.cuda.synchronize()
        t_kf.append(time.perf_counter() - t0)
        ls.check_lists(win)
        pix += cfg.iters * len(win) * W * H
        resident_max = max(resident_max, ls.res.resident())
        if f in train_frames:
            x, y, c = log_pairs(ls, f, conv_steps, study_k)
            X.append(x)
            Y.append(y)
            log(f"# keyframe {f}: logged {x.shape[0]} pairs, PSNR {c[0]:.2f} -> {c[-1]:.2f}")
        if arms is not None and f in eval_frames:
            rows.append(steps_to_psnr(ls, f, arms, study_k))
            r = rows[-1]
            log(f"# keyframe {f}: target {r['target_psnr']:.2f} dB; steps rule {r['rule']['steps']}, "
                f"constant {r['constant']['steps']}, learned {r['learned']['steps']}")
        if f % 20 == 0 or f == cfg.frames - 1:
            log(f"# keyframe {f}: {t_kf[-1] * 1e3:.0f} ms, window PSNR {ls.psnr(win):.2f} dB, resident "
                f"{ls.res.resident()} of {ls.n_scene}, loads {ls.res.loads}, evictions {ls.res.evictions}")
    total = float(np.sum(t_kf))
    return ls, dict(total_s=total, mpix_per_s=pix / total / 1e6, pixels=pix, keyframe_ms=[round(t * 1e3, 2) for t in t_kf],
                    resident_max=resident_max, n_scene=ls.n_scene, pool_gaussians=ls.pool.n,
                    h2d_gb=ls.res.h2d_bytes / 1e9, d2h_gb=ls.res.d2h_bytes / 1e9, loads=ls.res.loads,
                    evictions=ls.res.evictions, kmeans_s=ls.kmeans_s, eval=rows,
                    summary={a: _summary(rows, a) for a in ("rule", "constant", "learned")} if rows else None)


def _summary(rows, arm):
    st = [np.inf if r[arm]["steps"] is None else r[arm]["steps"] for r in rows]
    return dict(median_steps=float(np.median(st)), n=len(rows),
                mean_psnr_at={k: round(float(np.mean([r[arm]["psnr"][k] for r in rows])), 3)
                              for k in rows[0][arm]["psnr"]})
