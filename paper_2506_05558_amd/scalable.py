"""Scalable incremental construction (section 4.4): the active Gaussians on
the device, anchors in CPU RAM, and the sliding window between them.

Orchestration of libgsmi's calls only (every per-Gaussian step runs in the
library's kernels; torch supplies device and pinned host memory, streams
and events):

* creation trigger -- gs_anchor_sizes from the previous camera: more than
  40 % of the active Gaussians smaller than tau_min = 1 pixel;
* the anchor -- the active set before the update (parameters, both Adam
  moments, the per-Gaussian rates) and the keyframes it was optimised with,
  copied to pinned host memory by gs_anchor_offload on a side stream, at the
  location of the camera that triggered it;
* merging -- gs_anchor_merge_plan / _apply (a random 1/(k+1) of the too-fine
  primitives each merged with its k nearest too-fine neighbours, k = 3); the
  optimiser state of the new set is gathered with the kept indices, and the
  merged entries start afresh (moments 0, rate factor 1);
* sliding window -- the merged set becomes the active set the next
  iterations optimise;
* rendering from anchors -- the nearest anchor to a camera, blended with
  the second nearest by w(r) through gs_scale_opacity when their distances
  are similar.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import torch

from . import gsmi


@dataclass
class ActiveSet:
    """The Gaussians being optimised, with their sparse-Adam state."""
    g: gsmi.Gaussians
    m1: gsmi.Gaussians
    m2: gsmi.Gaussians
    rates: torch.Tensor  # (n,) per-Gaussian rate factors
    keyframes: List[int] = field(default_factory=list)

    @property
    def n(self):
        return self.g.n

    def tensors(self):
        return [*self.g.tensors(), *self.m1.tensors(), *self.m2.tensors(), self.rates]

    @staticmethod
    def fresh(g: gsmi.Gaussians, keyframes=()):
        return ActiveSet(g, g.zeros_like(), g.zeros_like(), torch.ones(g.n, dtype=torch.float32, device=g.means.device),
                         list(keyframes))


@dataclass
class Anchor:
    """An active set stored in CPU RAM."""
    location: np.ndarray  # centre of the camera that created it
    n: int
    sh_degree: int
    keyframes: List[int]
    host: torch.Tensor  # pinned uint8 block (gs_anchor_offload layout)
    done: torch.cuda.Event  # the copy has completed once this event has
    _source: Optional[list] = None  # the device tensors, held until the copy is done

    def wait(self):
        self.done.synchronize()
        self._source = None

    def shapes(self):
        n, nb = self.n, (self.sh_degree + 1) ** 2
        one = [(3, n), (3, n), (4, n), (n,), (nb, 3, n)]
        return one * 3 + [(n,)]


class AnchorManager:
    """Anchors of one capture: the trigger, offload, merge and reload."""

    def __init__(self, f: float, tau: float = 1.0, share: float = 0.4, k: int = 3, seed: int = 0,
                 stream: Optional[torch.cuda.Stream] = None):
        self.f, self.tau, self.share, self.k, self.seed = f, tau, share, k, seed
        self.stream = stream or torch.cuda.Stream()
        self.anchors: List[Anchor] = []

    def triggered(self, active: ActiveSet, pose_prev, flags: torch.Tensor) -> bool:
        """The creation test from the previous camera (pose [12] host values):
        writes the too-fine flags and reads back their count (one sync)."""
        count = gsmi.anchor_sizes(active.g, pose_prev, self.f, self.tau, flags=flags)
        return int(count.item()) > self.share * active.n

    def offload(self, active: ActiveSet, location) -> Anchor:
        """Copies the active set to a new anchor on the side stream, ordered
        after the work queued so far on the current stream."""
        src = active.tensors()
        host = torch.empty(gsmi.anchor_host_bytes(src), dtype=torch.uint8, pin_memory=True)
        ready = torch.cuda.Event()
        ready.record()
        done = torch.cuda.Event()
        with torch.cuda.stream(self.stream):
            self.stream.wait_event(ready)
            gsmi.anchor_offload(src, host)
            done.record(self.stream)
        a = Anchor(np.asarray(location, np.float64), active.n, active.g.sh_degree, list(active.keyframes), host, done,
                   src)
        self.anchors.append(a)
        return a

    def merge(self, active: ActiveSet, flags: torch.Tensor, seed: Optional[int] = None) -> ActiveSet:
        """The coarser active set: merged Gaussians, optimiser state gathered
        with the kept indices, merged entries reset (moments 0, rate 1)."""
        plan = gsmi.anchor_merge_plan(active.g, flags, self.k, self.seed if seed is None else seed)
        g, merged = gsmi.anchor_merge_apply(active.g, plan)
        keep = plan.keep_index
        m1 = gsmi.prune_gaussians(active.m1, keep)
        m2 = gsmi.prune_gaussians(active.m2, keep)
        for t in [*m1.tensors(), *m2.tensors()]:
            gsmi.masked_fill(t, merged, 0.0)
        rates = gsmi.gather_planes(active.rates, keep)
        gsmi.masked_fill(rates, merged, 1.0)
        return ActiveSet(g, m1, m2, rates, list(active.keyframes))

    def step(self, active: ActiveSet, pose_prev, location, seed: Optional[int] = None):
        """At a new camera: if the trigger fires from the previous camera,
        store the active set as an anchor and return the merged set (sliding
        window); else the set unchanged.  Returns (active set, anchor or None)."""
        flags = torch.empty(active.n, dtype=torch.int32, device=active.g.means.device)
        if not self.triggered(active, pose_prev, flags):
            return active, None
        anchor = self.offload(active, location)
        new = self.merge(active, flags, seed)
        new.keyframes = []  # the next window's keyframes
        return new, anchor

    def load(self, anchor: Anchor) -> ActiveSet:
        """The anchor's active set back on the device (current stream)."""
        anchor.wait()
        dev = torch.device("cuda", torch.cuda.current_device())
        ts = [torch.empty(s, dtype=torch.float32, device=dev) for s in anchor.shapes()]
        gsmi.anchor_reload(ts, anchor.host)
        g, m1, m2 = (gsmi.Gaussians(*ts[5 * i:5 * i + 5]) for i in range(3))
        return ActiveSet(g, m1, m2, ts[15], list(anchor.keyframes))

    def nearest(self, centre, overlap: float = 0.1):
        """The two anchors nearest to a camera centre and the nearer one's
        blending weight w(r) (1 with a single anchor)."""
        if not self.anchors:
            return None
        d = [float(np.linalg.norm(a.location - np.asarray(centre, np.float64))) for a in self.anchors]
        order = np.argsort(d, kind="stable")
        if len(order) == 1:
            return int(order[0]), None, 1.0
        i1, i2 = int(order[0]), int(order[1])
        if d[i2] == 0.0:
            return i1, i2, 0.5
        return i1, i2, gsmi.anchor_blend_weight(d[i1], d[i2], overlap)
