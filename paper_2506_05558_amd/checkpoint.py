"""Checkpoint and resume of an on-the-fly reconstruction: the active
Gaussians with their sparse-Adam state (both moments, per-Gaussian rate
factors), the camera poses and their optimiser state, and the anchors held
in CPU RAM (section 4.4: an anchor keeps its primitives, their optimisation
state and its keyframes).

Format: one safetensors file (tensor data only, nothing executable), the
tensors under fixed names and the small metadata (SH degree, keyframe
lists, anchor locations, step counters) as JSON in the file's string
metadata.  Device tensors are copied to the host for writing; loading puts
the active set back on the requested device and the anchors back into
pinned host memory in the offload layout, so that they can be reloaded by
gs_anchor_reload as before.  A save followed by a load restores every value
bit for bit.
"""
from __future__ import annotations

import json
from typing import Dict, List, Optional

import numpy as np
import torch
from safetensors.torch import load_file, save_file

FORMAT = "gsmi-checkpoint-1"
_PARTS = ("means", "log_scales", "quats", "opacity_logits", "sh")


def _gauss_dict(prefix: str, g) -> Dict[str, torch.Tensor]:
    return {f"{prefix}.{name}": t.detach().to("cpu").contiguous() for name, t in zip(_PARTS, g.tensors())}


def save(path: str, active=None, poses: Optional[Dict[str, torch.Tensor]] = None, anchors: Optional[list] = None,
         step: int = 0, extra: Optional[dict] = None) -> None:
    """active: an ActiveSet (g, m1, m2, rates, keyframes); poses: named pose
    tensors (e.g. the 6D parameters and their Adam moments); anchors: a list
    of Anchor (their copies must be complete: Anchor.wait is called)."""
    tensors: Dict[str, torch.Tensor] = {}
    meta = dict(format=FORMAT, step=int(step), extra=extra or {})
    if active is not None:
        tensors.update(_gauss_dict("active.g", active.g))
        tensors.update(_gauss_dict("active.m1", active.m1))
        tensors.update(_gauss_dict("active.m2", active.m2))
        tensors["active.rates"] = active.rates.detach().to("cpu").contiguous()
        meta["active"] = dict(sh_degree=active.g.sh_degree, keyframes=[int(k) for k in active.keyframes])
    for name, t in (poses or {}).items():
        tensors[f"poses.{name}"] = t.detach().to("cpu").contiguous()
    meta["poses"] = sorted((poses or {}).keys())
    meta["anchors"] = []
    for i, a in enumerate(anchors or []):
        if a.done is not None:
            a.wait()
        tensors[f"anchor{i}.host"] = a.host.detach().clone()
        meta["anchors"].append(dict(location=[float(x) for x in a.location], n=int(a.n), sh_degree=int(a.sh_degree),
                                    keyframes=[int(k) for k in a.keyframes]))
    save_file(tensors, path, metadata={"gsmi": json.dumps(meta)})


def load(path: str, device="cuda"):
    """Returns dict(active=ActiveSet or None, poses={name: tensor on device},
    anchors=[Anchor], step=int, extra=dict)."""
    from safetensors import safe_open

    with safe_open(path, framework="pt") as f:
        meta = json.loads(f.metadata()["gsmi"])
    if meta.get("format") != FORMAT:
        raise ValueError(f"{path}: not a {FORMAT} file")
    t = load_file(path, device="cpu")
    out = dict(step=meta["step"], extra=meta["extra"], active=None, anchors=[])
    if "active" in meta:
        from . import gsmi
        from .scalable import ActiveSet

        def gauss(prefix):
            return gsmi.Gaussians(*[t[f"{prefix}.{name}"].to(device) for name in _PARTS])

        out["active"] = ActiveSet(gauss("active.g"), gauss("active.m1"), gauss("active.m2"),
                                  t["active.rates"].to(device), list(meta["active"]["keyframes"]))
    out["poses"] = {name: t[f"poses.{name}"].to(device) for name in meta["poses"]}
    if meta["anchors"]:
        from .scalable import Anchor
        for i, am in enumerate(meta["anchors"]):
            host = torch.empty(t[f"anchor{i}.host"].numel(), dtype=torch.uint8, pin_memory=torch.cuda.is_available())
            host.copy_(t[f"anchor{i}.host"])
            done = torch.cuda.Event() if torch.cuda.is_available() else None
            if done is not None:
                done.record()
            out["anchors"].append(Anchor(np.asarray(am["location"], np.float64), am["n"], am["sh_degree"],
                                         list(am["keyframes"]), host, done))
    return out
