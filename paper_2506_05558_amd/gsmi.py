"""Python binding of libgsmi (the HIP rasterizer).  Argument marshalling only.

Every step runs in the library's HIP kernels; torch provides device memory
and the current stream.  Importing this module raises if the library has not
been built: there is no CPU or PyTorch fallback.

Names follow the C ABI in include/gs_api.h: project, bin_sort, render_fwd,
render_bwd, loss_l1, adam_step, pose_from_6d, pose_6d_bwd; ``rasterize`` is
the differentiable composition of the first four as a torch.autograd.Function
returning Gaussian and camera-pose gradients.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgsmi.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                      "(python paper_2506_05558_amd/build.py); there is no fallback")
_lib = C.CDLL(LIB_PATH)

GS_OK, GS_ERR_INVALID_ARG, GS_ERR_CAPACITY, GS_ERR_HIP, GS_ERR_WORKSPACE, GS_ERR_NONFINITE = range(6)
TILE = 16
REC_FLOATS = 16


class GsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"gsmi status {status}: {msg}")
        self.status = status


class _Camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("near_plane", C.c_float), ("bg", C.c_float * 3),
                ("pose", C.c_void_p)]


class _Params(C.Structure):
    _fields_ = [("eps2d", C.c_float), ("alpha_max", C.c_float), ("alpha_min", C.c_float), ("t_min", C.c_float),
                ("guard", C.c_float), ("mip_filter", C.c_int32)]


class _Gauss(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int32), ("means", C.c_void_p), ("log_scales", C.c_void_p),
                ("quats", C.c_void_p), ("opacity_logits", C.c_void_p), ("sh", C.c_void_p), ("filter3d", C.c_void_p)]


class _Proj(C.Structure):
    _fields_ = [("rec", C.c_void_p), ("radius", C.c_void_p), ("tiles_touched", C.c_void_p), ("bin", C.c_void_p)]


class _View(C.Structure):
    _fields_ = [("cam", _Camera), ("proj", _Proj), ("pair_grad", C.c_void_p), ("first_slot", C.c_void_p),
                ("dL_dpose", C.c_void_p), ("dL_dtwist", C.c_void_p)]


class _SpawnParams(C.Structure):
    _fields_ = [("sigma", C.c_float), ("mode", C.c_int32), ("k", C.c_int64), ("seed", C.c_uint64),
                ("opacity", C.c_float), ("min_prob", C.c_float)]


class _AdamGroups(C.Structure):
    _fields_ = [("lr_means", C.c_float), ("lr_log_scales", C.c_float), ("lr_quats", C.c_float),
                ("lr_opacity", C.c_float), ("lr_sh_dc", C.c_float), ("lr_sh_rest", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float), ("step", C.c_int32), ("lr_decay", C.c_float)]


_vp, _i64, _i32, _f, _sz = C.c_void_p, C.c_int64, C.c_int32, C.c_float, C.c_size_t
_P = C.POINTER
_sig = {
    "gs_default_params": (None, [_P(_Params)]),
    "gs_last_error": (C.c_char_p, []),
    "gs_project": (C.c_int, [_P(_Camera), _P(_Params), _P(_Gauss), _P(_Proj), _vp]),
    "gs_bin_sort_workspace": (C.c_int, [_i64, _i64, _P(_sz)]),
    "gs_bin_sort": (C.c_int, [_P(_Camera), _P(_Proj), _i64, _i64, _vp, _sz, _vp, _vp, _vp, _vp, _vp, _P(_i64),
                              _vp]),
    "gs_bin_sort_async": (C.c_int, [_P(_Camera), _P(_Proj), _i64, _i64, _vp, _sz, _vp, _vp, _vp, _vp, _vp, _vp,
                                    _vp]),
    "gs_render_fwd": (C.c_int, [_P(_Camera), _P(_Params), _P(_Proj), _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                _vp]),
    "gs_render_fwd_l1_workspace": (C.c_int, [_i32, _i32, _P(_sz)]),
    "gs_render_fwd_l1": (C.c_int, [_P(_Camera), _P(_Params), _P(_Proj), _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _f,
                                   _vp, _vp, _vp, _sz, _vp]),
    "gs_render_fwd_l1_noalloc": (C.c_int, [_P(_Camera), _P(_Params), _P(_Proj), _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                           _vp, _f, _vp, _vp, _vp]),
    "gs_render_bwd_workspace": (C.c_int, [_i64, _i64, _P(_sz)]),
    "gs_render_bwd": (C.c_int, [_P(_Camera), _P(_Params), _P(_Gauss), _P(_Proj), _vp, _vp, _vp, _vp, _i64, _vp,
                                _vp, _vp, _vp, _vp, _vp, _vp, _P(_Gauss), _vp, _vp, _vp, _sz, _vp]),
    "gs_project_views": (C.c_int, [_i32, _P(_View), _P(_Params), _P(_Gauss), _vp]),
    "gs_render_bwd_pairs": (C.c_int, [_P(_Camera), _P(_Params), _P(_Proj), _vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp,
                                      _vp, _vp, _vp, _vp, _vp]),
    "gs_project_bwd_views_workspace": (C.c_int, [_i64, _i32, _P(_sz)]),
    "gs_project_bwd_views": (C.c_int, [_i32, _P(_View), _P(_Params), _P(_Gauss), _P(_Gauss), _vp, _sz, _vp]),
    "gs_project_bwd_views_store": (C.c_int, [_i32, _P(_View), _P(_Params), _P(_Gauss), _P(_Gauss), _vp, _sz, _vp,
                                             _vp]),
    "gs_project_bwd_views_adam": (C.c_int, [_i32, _P(_View), _P(_Params), _P(_Gauss), _P(_Gauss), _P(_Gauss), _vp,
                                            _P(_AdamGroups), _P(_Gauss), _vp, _sz, _vp, _vp]),
    "gs_loss_workspace": (C.c_int, [_i64, _P(_sz)]),
    "gs_loss_l1": (C.c_int, [_vp, _vp, _i64, _f, _vp, _vp, _vp, _sz, _vp]),
    "gs_psnr_workspace": (C.c_int, [_i64, _P(_sz)]),
    "gs_psnr": (C.c_int, [_vp, _vp, _i64, _f, _vp, _vp, _sz, _vp]),
    "gs_count_nonfinite": (C.c_int, [_vp, _i64, _P(_i64), _vp]),
    "gs_adam_step": (C.c_int, [_vp, _vp, _vp, _vp, _i64, _f, _f, _f, _f, _i32, _vp, _vp, _i64, _vp]),
    "gs_lr_decay": (C.c_int, [_vp, _vp, _i64, _f, _vp]),
    "gs_downsample": (C.c_int, [_vp, _i32, _i32, _i32, _i32, _vp, _vp]),
    "gs_camera_level": (C.c_int, [_P(_Camera), _i32, _P(_Camera)]),
    "gs_prune_workspace": (C.c_int, [_i64, _P(_sz)]),
    "gs_prune_opacity": (C.c_int, [_vp, _i64, _f, _vp, _P(_i64), _vp, _sz, _vp]),
    "gs_gather_planes": (C.c_int, [_vp, _i64, _i32, _vp, _i64, _vp, _vp]),
    "gs_pose_from_6d": (C.c_int, [_vp, _vp, _i32, _vp]),
    "gs_pose_6d_bwd": (C.c_int, [_vp, _vp, _vp, _i32, _vp]),
    "gs_zero": (C.c_int, [_vp, _sz, _vp]),
    "gs_mark_visible": (C.c_int, [_vp, _i64, _vp, _vp]),
    "gs_default_spawn_params": (None, [_P(_SpawnParams)]),
    "gs_spawn_log_taps": (C.c_int, [_f, _P(C.c_float), _P(_i32)]),
    "gs_spawn_probability": (C.c_int, [_P(_Camera), _vp, _vp, _P(_SpawnParams), _vp, _vp, _vp]),
    "gs_spawn_select_workspace": (C.c_int, [_i32, _i32, _P(_sz)]),
    "gs_spawn_select": (C.c_int, [_P(_Camera), _vp, _P(_SpawnParams), _i64, _vp, _P(_i64), _vp, _sz, _vp]),
    "gs_spawn_rule": (C.c_int, [_P(_Camera), _vp, _vp, _vp, _vp, _i64, _P(_SpawnParams), _P(_Gauss), _i64,
                                _vp]),
    "gs_mlp_packed_bytes": (C.c_size_t, []),
    "gs_mlp_pack_bf16": (C.c_int, [_vp, _vp, _vp]),
    "gs_mlp_features": (C.c_int, [_P(_Camera), _vp, _vp, _vp, _i64, _vp, _vp]),
    "gs_mlp_forward_bf16": (C.c_int, [_vp, _vp, _i64, _vp, _vp]),
    "gs_spawn_mlp": (C.c_int, [_P(_Camera), _vp, _vp, _vp, _i64, _vp, _P(_Gauss), _i64, _vp]),
    "gs_mlp_train_workspace": (C.c_int, [_i64, _P(_sz)]),
    "gs_mlp_train_step": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _i64, _f, _f, _f, _f, _i32, _vp, _vp, _vp, _sz,
                                    _vp]),
    "gs_spawn_init_workspace": (C.c_int, [_i32, _i32, _i64, _P(_sz)]),
    "gs_spawn_init": (C.c_int, [_P(_Camera), _vp, _vp, _vp, _P(_SpawnParams), _vp, _P(_Gauss), _i64, _P(_i64), _vp,
                                _sz, _vp]),
    "gs_guided_depth": (C.c_int, [_i32, _i32, _i32, _f, _f, _f, _f, _vp, _i32, _P(_vp), _P(C.c_float), _vp, _i32, _f,
                                  _vp, _vp, _vp, _vp]),
    "gs_anchor_sizes": (C.c_int, [_vp, _vp, _i64, _P(C.c_float), _f, _f, _vp, _vp, _vp]),
    "gs_anchor_blend_weight": (C.c_int, [_f, _f, _f, _P(C.c_float)]),
    "gs_scale_opacity": (C.c_int, [_vp, _i64, _f, _vp, _vp]),
    "gs_anchor_merge_workspace": (C.c_int, [_i64, _P(_sz)]),
    "gs_anchor_merge_plan": (C.c_int, [_P(_Gauss), _vp, _i32, C.c_uint64, _vp, _vp, _vp, _vp, _vp, _P(_i64), _vp,
                                       _sz, _vp]),
    "gs_anchor_merge_apply": (C.c_int, [_P(_Gauss), _vp, _vp, _vp, _vp, _vp, _i32, _P(_Gauss), _vp, _vp]),
    "gs_masked_fill": (C.c_int, [_vp, _i64, _i32, _vp, _f, _vp]),
    "gs_pose_ransac_workspace": (C.c_int, [_i32, _P(_sz)]),
    "gs_pose_ransac": (C.c_int, [_vp, _vp, _i64, _f, _f, _f, _f, _P(C.c_double), _i32, _i32, _i32, _f, _i32, _f,
                                 C.c_uint64, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "gs_ba_bootstrap_workspace": (C.c_int, [_i32, _i32, _P(_sz)]),
    "gs_ba_bootstrap": (C.c_int, [_vp, _i32, _i32, _i32, _i32, _i32, _i32, _f, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "gs_anchor_host_bytes": (C.c_size_t, [_i32, _P(_sz)]),
    "gs_anchor_offload": (C.c_int, [_i32, _P(_vp), _P(_sz), _vp, _vp]),
    "gs_anchor_reload": (C.c_int, [_i32, _P(_vp), _P(_sz), _vp, _vp]),
    "gs_cells_assign": (C.c_int, [_vp, _i64, _vp, _i32, _vp, _vp]),
    "gs_cells_kmeans_workspace": (C.c_int, [_i64, _i32, _P(_sz)]),
    "gs_cells_kmeans": (C.c_int, [_vp, _i64, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "gs_cells_spheres_workspace": (C.c_int, [_i64, _i32, _P(_sz)]),
    "gs_cells_spheres": (C.c_int, [_vp, _vp, _i64, _vp, _vp, _i32, _f, _vp, _vp, _sz, _vp]),
    "gs_cells_visible": (C.c_int, [_vp, _vp, _i32, _P(_Camera), _f, _vp, _vp]),
    "gs_filter3d_update": (C.c_int, [_vp, _i64, _i32, _P(_Camera), _f, _f, _vp, _vp, _vp]),
    "gs_copy_rows": (C.c_int, [_vp, _sz, _vp, _sz, _sz, _sz, _vp]),
    "gs_fill_f32": (C.c_int, [_vp, _i64, _f, _vp]),
    "gs_probe_copy": (C.c_int, [_vp, _vp, _sz, _vp]),
    "gs_probe_valu": (C.c_int, [_i32, _i32, _i32, _vp, _vp]),
    "gs_profile_enable": (None, [C.c_int]),
    "gs_profile_reset": (None, []),
    "gs_profile_select": (None, [C.c_char_p]),
    "gs_profile_read": (C.c_int, [C.c_char_p, _P(C.c_double), _P(_i64)]),
}
for _name, (_res, _args) in _sig.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args


def exported_symbols():
    return sorted(_sig)


def _check(status):
    if status != GS_OK:
        raise GsError(status, _lib.gs_last_error().decode())


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else t.data_ptr()


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _require(t: torch.Tensor, dtype, shape, name):
    if t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous() or not t.is_cuda:
        raise ValueError(f"{name}: expected contiguous CUDA {dtype} {tuple(shape)}, got {t.dtype} "
                         f"{tuple(t.shape)} contiguous={t.is_contiguous()} device={t.device}")


@dataclass
class Params:
    eps2d: float = 0.3
    alpha_max: float = 0.99
    alpha_min: float = 1.0 / 255.0
    t_min: float = 1e-4
    guard: float = 1.3
    mip_filter: int = 0  # 1: eps2d is a screen-space filter with opacity compensation

    def c(self):
        return _Params(self.eps2d, self.alpha_max, self.alpha_min, self.t_min, self.guard, int(self.mip_filter))


@dataclass
class Camera:
    """Pinhole intrinsics (host) and a world->camera pose [12] on the device."""
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    pose: torch.Tensor  # float32 [12] = R row-major (9), t (3)
    near_plane: float = 0.2
    bg: tuple = (0.0, 0.0, 0.0)

    @property
    def tiles_x(self):
        return (self.width + TILE - 1) // TILE

    @property
    def tiles_y(self):
        return (self.height + TILE - 1) // TILE

    def c(self):
        _require(self.pose, torch.float32, (12,), "camera pose")
        return _Camera(self.width, self.height, self.fx, self.fy, self.cx, self.cy, self.near_plane,
                       (C.c_float * 3)(*self.bg), self.pose.data_ptr())


@dataclass
class Gaussians:
    """SoA parameter planes on the device (float32)."""
    means: torch.Tensor  # (3, N)
    log_scales: torch.Tensor  # (3, N)
    quats: torch.Tensor  # (4, N)
    opacity_logits: torch.Tensor  # (N,)
    sh: torch.Tensor  # ((d+1)^2, 3, N)
    filter3d: Optional[torch.Tensor] = None  # (N,) 3D smoothing-filter variance, or None

    @property
    def n(self):
        return int(self.means.shape[1])

    @property
    def sh_degree(self):
        return int(round(self.sh.shape[0] ** 0.5)) - 1

    def tensors(self):
        return [self.means, self.log_scales, self.quats, self.opacity_logits, self.sh]

    def c(self):
        n, d = self.n, self.sh_degree
        _require(self.means, torch.float32, (3, n), "means")
        _require(self.log_scales, torch.float32, (3, n), "log_scales")
        _require(self.quats, torch.float32, (4, n), "quats")
        _require(self.opacity_logits, torch.float32, (n,), "opacity_logits")
        _require(self.sh, torch.float32, ((d + 1) ** 2, 3, n), "sh")
        if self.filter3d is not None:
            _require(self.filter3d, torch.float32, (n,), "filter3d")
        return _Gauss(n, d, *[t.data_ptr() for t in self.tensors()], _ptr(self.filter3d))

    def zeros_like(self):
        return Gaussians(*[torch.zeros_like(t) for t in self.tensors()])

    @staticmethod
    def from_arrays(d: dict, device="cuda"):
        f = lambda a: torch.as_tensor(a, dtype=torch.float32).contiguous().to(device)
        return Gaussians(f(d["means"]), f(d["log_scales"]), f(d["quats"]), f(d["opacity_logits"]), f(d["sh"]))


@dataclass
class Projected:
    rec: torch.Tensor  # (N, 16) render records
    radius: torch.Tensor  # (2, N) int32 half-widths (rx, ry) of the support rect
    tiles_touched: torch.Tensor  # (N,) int32
    bin: Optional[torch.Tensor] = None  # (N, 4) int32: the binning's inputs (depth bits, tile rect), or None

    def c(self):
        return _Proj(self.rec.data_ptr(), self.radius.data_ptr(), self.tiles_touched.data_ptr(), _ptr(self.bin))


def default_params() -> Params:
    p = _Params()
    _lib.gs_default_params(C.byref(p))
    return Params(p.eps2d, p.alpha_max, p.alpha_min, p.t_min, p.guard, p.mip_filter)


def alloc_projected(n: int, device="cuda", bin: bool = True) -> Projected:
    """Output planes of a projection; with bin, also the binning's inputs
    (16 B per Gaussian), which spare the binning a read of the records."""
    return Projected(torch.empty((n, REC_FLOATS), dtype=torch.float32, device=device),
                     torch.empty((2, n), dtype=torch.int32, device=device),
                     torch.empty(n, dtype=torch.int32, device=device),
                     torch.empty((n, 4), dtype=torch.int32, device=device) if bin else None)


def project(cam: Camera, g: Gaussians, params: Params = Params(), out: Optional[Projected] = None) -> Projected:
    n = g.n
    dev = g.means.device
    if out is None:
        out = alloc_projected(n, dev)
    _check(_lib.gs_project(C.byref(cam.c()), C.byref(params.c()), C.byref(g.c()), C.byref(out.c()), _stream()))
    return out


@dataclass
class Binned:
    tile_ids: torch.Tensor  # (capacity,) uint32 as int32: tile of each sorted pair
    values: torch.Tensor  # (capacity,) uint32 as int32: Gaussian of each sorted pair
    slots: torch.Tensor  # (capacity,) uint32 as int32: emission index of each sorted pair
    ranges: torch.Tensor  # (T, 2) uint32 as int32
    first_slot: torch.Tensor  # (N,) uint32 as int32: first slot of each visible Gaussian
    n_instances: int


class BinSorter:
    """Holds the list buffers and workspace between calls; grows them on
    GS_ERR_CAPACITY (the library reports the required size)."""

    def __init__(self, capacity: int = 0, growth: float = 1.25):
        self.capacity = int(capacity)
        self.growth = growth
        self._bufs = None
        self._key = None

    def _alloc(self, n, T, dev):
        need = C.c_size_t()
        _check(_lib.gs_bin_sort_workspace(n, self.capacity, C.byref(need)))
        cap = max(self.capacity, 1)
        self._bufs = dict(ws=torch.empty(max(int(need.value), 1), dtype=torch.uint8, device=dev),
                          tile_ids=torch.empty(cap, dtype=torch.int32, device=dev),
                          values=torch.empty(cap, dtype=torch.int32, device=dev),
                          slots=torch.empty(cap, dtype=torch.int32, device=dev),
                          ranges=torch.empty((T, 2), dtype=torch.int32, device=dev),
                          first_slot=torch.empty(max(n, 1), dtype=torch.int32, device=dev))
        self._key = (n, T, self.capacity)

    def __call__(self, cam: Camera, proj: Projected, first_slot: Optional[torch.Tensor] = None) -> Binned:
        """first_slot: an (N,) int32 tensor of the caller's to receive the first
        slots (kept per view by a multi-view adjoint); default: a held buffer."""
        n = int(proj.tiles_touched.shape[0])
        T = cam.tiles_x * cam.tiles_y
        dev = proj.rec.device
        for _ in range(2):
            if self._key != (n, T, self.capacity) or self._bufs is None:
                self._alloc(n, T, dev)
            b = self._bufs
            fs = b["first_slot"] if first_slot is None else first_slot
            if first_slot is not None:
                _require(first_slot, torch.int32, (n,), "first_slot")
            m = C.c_int64()
            st = _lib.gs_bin_sort(C.byref(cam.c()), C.byref(proj.c()), n, self.capacity, b["ws"].data_ptr(),
                                  b["ws"].numel(), b["tile_ids"].data_ptr(), b["values"].data_ptr(),
                                  b["slots"].data_ptr(), b["ranges"].data_ptr(), fs.data_ptr(), C.byref(m),
                                  _stream())
            if st == GS_ERR_CAPACITY:
                self.capacity = int(m.value * self.growth) + 1024
                continue
            _check(st)
            return Binned(b["tile_ids"], b["values"], b["slots"], b["ranges"], fs, int(m.value))
        raise GsError(GS_ERR_CAPACITY, "bin_sort: capacity did not converge")


    def reserve(self, n: int, tiles: int, device) -> None:
        """Allocates the buffers for n Gaussians and `tiles` tiles at the
        current capacity, so that later calls (on any stream) allocate nothing."""
        if self._key != (n, tiles, self.capacity) or self._bufs is None:
            self._alloc(n, tiles, device)

    def sort_async(self, cam: Camera, proj: Projected, n_dev: torch.Tensor,
                   first_slot: Optional[torch.Tensor] = None) -> Binned:
        """gs_bin_sort_async: no host synchronisation; the pair count goes to
        n_dev (a one-element int32 device tensor).  The lists are valid only if
        n_dev <= self.capacity, which the caller checks later; n_instances of
        the result is the capacity (an upper bound)."""
        n = int(proj.tiles_touched.shape[0])
        T = cam.tiles_x * cam.tiles_y
        if self._key != (n, T, self.capacity) or self._bufs is None:
            self._alloc(n, T, proj.rec.device)
        b = self._bufs
        fs = b["first_slot"] if first_slot is None else first_slot
        _require(n_dev, torch.int32, (1,), "n_dev")
        _check(_lib.gs_bin_sort_async(C.byref(cam.c()), C.byref(proj.c()), n, self.capacity, b["ws"].data_ptr(),
                                      b["ws"].numel(), b["tile_ids"].data_ptr(), b["values"].data_ptr(),
                                      b["slots"].data_ptr(), b["ranges"].data_ptr(), fs.data_ptr(),
                                      n_dev.data_ptr(), _stream()))
        return Binned(b["tile_ids"], b["values"], b["slots"], b["ranges"], fs, self.capacity)


def bin_sort(cam: Camera, proj: Projected, sorter: Optional[BinSorter] = None) -> Binned:
    return (sorter or BinSorter())(cam, proj)


@dataclass
class Frame:
    image: torch.Tensor  # (3, H, W)
    depth: torch.Tensor  # (H, W)
    alpha: torch.Tensor  # (H, W)
    final_t: torch.Tensor  # (H, W)
    n_contrib: torch.Tensor  # (H, W) int32
    stats: Optional[torch.Tensor] = None  # (4, H, W) int32: tile entries to the stop, evaluated, support, composited


def render_fwd(cam: Camera, proj: Projected, binned: Binned, params: Params = Params(),
               count_pairs: bool = False, out: Optional[Frame] = None) -> Frame:
    H, W = cam.height, cam.width
    dev = proj.rec.device
    if out is None:
        out = Frame(torch.empty((3, H, W), dtype=torch.float32, device=dev),
                    torch.empty((H, W), dtype=torch.float32, device=dev),
                    torch.empty((H, W), dtype=torch.float32, device=dev),
                    torch.empty((H, W), dtype=torch.float32, device=dev),
                    torch.empty((H, W), dtype=torch.int32, device=dev),
                    torch.empty((4, H, W), dtype=torch.int32, device=dev) if count_pairs else None)
    _check(_lib.gs_render_fwd(C.byref(cam.c()), C.byref(params.c()), C.byref(proj.c()), binned.values.data_ptr(),
                              binned.ranges.data_ptr(), out.image.data_ptr(), out.depth.data_ptr(),
                              out.alpha.data_ptr(), out.final_t.data_ptr(), out.n_contrib.data_ptr(),
                              _ptr(out.stats), _stream()))
    return out


def render_fwd_l1_workspace(width: int, height: int) -> int:
    need = C.c_size_t()
    _check(_lib.gs_render_fwd_l1_workspace(width, height, C.byref(need)))
    return int(need.value)


def render_fwd_l1(cam: Camera, proj: Projected, binned: Binned, target: torch.Tensor, grad_scale: float,
                  dL_dimage: torch.Tensor, sums: torch.Tensor, ws: Optional[torch.Tensor] = None,
                  params: Params = Params(), out: Optional[Frame] = None) -> Frame:
    """gs_render_fwd_l1: the forward with the L1 loss fused in; dL_dimage
    (3, H, W) float32 and sums (2,) float64 are written.  ws: a uint8 device
    tensor of at least render_fwd_l1_workspace(W, H) bytes (new if None)."""
    H, W = cam.height, cam.width
    dev = proj.rec.device
    _require(target, torch.float32, (3, H, W), "target")
    _require(dL_dimage, torch.float32, (3, H, W), "dL_dimage")
    _require(sums, torch.float64, (2,), "sums")
    if out is None:
        out = Frame(torch.empty((3, H, W), dtype=torch.float32, device=dev),
                    torch.empty((H, W), dtype=torch.float32, device=dev),
                    torch.empty((H, W), dtype=torch.float32, device=dev),
                    torch.empty((H, W), dtype=torch.float32, device=dev),
                    torch.empty((H, W), dtype=torch.int32, device=dev))
    need = render_fwd_l1_workspace(W, H)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
    _check(_lib.gs_render_fwd_l1(C.byref(cam.c()), C.byref(params.c()), C.byref(proj.c()), binned.values.data_ptr(),
                                 binned.ranges.data_ptr(), out.image.data_ptr(), out.depth.data_ptr(),
                                 out.alpha.data_ptr(), out.final_t.data_ptr(), out.n_contrib.data_ptr(),
                                 target.data_ptr(), grad_scale, dL_dimage.data_ptr(), sums.data_ptr(), ws.data_ptr(),
                                 ws.numel(), _stream()))
    return out


def render_fwd_l1_noalloc(cam: Camera, proj: Projected, binned: Binned, target: torch.Tensor, grad_scale: float,
                          dL_dimage: torch.Tensor, sums: torch.Tensor, out: Frame, params: Params = Params()) -> Frame:
    """gs_render_fwd_l1_noalloc: render_fwd_l1 with the library's fixed
    scratch instead of a workspace; every output buffer is the caller's
    (out, dL_dimage, sums), so the call allocates nothing."""
    H, W = cam.height, cam.width
    _require(target, torch.float32, (3, H, W), "target")
    _require(dL_dimage, torch.float32, (3, H, W), "dL_dimage")
    _require(sums, torch.float64, (2,), "sums")
    _require(out.image, torch.float32, (3, H, W), "image")
    for t, nm in ((out.depth, "depth"), (out.alpha, "alpha"), (out.final_t, "final_t")):
        _require(t, torch.float32, (H, W), nm)
    _require(out.n_contrib, torch.int32, (H, W), "n_contrib")
    _check(_lib.gs_render_fwd_l1_noalloc(C.byref(cam.c()), C.byref(params.c()), C.byref(proj.c()),
                                         binned.values.data_ptr(), binned.ranges.data_ptr(), out.image.data_ptr(),
                                         out.depth.data_ptr(), out.alpha.data_ptr(), out.final_t.data_ptr(),
                                         out.n_contrib.data_ptr(), target.data_ptr(), grad_scale,
                                         dL_dimage.data_ptr(), sums.data_ptr(), _stream()))
    return out


def render_bwd_workspace(n: int, n_instances: int) -> int:
    need = C.c_size_t()
    _check(_lib.gs_render_bwd_workspace(n, n_instances, C.byref(need)))
    return int(need.value)


def render_bwd(cam: Camera, g: Gaussians, proj: Projected, binned: Binned, frame: Frame,
               dL_dimage: torch.Tensor, dL_ddepth: Optional[torch.Tensor] = None,
               dL_dalpha: Optional[torch.Tensor] = None, grads: Optional[Gaussians] = None,
               dL_dpose: Optional[torch.Tensor] = None, dL_dtwist: Optional[torch.Tensor] = None,
               params: Params = Params(), ws: Optional[torch.Tensor] = None):
    """Accumulates into grads (new zeros if None) and the optional float64
    dL_dpose [12] / dL_dtwist [6]; returns grads.  ws, if given, is grown
    by reallocation only when too small (pass a large one to avoid it)."""
    H, W = cam.height, cam.width
    _require(dL_dimage, torch.float32, (3, H, W), "dL_dimage")
    if dL_ddepth is not None:
        _require(dL_ddepth, torch.float32, (H, W), "dL_ddepth")
    if dL_dalpha is not None:
        _require(dL_dalpha, torch.float32, (H, W), "dL_dalpha")
    if grads is None:
        grads = g.zeros_like()
    need = render_bwd_workspace(g.n, binned.n_instances)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=g.means.device)
    for t, nm, k in ((dL_dpose, "dL_dpose", 12), (dL_dtwist, "dL_dtwist", 6)):
        if t is not None:
            _require(t, torch.float64, (k,), nm)
    _check(_lib.gs_render_bwd(C.byref(cam.c()), C.byref(params.c()), C.byref(g.c()), C.byref(proj.c()),
                              binned.values.data_ptr(), binned.slots.data_ptr(), binned.ranges.data_ptr(),
                              binned.first_slot.data_ptr(), binned.n_instances, frame.image.data_ptr(),
                              frame.depth.data_ptr(), frame.final_t.data_ptr(), frame.n_contrib.data_ptr(),
                              dL_dimage.data_ptr(), _ptr(dL_ddepth), _ptr(dL_dalpha), C.byref(grads.c()),
                              _ptr(dL_dpose), _ptr(dL_dtwist), ws.data_ptr(), ws.numel(), _stream()))
    return grads


# -------------------------------------------------------- several views
@dataclass
class View:
    """One view of a window: its camera, its projection buffers, and the
    adjoint's per-view inputs (pair gradients, first slots) and outputs."""
    cam: Camera
    proj: Projected
    pair_grad: Optional[torch.Tensor] = None  # (capacity, 12) float32
    first_slot: Optional[torch.Tensor] = None  # (N,) int32
    dL_dpose: Optional[torch.Tensor] = None  # (12,) float64
    dL_dtwist: Optional[torch.Tensor] = None  # (6,) float64

    def c(self):
        return _View(self.cam.c(), self.proj.c(), _ptr(self.pair_grad), _ptr(self.first_slot), _ptr(self.dL_dpose),
                     _ptr(self.dL_dtwist))


def _views_c(views):
    arr = (_View * max(len(views), 1))()
    for k, v in enumerate(views):
        arr[k] = v.c()
    return arr


def project_views(views, g: Gaussians, params: Params = Params()):
    """Projects g into every view's proj buffers (parameters read once)."""
    _check(_lib.gs_project_views(len(views), _views_c(views), C.byref(params.c()), C.byref(g.c()), _stream()))


def render_bwd_pairs(cam: Camera, proj: Projected, binned: Binned, frame: Frame, dL_dimage: torch.Tensor,
                     pair_grad: torch.Tensor, dL_ddepth: Optional[torch.Tensor] = None,
                     dL_dalpha: Optional[torch.Tensor] = None, params: Params = Params()):
    """The compositing adjoint of one view into pair_grad (capacity, 12)."""
    H, W = cam.height, cam.width
    _require(dL_dimage, torch.float32, (3, H, W), "dL_dimage")
    if pair_grad.shape[0] < binned.n_instances or pair_grad.dtype != torch.float32:
        raise ValueError("pair_grad: need float32 (>= n_instances, 12)")
    _check(_lib.gs_render_bwd_pairs(C.byref(cam.c()), C.byref(params.c()), C.byref(proj.c()),
                                    binned.values.data_ptr(), binned.slots.data_ptr(), binned.ranges.data_ptr(),
                                    binned.n_instances, frame.image.data_ptr(), frame.depth.data_ptr(),
                                    frame.final_t.data_ptr(), frame.n_contrib.data_ptr(), dL_dimage.data_ptr(),
                                    _ptr(dL_ddepth), _ptr(dL_dalpha), pair_grad.data_ptr(), _stream()))


def project_bwd_views_workspace(n: int, n_views: int) -> int:
    need = C.c_size_t()
    _check(_lib.gs_project_bwd_views_workspace(n, n_views, C.byref(need)))
    return int(need.value)


def project_bwd_views(views, g: Gaussians, grads: Gaussians, params: Params = Params(),
                      ws: Optional[torch.Tensor] = None, store: bool = False,
                      visible: Optional[torch.Tensor] = None):
    """Chains every view's pair gradients to the parameters (summed over the
    views into grads: added, or with store=True written, no clearing needed)
    and to each view's pose gradient.  With store=True, visible (int32 [n])
    is overwritten with the set the sparse step updates (some view's tile
    count positive)."""
    need = project_bwd_views_workspace(g.n, len(views))
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=g.means.device)
    args = (len(views), _views_c(views), C.byref(params.c()), C.byref(g.c()), C.byref(grads.c()), ws.data_ptr(),
            ws.numel())
    if store:
        if visible is not None:
            _require(visible, torch.int32, (g.n,), "visible")
        _check(_lib.gs_project_bwd_views_store(*args, _ptr(visible), _stream()))
    else:
        if visible is not None:
            raise ValueError("project_bwd_views: the visible set is written by the store form only")
        _check(_lib.gs_project_bwd_views(*args, _stream()))
    return grads


@dataclass
class AdamGroups:
    """Rates per parameter group and Adam's constants for
    project_bwd_views_adam (gs_adam_groups)."""
    lr_means: float
    lr_log_scales: float
    lr_quats: float
    lr_opacity: float
    lr_sh_dc: float
    lr_sh_rest: float
    step: int
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-15
    lr_decay: float = 1.0

    def c(self):
        return _AdamGroups(self.lr_means, self.lr_log_scales, self.lr_quats, self.lr_opacity, self.lr_sh_dc,
                           self.lr_sh_rest, self.beta1, self.beta2, self.eps, int(self.step), self.lr_decay)


def project_bwd_views_adam(views, g: Gaussians, grads: Gaussians, m1: Gaussians, m2: Gaussians, opt: AdamGroups,
                           visible: torch.Tensor, lr_scale: Optional[torch.Tensor] = None,
                           params: Params = Params(), ws: Optional[torch.Tensor] = None):
    """The store-form adjoint of the views followed by the sparse Adam step on
    every parameter group and the rate decay (gs_project_bwd_views_adam): g,
    m1, m2, lr_scale and visible are updated in place; grads is scratch."""
    _require(visible, torch.int32, (g.n,), "visible")
    if lr_scale is not None:
        _require(lr_scale, torch.float32, (g.n,), "lr_scale")
    need = project_bwd_views_workspace(g.n, len(views))
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=g.means.device)
    _check(_lib.gs_project_bwd_views_adam(len(views), _views_c(views), C.byref(params.c()), C.byref(g.c()),
                                          C.byref(m1.c()), C.byref(m2.c()), _ptr(lr_scale), C.byref(opt.c()),
                                          C.byref(grads.c()), ws.data_ptr(), ws.numel(), visible.data_ptr(),
                                          _stream()))


def loss_l1(image: torch.Tensor, target: torch.Tensor, grad_scale: Optional[float] = None,
            dL_dimage: Optional[torch.Tensor] = None, sums: Optional[torch.Tensor] = None,
            ws: Optional[torch.Tensor] = None):
    """sums[0] = sum |image - target|, sums[1] = sum of squares (float64,
    device); dL_dimage = grad_scale * sign(image - target)."""
    count = image.numel()
    if grad_scale is None:
        grad_scale = 1.0 / max(count, 1)
    if sums is None:
        sums = torch.empty(2, dtype=torch.float64, device=image.device)
    need = C.c_size_t()
    _check(_lib.gs_loss_workspace(count, C.byref(need)))
    if ws is None or ws.numel() < need.value:
        ws = torch.empty(int(need.value), dtype=torch.uint8, device=image.device)
    _check(_lib.gs_loss_l1(image.data_ptr(), target.data_ptr(), count, grad_scale, _ptr(dL_dimage),
                           sums.data_ptr(), ws.data_ptr(), ws.numel(), _stream()))
    return sums


def psnr(image: torch.Tensor, target: torch.Tensor, peak: float = 1.0, out: Optional[torch.Tensor] = None,
         ws: Optional[torch.Tensor] = None):
    """out[0] = PSNR in dB (+inf for equal images), out[1] = MSE (float64,
    device, binary64 sums)."""
    count = image.numel()
    if out is None:
        out = torch.empty(2, dtype=torch.float64, device=image.device)
    need = C.c_size_t()
    _check(_lib.gs_psnr_workspace(count, C.byref(need)))
    if ws is None or ws.numel() < need.value:
        ws = torch.empty(int(need.value), dtype=torch.uint8, device=image.device)
    _check(_lib.gs_psnr(image.data_ptr(), target.data_ptr(), count, peak, out.data_ptr(), ws.data_ptr(),
                        ws.numel(), _stream()))
    return out


def count_nonfinite(x: torch.Tensor) -> int:
    """Number of NaN and infinite values in a float32 tensor (synchronises)."""
    assert x.dtype == torch.float32 and x.is_contiguous()
    n = C.c_int64()
    _check(_lib.gs_count_nonfinite(x.data_ptr(), x.numel(), C.byref(n), _stream()))
    return int(n.value)


def adam_step(param, grad, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-15, visible=None, n_stride=0,
              lr_scale=None):
    _check(_lib.gs_adam_step(param.data_ptr(), grad.data_ptr(), m.data_ptr(), v.data_ptr(), param.numel(), lr,
                             beta1, beta2, eps, step, _ptr(visible), _ptr(lr_scale), n_stride, _stream()))


def lr_decay(lr_scale: torch.Tensor, decay: float, visible: Optional[torch.Tensor] = None):
    """lr_scale[i] *= decay for the Gaussians a sparse step processed."""
    _check(_lib.gs_lr_decay(lr_scale.data_ptr(), _ptr(visible), lr_scale.numel(), decay, _stream()))


# ------------------------------------------------------ multi-scale training
def coarse_level(iteration: int, start_level: int = 3, every: int = 5) -> int:
    """Downsampling level of a newly added image at a joint iteration: 2^3
    first, one level less every five iterations (section 4.3)."""
    return max(0, start_level - iteration // every)


def downsample(image: torch.Tensor, level: int, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """[C][H][W] -> [C][H >> level][W >> level] box filter."""
    if image.dim() != 3:
        raise ValueError(f"image: expected [C][H][W], got {tuple(image.shape)}")
    _require(image, torch.float32, image.shape, "image")
    c, h, w = image.shape
    if out is None:
        out = torch.empty((c, h >> level, w >> level), dtype=torch.float32, device=image.device)
    _check(_lib.gs_downsample(image.data_ptr(), c, w, h, level, out.data_ptr(), _stream()))
    return out


def camera_level(cam: Camera, level: int) -> Camera:
    """The camera of the 2^level-downsampled image (same pose tensor)."""
    out = _Camera()
    _check(_lib.gs_camera_level(C.byref(cam.c()), level, C.byref(out)))
    return Camera(out.width, out.height, out.fx, out.fy, out.cx, out.cy, cam.pose, cam.near_plane, cam.bg)


def prune_opacity(opacity_logits: torch.Tensor, min_opacity: float = 0.005,
                  keep_index: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Ascending int32 indices of the Gaussians opacity culling keeps."""
    _require(opacity_logits, torch.float32, (opacity_logits.numel(),), "opacity_logits")
    n = opacity_logits.numel()
    need = C.c_size_t()
    _check(_lib.gs_prune_workspace(n, C.byref(need)))
    if ws is None or ws.numel() < need.value:
        ws = torch.empty(max(int(need.value), 1), dtype=torch.uint8, device=opacity_logits.device)
    if keep_index is None:
        keep_index = torch.empty(max(n, 1), dtype=torch.int32, device=opacity_logits.device)
    kept = C.c_int64()
    _check(_lib.gs_prune_opacity(opacity_logits.data_ptr(), n, min_opacity, keep_index.data_ptr(), C.byref(kept),
                                 ws.data_ptr(), ws.numel(), _stream()))
    return keep_index[:kept.value]


def gather_planes(src: torch.Tensor, index: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """src [..., n] -> [..., m]: column j is column index[j] (all leading
    dimensions are planes)."""
    _require(src, torch.float32, src.shape, "src")
    _require(index, torch.int32, (index.numel(),), "index")
    n, m = src.shape[-1], index.numel()
    planes = src.numel() // max(n, 1)
    if out is None:
        out = torch.empty((*src.shape[:-1], m), dtype=torch.float32, device=src.device)
    _check(_lib.gs_gather_planes(src.data_ptr(), n, planes, index.data_ptr(), m, out.data_ptr(), _stream()))
    return out


def prune_gaussians(g: Gaussians, keep_index: torch.Tensor) -> Gaussians:
    """The kept Gaussians' parameter planes (new tensors, same order)."""
    return Gaussians(*(gather_planes(t, keep_index) for t in g.tensors()))


def pose_from_6d(x: torch.Tensor, pose: torch.Tensor):
    _check(_lib.gs_pose_from_6d(x.data_ptr(), pose.data_ptr(), x.shape[0], _stream()))


def pose_6d_bwd(x: torch.Tensor, dL_dpose: torch.Tensor, dL_dx: torch.Tensor):
    _check(_lib.gs_pose_6d_bwd(x.data_ptr(), dL_dpose.data_ptr(), dL_dx.data_ptr(), x.shape[0], _stream()))


def zero_(t: torch.Tensor):
    """Zero a contiguous device tensor with the library's fill kernel."""
    _check(_lib.gs_zero(t.data_ptr(), t.numel() * t.element_size(), _stream()))
    return t


def mark_visible(proj: Projected, mask: torch.Tensor):
    _check(_lib.gs_mark_visible(proj.tiles_touched.data_ptr(), proj.tiles_touched.numel(), mask.data_ptr(),
                                _stream()))


# ------------------------------------------------------------------ spawning
SPAWN_BERNOULLI, SPAWN_FIXED_K = 0, 1


@dataclass
class SpawnParams:
    sigma: float = 1.0
    mode: int = SPAWN_BERNOULLI
    k: int = 0
    seed: int = 0
    opacity: float = 0.1
    min_prob: float = 1e-4

    def c(self):
        return _SpawnParams(self.sigma, self.mode, self.k, self.seed & ((1 << 64) - 1), self.opacity, self.min_prob)


def default_spawn_params() -> SpawnParams:
    p = _SpawnParams()
    _lib.gs_default_spawn_params(C.byref(p))
    return SpawnParams(p.sigma, p.mode, p.k, p.seed, p.opacity, p.min_prob)


def spawn_log_taps(sigma: float = 1.0):
    """The library's float32 LoG taps as a (2r+1, 2r+1) CPU tensor (host call)."""
    buf = (C.c_float * 289)()
    r = C.c_int32()
    _check(_lib.gs_spawn_log_taps(sigma, buf, C.byref(r)))
    n = 2 * r.value + 1
    return torch.tensor(list(buf[:n * n]), dtype=torch.float32).reshape(n, n)


def spawn_probability(cam: Camera, image: torch.Tensor, rendered: Optional[torch.Tensor] = None,
                      sp: SpawnParams = SpawnParams(), p_l: Optional[torch.Tensor] = None,
                      p_s: Optional[torch.Tensor] = None):
    """(P_L, P_s) [H][W] of a [3][H][W] image against the rendered one (Eq. 1-3)."""
    H, W = cam.height, cam.width
    _require(image, torch.float32, (3, H, W), "image")
    if rendered is not None:
        _require(rendered, torch.float32, (3, H, W), "rendered")
    if p_l is None:
        p_l = torch.empty((H, W), dtype=torch.float32, device=image.device)
    if p_s is None:
        p_s = torch.empty((H, W), dtype=torch.float32, device=image.device)
    _require(p_l, torch.float32, (H, W), "p_l")
    _require(p_s, torch.float32, (H, W), "p_s")
    _check(_lib.gs_spawn_probability(C.byref(cam.c()), image.data_ptr(), _ptr(rendered), C.byref(sp.c()),
                                     p_l.data_ptr(), p_s.data_ptr(), _stream()))
    return p_l, p_s


def spawn_select(cam: Camera, p_s: torch.Tensor, sp: SpawnParams = SpawnParams(),
                 capacity: Optional[int] = None, ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Flat indices (int32, increasing) of the pixels that spawn."""
    H, W = cam.height, cam.width
    _require(p_s, torch.float32, (H, W), "p_s")
    need = C.c_size_t()
    _check(_lib.gs_spawn_select_workspace(W, H, C.byref(need)))
    if ws is None or ws.numel() < need.value:
        ws = torch.empty(int(need.value), dtype=torch.uint8, device=p_s.device)
    if capacity is None:
        capacity = H * W
    pixels = torch.empty(max(capacity, 1), dtype=torch.int32, device=p_s.device)
    count = C.c_int64()
    _check(_lib.gs_spawn_select(C.byref(cam.c()), p_s.data_ptr(), C.byref(sp.c()), capacity, pixels.data_ptr(),
                                C.byref(count), ws.data_ptr(), ws.numel(), _stream()))
    return pixels[:count.value]


def spawn_rule(cam: Camera, image: torch.Tensor, depth: torch.Tensor, p_l: torch.Tensor, pixels: torch.Tensor,
               out: Gaussians, offset: int = 0, sp: SpawnParams = SpawnParams()):
    """Writes the direct rule's parameters of the spawned pixels into out[offset:offset+len(pixels)]."""
    H, W = cam.height, cam.width
    _require(image, torch.float32, (3, H, W), "image")
    _require(depth, torch.float32, (H, W), "depth")
    _require(p_l, torch.float32, (H, W), "p_l")
    if pixels.numel():
        _require(pixels, torch.int32, (pixels.numel(),), "pixels")
    _check(_lib.gs_spawn_rule(C.byref(cam.c()), image.data_ptr(), depth.data_ptr(), p_l.data_ptr(),
                              _ptr(pixels) if pixels.numel() else None, pixels.numel(), C.byref(sp.c()),
                              C.byref(out.c()), offset, _stream()))
    return out


def spawn_init_workspace(width: int, height: int, capacity: int) -> int:
    need = C.c_size_t()
    _check(_lib.gs_spawn_init_workspace(width, height, capacity, C.byref(need)))
    return int(need.value)


def spawn_init(cam: Camera, image: torch.Tensor, depth: torch.Tensor, out: Gaussians, offset: int = 0,
               rendered: Optional[torch.Tensor] = None, sp: SpawnParams = SpawnParams(),
               mlp_packed: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None) -> int:
    """The whole spawn step; returns the number of primitives written at out[offset:]."""
    H, W = cam.height, cam.width
    _require(image, torch.float32, (3, H, W), "image")
    _require(depth, torch.float32, (H, W), "depth")
    if rendered is not None:
        _require(rendered, torch.float32, (3, H, W), "rendered")
    need = spawn_init_workspace(W, H, out.n - offset)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=image.device)
    n = C.c_int64()
    _check(_lib.gs_spawn_init(C.byref(cam.c()), image.data_ptr(), depth.data_ptr(), _ptr(rendered), C.byref(sp.c()),
                              _ptr(mlp_packed), C.byref(out.c()), offset, C.byref(n), ws.data_ptr(), ws.numel(),
                              _stream()))
    return n.value


# ----------------------------------------------------------------- spawn MLP
MLP_INPUTS, MLP_OUTPUTS, MLP_PARAMS = 196, 7, 17223


def mlp_pack_bf16(theta: torch.Tensor, packed: Optional[torch.Tensor] = None) -> torch.Tensor:
    _require(theta, torch.float32, (MLP_PARAMS,), "theta")
    nbytes = int(_lib.gs_mlp_packed_bytes())
    if packed is None:
        packed = torch.empty(nbytes, dtype=torch.uint8, device=theta.device)
    _check(_lib.gs_mlp_pack_bf16(theta.data_ptr(), packed.data_ptr(), _stream()))
    return packed


def mlp_features(cam: Camera, image: torch.Tensor, depth: torch.Tensor, pixels: torch.Tensor) -> torch.Tensor:
    H, W = cam.height, cam.width
    _require(image, torch.float32, (3, H, W), "image")
    _require(depth, torch.float32, (H, W), "depth")
    out = torch.empty((pixels.numel(), MLP_INPUTS), dtype=torch.float32, device=image.device)
    if pixels.numel():
        _require(pixels, torch.int32, (pixels.numel(),), "pixels")
        _check(_lib.gs_mlp_features(C.byref(cam.c()), image.data_ptr(), depth.data_ptr(), pixels.data_ptr(),
                                    pixels.numel(), out.data_ptr(), _stream()))
    return out


def mlp_forward_bf16(packed: torch.Tensor, features: torch.Tensor) -> torch.Tensor:
    n = features.shape[0]
    _require(features, torch.float32, (n, MLP_INPUTS), "features")
    out = torch.empty((n, MLP_OUTPUTS), dtype=torch.float32, device=features.device)
    _check(_lib.gs_mlp_forward_bf16(packed.data_ptr(), features.data_ptr(), n, out.data_ptr(), _stream()))
    return out


def spawn_mlp(cam: Camera, image: torch.Tensor, depth: torch.Tensor, pixels: torch.Tensor, packed: torch.Tensor,
              out: Gaussians, offset: int = 0):
    H, W = cam.height, cam.width
    _require(image, torch.float32, (3, H, W), "image")
    _require(depth, torch.float32, (H, W), "depth")
    if pixels.numel():
        _require(pixels, torch.int32, (pixels.numel(),), "pixels")
    _check(_lib.gs_spawn_mlp(C.byref(cam.c()), image.data_ptr(), depth.data_ptr(),
                             _ptr(pixels) if pixels.numel() else None, pixels.numel(), packed.data_ptr(),
                             C.byref(out.c()), offset, _stream()))
    return out


class MlpTrainer:
    """FP32 training state of the spawn MLP (theta, Adam moments, workspace)."""

    def __init__(self, theta: torch.Tensor, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
                 eps: float = 1e-8):
        _require(theta, torch.float32, (MLP_PARAMS,), "theta")
        self.theta = theta
        self.m = torch.zeros_like(theta)
        self.v = torch.zeros_like(theta)
        self.lr, self.beta1, self.beta2, self.eps = lr, beta1, beta2, eps
        self.step_count = 0
        self.loss = torch.zeros(1, dtype=torch.float32, device=theta.device)
        self.ws = torch.empty(0, dtype=torch.uint8, device=theta.device)

    def step(self, features: torch.Tensor, targets: torch.Tensor, lr: Optional[float] = None,
             grad: Optional[torch.Tensor] = None):
        b = features.shape[0]
        _require(features, torch.float32, (b, MLP_INPUTS), "features")
        _require(targets, torch.float32, (b, MLP_OUTPUTS), "targets")
        need = C.c_size_t()
        _check(_lib.gs_mlp_train_workspace(b, C.byref(need)))
        if self.ws.numel() < need.value:
            self.ws = torch.empty(int(need.value), dtype=torch.uint8, device=features.device)
        lr = self.lr if lr is None else lr
        if lr != 0.0:
            self.step_count += 1
        _check(_lib.gs_mlp_train_step(self.theta.data_ptr(), self.m.data_ptr(), self.v.data_ptr(),
                                      features.data_ptr(), targets.data_ptr(), b, lr, self.beta1, self.beta2,
                                      self.eps, max(self.step_count, 1), self.loss.data_ptr(), _ptr(grad),
                                      self.ws.data_ptr(), self.ws.numel(), _stream()))
        return self.loss


def guided_depth(feat_i: torch.Tensor, feat_nb, rel_poses, zmono: torch.Tensor, fx: float, fy: float, cx: float,
                 cy: float, n_cand: int = 32, r_inv: float = 0.1, out=None):
    """Depth around the monocular depth by feature correlation with the
    neighbouring frames.  feat_i, feat_nb[j]: float16 [H][W][C]; rel_poses:
    [n_nb][12] (host values: R row-major, t); returns (depth, best, choice)."""
    H, W, Cc = feat_i.shape
    for f in [feat_i, *feat_nb]:
        _require(f, torch.float16, (H, W, Cc), "features")
    _require(zmono, torch.float32, (H, W), "zmono")
    if out is None:
        dev = feat_i.device
        out = (torch.empty((H, W), dtype=torch.float32, device=dev),
               torch.empty((H, W), dtype=torch.int32, device=dev),
               torch.empty((H, W), dtype=torch.int32, device=dev))
    depth, best, choice = out
    ptrs = (_vp * len(feat_nb))(*[f.data_ptr() for f in feat_nb])
    poses = np.ascontiguousarray(np.asarray(rel_poses, np.float32).reshape(len(feat_nb), 12))
    _check(_lib.gs_guided_depth(W, H, Cc, fx, fy, cx, cy, feat_i.data_ptr(), len(feat_nb), ptrs,
                                poses.ctypes.data_as(_P(C.c_float)), zmono.data_ptr(), n_cand, r_inv,
                                depth.data_ptr(), _ptr(best), _ptr(choice), _stream()))
    return depth, best, choice


# ------------------------------------------------------------------ anchors
def anchor_sizes(g: Gaussians, pose, f: float, tau: float = 1.0, flags: Optional[torch.Tensor] = None,
                 count: Optional[torch.Tensor] = None):
    """Count (device int64 [1]) of the Gaussians smaller than tau pixels
    from the camera with world->camera pose [12] (host values); flags [n]
    optional.  An anchor is created when count > 0.4 n."""
    if count is None:
        count = torch.zeros(1, dtype=torch.int64, device=g.means.device)
    p = (C.c_float * 12)(*[float(x) for x in np.asarray(pose, np.float32).reshape(12)])
    _check(_lib.gs_anchor_sizes(g.means.data_ptr(), g.log_scales.data_ptr(), g.n, p, f, tau, _ptr(flags),
                                count.data_ptr(), _stream()))
    return count


def anchor_blend_weight(d1: float, d2: float, overlap: float = 0.1) -> float:
    w = C.c_float()
    _check(_lib.gs_anchor_blend_weight(d1, d2, overlap, C.byref(w)))
    return w.value


def scale_opacity(logits: torch.Tensor, w: float, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """logit(w sigmoid(logits)): the opacities of an anchor's Gaussians at blend weight w."""
    if out is None:
        out = torch.empty_like(logits)
    _check(_lib.gs_scale_opacity(logits.data_ptr(), logits.numel(), w, out.data_ptr(), _stream()))
    return out


@dataclass
class MergePlan:
    cls: torch.Tensor  # (n,) int32: 0 other, 1 selected, 2 candidate
    nbr: torch.Tensor  # (n, k) int32
    owner: torch.Tensor  # (n,) int32
    new_index: torch.Tensor  # (n,) int32
    keep_index: torch.Tensor  # (n_keep,) int32 view
    k: int


def anchor_merge_plan(g: Gaussians, fine: torch.Tensor, k: int = 3, seed: int = 0,
                      ws: Optional[torch.Tensor] = None) -> MergePlan:
    """gs_anchor_merge_plan: which too-fine primitives merge with which
    (synchronises for the counts)."""
    n = g.n
    dev = g.means.device
    _require(fine, torch.int32, (n,), "fine")
    need = C.c_size_t()
    _check(_lib.gs_anchor_merge_workspace(n, C.byref(need)))
    if ws is None or ws.numel() < need.value:
        ws = torch.empty(max(int(need.value), 1), dtype=torch.uint8, device=dev)
    i32 = lambda *s: torch.empty(s, dtype=torch.int32, device=dev)
    cls, nbr, owner, new_index, keep = i32(n), i32(n, k), i32(n), i32(n), i32(max(n, 1))
    n_keep = C.c_int64()
    _check(_lib.gs_anchor_merge_plan(C.byref(g.c()), fine.data_ptr(), k, seed & ((1 << 64) - 1), cls.data_ptr(),
                                     nbr.data_ptr(), owner.data_ptr(), new_index.data_ptr(), keep.data_ptr(),
                                     C.byref(n_keep), ws.data_ptr(), ws.numel(), _stream()))
    return MergePlan(cls, nbr, owner, new_index, keep[:n_keep.value], k)


def anchor_merge_apply(g: Gaussians, plan: MergePlan, out: Optional[Gaussians] = None,
                       merged: Optional[torch.Tensor] = None):
    """gs_anchor_merge_apply: the new active set (n_keep Gaussians) and the
    int32 flags of its merged entries."""
    m = plan.keep_index.numel()
    dev = g.means.device
    if out is None:
        z = lambda *s: torch.empty(s, dtype=torch.float32, device=dev)
        out = Gaussians(z(3, m), z(3, m), z(4, m), z(m), z(g.sh.shape[0], 3, m))
    if merged is None:
        merged = torch.empty(m, dtype=torch.int32, device=dev)
    _check(_lib.gs_anchor_merge_apply(C.byref(g.c()), plan.cls.data_ptr(), plan.nbr.data_ptr(),
                                      plan.owner.data_ptr(), plan.new_index.data_ptr(), plan.keep_index.data_ptr(),
                                      plan.k, C.byref(out.c()), merged.data_ptr(), _stream()))
    return out, merged


def masked_fill(planes: torch.Tensor, mask: torch.Tensor, value: float = 0.0):
    """planes [..., n] float32: planes[..., i] = value where mask[i] != 0."""
    n = mask.numel()
    _require(mask, torch.int32, (n,), "mask")
    if planes.shape[-1] != n or not planes.is_contiguous() or planes.dtype != torch.float32:
        raise ValueError("planes: contiguous float32 [..., n]")
    _check(_lib.gs_masked_fill(planes.data_ptr(), n, planes.numel() // max(n, 1), mask.data_ptr(), value, _stream()))


def _plane_lists(tensors):
    k = len(tensors)
    ptrs = (_vp * max(k, 1))(*[t.data_ptr() for t in tensors])
    sizes = (_sz * max(k, 1))(*[t.numel() * t.element_size() for t in tensors])
    return k, ptrs, sizes


def anchor_host_bytes(tensors) -> int:
    k, _, sizes = _plane_lists(tensors)
    return int(_lib.gs_anchor_host_bytes(k, sizes))


def anchor_offload(tensors, host: torch.Tensor):
    """gs_anchor_offload: the device tensors into one pinned uint8 host block
    (asynchronous on the current stream)."""
    for t in tensors:
        if not t.is_contiguous() or not t.is_cuda:
            raise ValueError("anchor_offload: contiguous device tensors only")
    if host.device.type != "cpu" or host.dtype != torch.uint8 or host.numel() < anchor_host_bytes(tensors):
        raise ValueError("anchor_offload: host block too small or not a uint8 CPU tensor")
    k, ptrs, sizes = _plane_lists(tensors)
    _check(_lib.gs_anchor_offload(k, ptrs, sizes, host.data_ptr(), _stream()))


def anchor_reload(tensors, host: torch.Tensor):
    """gs_anchor_reload: the host block back into the device tensors."""
    for t in tensors:
        if not t.is_contiguous() or not t.is_cuda:
            raise ValueError("anchor_reload: contiguous device tensors only")
    if host.device.type != "cpu" or host.dtype != torch.uint8 or host.numel() < anchor_host_bytes(tensors):
        raise ValueError("anchor_reload: host block too small or not a uint8 CPU tensor")
    k, ptrs, sizes = _plane_lists(tensors)
    _check(_lib.gs_anchor_reload(k, ptrs, sizes, host.data_ptr(), _stream()))


# ------------------------------------------------------ mini bundle adjustment
def pose_ransac(X: torch.Tensor, uv: torch.Tensor, fx: float, fy: float, cx: float, cy: float, pose0,
                n_hyp: int = 128, sample: int = 6, hyp_iters: int = 10, tau: float = 2.0, refine_iters: int = 20,
                huber_delta: float = 1.0, seed: int = 0, ws: Optional[torch.Tensor] = None):
    """gs_pose_ransac: (pose float64 [12], pose float32 [12], inliers int32 [K],
    n_inliers int32 [1], hypothesis counts int32 [n_hyp]) on the device."""
    K = X.shape[1]
    _require(X, torch.float32, (3, K), "X")
    _require(uv, torch.float32, (2, K), "uv")
    dev = X.device
    need = C.c_size_t()
    _check(_lib.gs_pose_ransac_workspace(n_hyp, C.byref(need)))
    if ws is None or ws.numel() < need.value:
        ws = torch.empty(int(need.value), dtype=torch.uint8, device=dev)
    p0 = (C.c_double * 12)(*[float(x) for x in np.asarray(pose0, np.float64).reshape(12)])
    pose = torch.empty(12, dtype=torch.float64, device=dev)
    pose32 = torch.empty(12, dtype=torch.float32, device=dev)
    inl = torch.empty(K, dtype=torch.int32, device=dev)
    n_inl = torch.empty(1, dtype=torch.int32, device=dev)
    counts = torch.empty(n_hyp, dtype=torch.int32, device=dev)
    _check(_lib.gs_pose_ransac(X.data_ptr(), uv.data_ptr(), K, fx, fy, cx, cy, p0, n_hyp, sample, hyp_iters, tau,
                               refine_iters, huber_delta, seed & ((1 << 64) - 1), inl.data_ptr(), n_inl.data_ptr(),
                               pose.data_ptr(), pose32.data_ptr(), counts.data_ptr(), ws.data_ptr(), ws.numel(),
                               _stream()))
    return pose, pose32, inl, n_inl, counts


def ba_bootstrap(uv: torch.Tensor, width: int, height: int, iters: int = 200, mad_from: int = -1,
                 huber_delta: float = 1.0, trace: bool = False, ws: Optional[torch.Tensor] = None):
    """gs_ba_bootstrap on uv [V][2][P]: (f [1], poses [V][12], X [3][P],
    trace [iters][3] or None), float64 on the device."""
    V, _, P = uv.shape
    _require(uv, torch.float32, (V, 2, P), "uv")
    dev = uv.device
    need = C.c_size_t()
    _check(_lib.gs_ba_bootstrap_workspace(V, P, C.byref(need)))
    if ws is None or ws.numel() < need.value:
        ws = torch.empty(int(need.value), dtype=torch.uint8, device=dev)
    d = lambda *s: torch.empty(s, dtype=torch.float64, device=dev)
    f, poses, X = d(1), d(V, 12), d(3, P)
    tr = d(max(iters, 1), 3) if trace else None
    _check(_lib.gs_ba_bootstrap(uv.data_ptr(), V, P, width, height, iters, mad_from, huber_delta, f.data_ptr(),
                                poses.data_ptr(), X.data_ptr(), _ptr(tr), ws.data_ptr(), ws.numel(), _stream()))
    return f, poses, X, tr


def probe_copy(src: torch.Tensor, dst: torch.Tensor):
    """dst = src with the library's 16-byte copy kernel (HBM rate probe)."""
    _check(_lib.gs_probe_copy(src.data_ptr(), dst.data_ptr(), src.numel() * src.element_size(), _stream()))


def probe_valu(kind: int, blocks: int, iters: int, out: torch.Tensor):
    """blocks x 256 lanes x iters x 8 chained v_fma_f32 (kind 0) or v_exp_f32 (kind 1)."""
    _check(_lib.gs_probe_valu(kind, blocks, iters, out.data_ptr(), _stream()))


def profile_enable(on: bool = True):
    _lib.gs_profile_enable(1 if on else 0)


def profile_select(names=None):
    """Bracket only the named kernels (an iterable of names); None: all."""
    _lib.gs_profile_select(None if names is None else ",".join(names).encode())


def profile_reset():
    _lib.gs_profile_reset()


def profile_read(kernel: str):
    ms, cnt = C.c_double(), C.c_int64()
    _check(_lib.gs_profile_read(kernel.encode(), C.byref(ms), C.byref(cnt)))
    return ms.value, cnt.value


# ------------------------------------------------------------------ autograd
class _Rasterize(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity_logits, sh, pose, cam_static, params, sorter, shared):
        g = Gaussians(means.contiguous(), log_scales.contiguous(), quats.contiguous(), opacity_logits.contiguous(),
                      sh.contiguous())
        cam = Camera(cam_static.width, cam_static.height, cam_static.fx, cam_static.fy, cam_static.cx,
                     cam_static.cy, pose.detach().contiguous(), cam_static.near_plane, cam_static.bg)
        proj = project(cam, g, params)
        binned = sorter(cam, proj)
        frame = render_fwd(cam, proj, binned, params)
        if shared:
            # the sorter's buffers are reused by its next call (another view of
            # the same loss may run before this backward): keep this view's own
            # lists (the first n_instances pairs, the ranges and first slots)
            M = binned.n_instances
            binned = Binned(binned.tile_ids[:M].clone(), binned.values[:M].clone(), binned.slots[:M].clone(),
                            binned.ranges.clone(), binned.first_slot.clone(), M)
        ctx.state = (g, cam, proj, binned, frame, params)
        ctx.mark_non_differentiable(frame.n_contrib)
        return frame.image, frame.depth, frame.alpha

    @staticmethod
    def backward(ctx, g_image, g_depth, g_alpha):
        g, cam, proj, binned, frame, params = ctx.state
        f = lambda t: None if t is None else t.contiguous()
        g_image = f(g_image) if g_image is not None else torch.zeros_like(frame.image)
        d_pose = torch.zeros(12, dtype=torch.float64, device=g.means.device)
        grads = render_bwd(cam, g, proj, binned, frame, g_image, f(g_depth), f(g_alpha), dL_dpose=d_pose,
                           params=params)
        return (grads.means, grads.log_scales, grads.quats, grads.opacity_logits, grads.sh,
                d_pose.to(torch.float32), None, None, None, None)


def rasterize(g: Gaussians, cam: Camera, params: Params = Params(), sorter: Optional[BinSorter] = None):
    """Differentiable render: returns (image (3,H,W), depth (H,W), alpha (H,W)).
    Gradients flow to every Gaussian plane and to cam.pose (float32 [12]).
    A caller's sorter may be shared by several calls before their backward:
    each call then keeps a copy of its own lists."""
    return _Rasterize.apply(g.means, g.log_scales, g.quats, g.opacity_logits, g.sh, cam.pose, cam, params,
                            sorter or BinSorter(), sorter is not None)


# ------------------------------------------------------------ spatial cells
def _ws(query, *args, device="cuda"):
    need = C.c_size_t()
    _check(query(*args, C.byref(need)))
    return torch.empty(max(int(need.value), 1), dtype=torch.uint8, device=device)


def cells_assign(means: torch.Tensor, centroids: torch.Tensor) -> torch.Tensor:
    """gs_cells_assign: nearest centroid (float64 [k][3]) of every mean."""
    n, k = means.shape[1], centroids.shape[0]
    _require(means, torch.float32, (3, n), "means")
    _require(centroids, torch.float64, (k, 3), "centroids")
    labels = torch.empty(n, dtype=torch.int32, device=means.device)
    _check(_lib.gs_cells_assign(means.data_ptr(), n, centroids.data_ptr(), k, labels.data_ptr(), _stream()))
    return labels


def cells_kmeans(means: torch.Tensor, k: int, iters: int, centroids: Optional[torch.Tensor] = None,
                 with_order: bool = True):
    """gs_cells_kmeans: (centroids [k][3] float64, labels, order, offsets);
    starts from the spread initial centroids unless centroids are given."""
    n = means.shape[1]
    _require(means, torch.float32, (3, n), "means")
    dev = means.device
    init = centroids is None
    cent = torch.empty((k, 3), dtype=torch.float64, device=dev) if init else centroids
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    order = torch.empty(n, dtype=torch.int32, device=dev) if with_order else None
    offsets = torch.empty(k + 1, dtype=torch.int64, device=dev) if with_order else None
    ws = _ws(_lib.gs_cells_kmeans_workspace, n, k, device=dev)
    _check(_lib.gs_cells_kmeans(means.data_ptr(), n, k, iters, int(init), cent.data_ptr(), labels.data_ptr(),
                                _ptr(order), _ptr(offsets), ws.data_ptr(), ws.numel(), _stream()))
    return cent, labels, order, offsets


def cells_spheres(means: torch.Tensor, log_scales: torch.Tensor, labels: torch.Tensor, centroids: torch.Tensor,
                  margin: float = 3.0) -> torch.Tensor:
    n, k = means.shape[1], centroids.shape[0]
    radius = torch.empty(k, dtype=torch.float64, device=means.device)
    ws = _ws(_lib.gs_cells_spheres_workspace, n, k, device=means.device)
    _check(_lib.gs_cells_spheres(means.data_ptr(), log_scales.data_ptr(), n, labels.data_ptr(), centroids.data_ptr(),
                                 k, margin, radius.data_ptr(), ws.data_ptr(), ws.numel(), _stream()))
    return radius


def cells_visible(centroids: torch.Tensor, radius: torch.Tensor, cam: Camera, guard: float = 1.3,
                  out: Optional[torch.Tensor] = None) -> torch.Tensor:
    k = centroids.shape[0]
    if out is None:
        out = torch.empty(k, dtype=torch.int32, device=centroids.device)
    _check(_lib.gs_cells_visible(centroids.data_ptr(), radius.data_ptr(), k, C.byref(cam.c()), guard,
                                 out.data_ptr(), _stream()))
    return out


def copy_rows(dst_ptr: int, dpitch: int, src_ptr: int, spitch: int, width: int, height: int):
    """gs_copy_rows on the current stream (raw addresses: device or pinned host)."""
    _check(_lib.gs_copy_rows(dst_ptr, dpitch, src_ptr, spitch, width, height, _stream()))


def fill_(t: torch.Tensor, value: float):
    """gs_fill_f32 over a contiguous float32 device tensor."""
    assert t.dtype == torch.float32 and t.is_contiguous()
    _check(_lib.gs_fill_f32(t.data_ptr(), t.numel(), value, _stream()))


def filter3d_update(means: torch.Tensor, cams, nu_max: torch.Tensor, filter3d: Optional[torch.Tensor] = None,
                    guard: float = 1.15, s_f: float = 0.2):
    """gs_filter3d_update: nu_max = max(nu_max, the cameras' sampling rates);
    filter3d = (s_f / nu_max)^2 (0 where no camera has seen the Gaussian)."""
    n = means.shape[1]
    _require(nu_max, torch.float32, (n,), "nu_max")
    arr = (_Camera * max(len(cams), 1))()
    for k, c in enumerate(cams):
        arr[k] = c.c()
    _check(_lib.gs_filter3d_update(means.data_ptr(), n, len(cams), arr, guard, s_f, nu_max.data_ptr(),
                                   _ptr(filter3d), _stream()))
    return filter3d
