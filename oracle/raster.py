"""ctypes front end of the FP64 C oracle (gs_oracle.c).

Test infrastructure only: tests, the smoke check and the CPU baseline of the
benchmark call it; the product path never does.

Every function follows the plain definition of the splatting rasterizer
(EWA projection, per-pixel front-to-back compositing over all visible
Gaussians in (depth, index) order, transmittance cutoff) and its analytic
adjoint; see the header of gs_oracle.c for the statement.  Inputs are the
same float32 SoA planes the HIP path receives, widened exactly to float64.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gs_oracle.c")
_LIB = os.path.join(_HERE, "libgs_oracle.so")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C11, -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
                               "-ffp-contract=off", "-o", tmp, _SRC, "-lm", "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


class _Cam(C.Structure):
    _fields_ = [("R", C.c_double * 9), ("t", C.c_double * 3), ("fx", C.c_double), ("fy", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double), ("width", C.c_int32), ("height", C.c_int32),
                ("near_plane", C.c_double), ("bg", C.c_double * 3), ("eps2d", C.c_double),
                ("alpha_max", C.c_double), ("alpha_min", C.c_double), ("t_min", C.c_double),
                ("guard", C.c_double), ("mip_filter", C.c_int32)]


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class _Gauss(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int32), ("means", _dp), ("log_scales", _dp),
                ("quats", _dp), ("opacity_logits", _dp), ("sh", _dp)]


class _Proj(C.Structure):
    _fields_ = [("mean2d", _dp), ("depth", _dp), ("conic", _dp), ("cov2d", _dp), ("opacity", _dp),
                ("rgb", _dp), ("radius", _dp), ("half", _dp), ("visible", _ip), ("clamped", _ip)]


_lib = None


def lib():
    """The oracle library (GS_ORACLE_LIB names another build of gs_oracle.c,
    e.g. one with the address and undefined-behaviour sanitizers)."""
    global _lib
    if _lib is None:
        _lib = C.CDLL(os.environ.get("GS_ORACLE_LIB") or build())
        _lib.orc_render.restype = C.c_int
        _lib.orc_render_bwd.restype = C.c_int
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def _i(a):
    return a.ctypes.data_as(_ip) if a is not None else None


@dataclass
class Camera:
    """Pinhole camera, world->camera pose, and the compositing constants."""
    R: np.ndarray
    t: np.ndarray
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    near_plane: float = 0.2
    bg: tuple = (0.0, 0.0, 0.0)
    eps2d: float = 0.3
    alpha_max: float = 0.99
    alpha_min: float = 1.0 / 255.0
    t_min: float = 1e-4
    guard: float = 1.3
    mip_filter: int = 0  # 1: eps2d is a screen-space filter, opacity scaled by sqrt(det Sigma2_raw / det Sigma2)

    @staticmethod
    def from_view(view, **kw):
        return Camera(np.asarray(view.R, np.float32).astype(np.float64),
                      np.asarray(view.t, np.float32).astype(np.float64),
                      float(np.float32(view.fx)), float(np.float32(view.fy)), float(np.float32(view.cx)),
                      float(np.float32(view.cy)), view.width, view.height, **kw)

    def c(self) -> _Cam:
        c = _Cam()
        c.R[:] = [float(x) for x in np.asarray(self.R, np.float64).reshape(9)]
        c.t[:] = [float(x) for x in np.asarray(self.t, np.float64).reshape(3)]
        c.fx, c.fy, c.cx, c.cy = self.fx, self.fy, self.cx, self.cy
        c.width, c.height = self.width, self.height
        c.near_plane = self.near_plane
        c.bg[:] = list(self.bg)
        c.eps2d, c.alpha_max, c.alpha_min, c.t_min, c.guard = (self.eps2d, self.alpha_max, self.alpha_min,
                                                                 self.t_min, self.guard)
        c.mip_filter = int(self.mip_filter)
        return c


class Gaussians:
    """float64 copies of the SoA planes (kept alive for the C calls)."""

    def __init__(self, means, log_scales, quats, opacity_logits, sh, sh_degree):
        f = lambda a: np.ascontiguousarray(np.asarray(a, np.float64))
        self.means, self.log_scales, self.quats = f(means), f(log_scales), f(quats)
        self.opacity_logits, self.sh = f(opacity_logits), f(sh)
        self.sh_degree = int(sh_degree)
        self.n = self.means.shape[1]
        assert self.sh.shape == ((self.sh_degree + 1) ** 2, 3, self.n)

    @staticmethod
    def from_scene(scene):
        return Gaussians(scene.means, scene.log_scales, scene.quats, scene.opacity_logits, scene.sh,
                         scene.sh_degree)

    def c(self) -> _Gauss:
        return _Gauss(self.n, self.sh_degree, _d(self.means), _d(self.log_scales), _d(self.quats),
                      _d(self.opacity_logits), _d(self.sh))


def project(cam: Camera, g: Gaussians) -> dict:
    """Per-Gaussian EWA projection (FP64)."""
    n = g.n
    out = dict(mean2d=np.zeros((2, n)), depth=np.zeros(n), conic=np.zeros((3, n)), cov2d=np.zeros((3, n)),
               opacity=np.zeros(n), rgb=np.zeros((3, n)), radius=np.zeros(n), half=np.zeros((2, n)),
               visible=np.zeros(n, np.int32), clamped=np.zeros(n, np.int32))
    p = _Proj(_d(out["mean2d"]), _d(out["depth"]), _d(out["conic"]), _d(out["cov2d"]), _d(out["opacity"]),
              _d(out["rgb"]), _d(out["radius"]), _d(out["half"]), _i(out["visible"]), _i(out["clamped"]))
    gc = g.c()
    lib().orc_project(C.byref(cam.c()), C.byref(gc), C.byref(p))
    out["_c"] = p
    return out


def _nthreads(nthreads):
    return int(nthreads or min(os.cpu_count() or 1, 64))


def render(cam: Camera, proj: dict, crop=None, flag_rel: float = 1e-5, nthreads=None) -> dict:
    """Brute-force compositing over the crop (x0, y0, w, h), default full image."""
    x0, y0, cw, ch = crop if crop is not None else (0, 0, cam.width, cam.height)
    n = proj["depth"].shape[0]
    out = dict(image=np.zeros((3, ch, cw)), depth=np.zeros((ch, cw)), alpha=np.zeros((ch, cw)),
               final_t=np.zeros((ch, cw)), n_contrib=np.zeros((ch, cw), np.int32),
               n_support=np.zeros((ch, cw), np.int32), flags=np.zeros((ch, cw), np.int32))
    lib().orc_render(C.byref(cam.c()), C.byref(proj["_c"]), C.c_int64(n), x0, y0, cw, ch,
                     C.c_double(flag_rel), _nthreads(nthreads), _d(out["image"]), _d(out["depth"]),
                     _d(out["alpha"]), _d(out["final_t"]), _i(out["n_contrib"]), _i(out["n_support"]),
                     _i(out["flags"]))
    return out


def render_bwd(cam: Camera, proj: dict, g_image=None, g_depth=None, g_alpha=None, crop=None, nthreads=None):
    """Per-Gaussian gradients of the 2D quantities, [n][10] =
    (d mean2d x, y, d conic A, B, C, d opacity, d rgb r, g, b, d depth)."""
    x0, y0, cw, ch = crop if crop is not None else (0, 0, cam.width, cam.height)
    n = proj["depth"].shape[0]
    g2d = np.zeros((n, 10))
    f = lambda a: None if a is None else np.ascontiguousarray(np.asarray(a, np.float64))
    gi, gd, ga = f(g_image), f(g_depth), f(g_alpha)
    rc = lib().orc_render_bwd(C.byref(cam.c()), C.byref(proj["_c"]), C.c_int64(n), x0, y0, cw, ch,
                              _nthreads(nthreads), _d(gi), _d(gd), _d(ga), _d(g2d))
    if rc != 0:
        raise MemoryError("oracle render_bwd: allocation failed")
    return g2d


def project_bwd(cam: Camera, g: Gaussians, g2d: np.ndarray) -> dict:
    """Chain the 2D gradients to the parameters and to the camera pose."""
    n = g.n
    out = dict(means=np.zeros((3, n)), log_scales=np.zeros((3, n)), quats=np.zeros((4, n)),
               opacity_logits=np.zeros(n), sh=np.zeros_like(g.sh), R=np.zeros(9), t=np.zeros(3),
               twist=np.zeros(6))
    g2d = np.ascontiguousarray(g2d, np.float64)
    lib().orc_project_bwd(C.byref(cam.c()), C.byref(g.c()), _d(g2d), _d(out["means"]), _d(out["log_scales"]),
                          _d(out["quats"]), _d(out["opacity_logits"]), _d(out["sh"]), _d(out["R"]), _d(out["t"]),
                          _d(out["twist"]))
    out["R"] = out["R"].reshape(3, 3)
    return out


def forward(cam: Camera, g: Gaussians, crop=None, flag_rel: float = 1e-5, nthreads=None):
    proj = project(cam, g)
    return proj, render(cam, proj, crop, flag_rel, nthreads)


def backward(cam: Camera, g: Gaussians, proj: dict, g_image=None, g_depth=None, g_alpha=None, crop=None,
             nthreads=None) -> dict:
    g2d = render_bwd(cam, proj, g_image, g_depth, g_alpha, crop, nthreads)
    out = project_bwd(cam, g, g2d)
    out["g2d"] = g2d
    return out


def sh_basis(deg: int, dirs: np.ndarray) -> np.ndarray:
    """Real SH basis values at unit directions dirs (M,3) -> (M,(deg+1)^2)."""
    nb = (deg + 1) ** 2
    out = np.zeros((dirs.shape[0], 16))
    buf = np.zeros(16)
    for k in range(dirs.shape[0]):
        d = np.ascontiguousarray(dirs[k], np.float64)
        lib().orc_sh_basis(deg, _d(d), _d(buf))
        out[k] = buf
    return out[:, :nb]


def quat_to_rot(q) -> np.ndarray:
    q = np.ascontiguousarray(np.asarray(q, np.float64))
    R = np.zeros(9)
    lib().orc_quat_to_rot(_d(q), _d(R))
    return R.reshape(3, 3)
