"""The C ABI library loads and exports every entry point include/gs_api.h
declares, and its host-side argument checks reject bad calls before any
launch (these run without a GPU: nothing reaches the device)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gs_api.h")
# GSMI_LIB: another build of the same sources (e.g. the host code under AddressSanitizer)
LIB = os.environ.get("GSMI_LIB") or os.path.join(ROOT, "paper_2506_05558_amd", "libgsmi.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gs_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libgsmi.so is not built (run __graft_entry__.build())")
    return C.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert len(names) >= 16
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_the_header(lib):
    from paper_2506_05558_amd import gsmi
    assert set(declared()) <= set(gsmi.exported_symbols())


def test_default_params(lib):
    from paper_2506_05558_amd import gsmi
    p = gsmi.default_params()
    assert abs(p.eps2d - 0.3) < 1e-7 and abs(p.alpha_max - 0.99) < 1e-7
    assert abs(p.alpha_min - 1 / 255) < 1e-9 and abs(p.t_min - 1e-4) < 1e-10 and abs(p.guard - 1.3) < 1e-7
    assert p.mip_filter == 0
    # the C struct matches the header's layout: five floats, then the filter flag
    assert C.sizeof(gsmi._Params) == 24 and gsmi._Params.mip_filter.offset == 20


def test_host_validation_rejects_bad_calls(lib):
    from paper_2506_05558_amd import gsmi as g
    lib.gs_last_error.restype = C.c_char_p
    cam = g._Camera(0, 10, 1.0, 1.0, 0.0, 0.0, 0.2, (C.c_float * 3)(0, 0, 0), None)
    prm = g._Params(0.3, 0.99, 1 / 255, 1e-4, 1.3)
    gau = g._Gauss(10, 0, None, None, None, None, None)
    prj = g._Proj(None, None, None)
    # zero-sized image
    assert lib.gs_project(C.byref(cam), C.byref(prm), C.byref(gau), C.byref(prj), None) == g.GS_ERR_INVALID_ARG
    assert b"image size" in lib.gs_last_error()
    cam.width = 10
    # missing pose
    assert lib.gs_project(C.byref(cam), C.byref(prm), C.byref(gau), C.byref(prj), None) == g.GS_ERR_INVALID_ARG
    cam.pose = 16  # any non-NULL value: validation fails before it is used
    # NULL parameter planes with n > 0
    assert lib.gs_project(C.byref(cam), C.byref(prm), C.byref(gau), C.byref(prj), None) == g.GS_ERR_INVALID_ARG
    # SH degree out of range
    gau.sh_degree = 4
    assert lib.gs_project(C.byref(cam), C.byref(prm), C.byref(gau), C.byref(prj), None) == g.GS_ERR_INVALID_ARG
    assert b"sh_degree" in lib.gs_last_error()
    # n < 0
    gau.sh_degree, gau.n = 0, -1
    assert lib.gs_project(C.byref(cam), C.byref(prm), C.byref(gau), C.byref(prj), None) == g.GS_ERR_INVALID_ARG
    # NULL camera
    assert lib.gs_render_fwd(None, C.byref(prm), C.byref(prj), None, None, None, None, None, None, None, None,
                             None) == g.GS_ERR_INVALID_ARG
    # Adam: step must be >= 1
    lib.gs_adam_step.argtypes = [C.c_void_p] * 4 + [C.c_int64, C.c_float, C.c_float, C.c_float, C.c_float,
                                                    C.c_int32, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]
    assert lib.gs_adam_step(None, None, None, None, 10, 1e-3, 0.9, 0.999, 1e-8, 0, None, None, 0,
                            None) == g.GS_ERR_INVALID_ARG
    # per-Gaussian rates need a plane stride
    assert lib.gs_adam_step(1, 1, 1, 1, 10, 1e-3, 0.9, 0.999, 1e-8, 1, None, 1, 0,
                            None) == g.GS_ERR_INVALID_ARG


def test_workspace_queries(lib):
    sz = C.c_size_t()
    lib.gs_bin_sort_workspace.argtypes = [C.c_int64, C.c_int64, C.POINTER(C.c_size_t)]
    assert lib.gs_bin_sort_workspace(2_000_000, 20_000_000, C.byref(sz)) == 0
    assert sz.value >= 4 * (8 * 2_000_000 + 2 * 20_000_000)
    assert lib.gs_bin_sort_workspace(-1, 0, C.byref(sz)) == 1
    lib.gs_render_bwd_workspace.argtypes = [C.c_int64, C.c_int64, C.POINTER(C.c_size_t)]
    assert lib.gs_render_bwd_workspace(1000, 3000, C.byref(sz)) == 0 and sz.value >= 48 * 3000
    # the projection adjoint keeps each view's clamped colour gradient (3 floats per Gaussian) between
    # its geometry and SH passes, for up to eight views per pass
    lib.gs_project_bwd_views_workspace.argtypes = [C.c_int64, C.c_int32, C.POINTER(C.c_size_t)]
    for nv, per in [(1, 1), (8, 8), (20, 8)]:
        assert lib.gs_project_bwd_views_workspace(100_000, nv, C.byref(sz)) == 0
        assert sz.value >= 12 * per * 100_000
    # larger inputs never need less
    sizes = []
    for n, cap in [(10, 10), (10_000, 10), (10_000, 100_000), (1_000_000, 100_000)]:
        assert lib.gs_bin_sort_workspace(n, cap, C.byref(sz)) == 0
        sizes.append(sz.value)
    assert sizes == sorted(sizes)


def test_spawn_taps_equal_the_oracle_bitwise(lib):
    """The library's LoG taps (host arithmetic: libm exp, exactly rounded
    mean) are the oracle's taps rounded to float32, bit for bit."""
    import numpy as np
    from oracle import spawn
    from paper_2506_05558_amd import gsmi
    for sigma in (1.0, 0.7, 1.5, 2.0):
        t = gsmi.spawn_log_taps(sigma).numpy()
        o = spawn.log_kernel_f64(float(np.float32(sigma))).astype(np.float32)
        assert t.shape == o.shape and np.array_equal(t.view(np.uint32), o.view(np.uint32)), sigma
    with pytest.raises(gsmi.GsError):
        gsmi.spawn_log_taps(2.5)  # radius beyond the kernel's halo


def test_spawn_validation(lib):
    from paper_2506_05558_amd import gsmi as g
    cam = g._Camera(16, 16, 10.0, 10.0, 8.0, 8.0, 0.2, (C.c_float * 3)(0, 0, 0), 16)
    sp = g._SpawnParams()
    g._lib.gs_default_spawn_params(C.byref(sp))
    assert abs(sp.sigma - 1.0) < 1e-7 and sp.mode == g.SPAWN_BERNOULLI and abs(sp.opacity - 0.1) < 1e-7
    # NULL image
    assert g._lib.gs_spawn_probability(C.byref(cam), None, None, C.byref(sp), None, 16, None) == g.GS_ERR_INVALID_ARG
    sp.mode = 7
    assert g._lib.gs_spawn_probability(C.byref(cam), 16, None, C.byref(sp), None, 16, None) == g.GS_ERR_INVALID_ARG
    assert b"mode" in g._lib.gs_last_error()
    sp.mode, sp.k = g.SPAWN_FIXED_K, -1
    n = C.c_int64()
    assert g._lib.gs_spawn_select(C.byref(cam), 16, C.byref(sp), 0, None, C.byref(n), None, 0,
                                  None) == g.GS_ERR_INVALID_ARG
    sp.k, sp.opacity = 10, 1.0
    gau = g._Gauss(4, 0, 16, 16, 16, 16, 16)
    assert g._lib.gs_spawn_rule(C.byref(cam), 16, 16, 16, 16, 1, C.byref(sp), C.byref(gau), 0,
                                None) == g.GS_ERR_INVALID_ARG
    sp.opacity = 0.1
    # destination too small: offset + count > n
    assert g._lib.gs_spawn_rule(C.byref(cam), 16, 16, 16, 16, 3, C.byref(sp), C.byref(gau), 2,
                                None) == g.GS_ERR_CAPACITY
    sz = C.c_size_t()
    assert g._lib.gs_spawn_select_workspace(1920, 1080, C.byref(sz)) == 0 and sz.value >= 24 * 1920 * 1080


def test_camera_level_equals_the_oracle(lib):
    # host-only: the coarse camera is computed on the host (the pose pointer
    # is only copied, never dereferenced)
    import numpy as np

    from oracle import multiscale as ms
    from paper_2506_05558_amd import gsmi
    cam = gsmi._Camera(1920, 1080, 1111.5, 1050.25, 959.5, 539.5, 0.2, (C.c_float * 3)(0.1, 0.2, 0.3), 0x1000)
    for level in range(5):
        out = gsmi._Camera()
        assert gsmi._lib.gs_camera_level(C.byref(cam), level, C.byref(out)) == 0
        ref = ms.camera_level(cam.width, cam.height, float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy),
                              level)
        assert (out.width, out.height) == ref[:2]
        assert [out.fx, out.fy, out.cx, out.cy] == [float(np.float32(x)) for x in ref[2:]]
        assert out.pose == cam.pose and out.near_plane == cam.near_plane and list(out.bg) == list(cam.bg)
    bad = gsmi._Camera()
    assert gsmi._lib.gs_camera_level(C.byref(cam), 5, C.byref(bad)) == 1
    tiny = gsmi._Camera(7, 9, 1.0, 1.0, 3.0, 4.0, 0.2, (C.c_float * 3)(), 0x1000)
    assert gsmi._lib.gs_camera_level(C.byref(tiny), 3, C.byref(bad)) == 1  # 7 >> 3 = 0 columns


def test_multiscale_validation(lib):
    from paper_2506_05558_amd import gsmi
    L = gsmi._lib
    assert L.gs_downsample(1, 3, 64, 64, 5, 2, None) == 1        # level out of range
    assert L.gs_downsample(1, 3, 4, 64, 3, 2, None) == 1         # narrower than one block
    assert L.gs_downsample(None, 3, 64, 64, 2, 2, None) == 1     # NULL input
    kept = C.c_int64(-1)
    assert L.gs_prune_opacity(1, 10, 0.0, 1, C.byref(kept), 1, 1 << 20, None) == 1
    assert L.gs_prune_opacity(1, 10, 0.005, 1, C.byref(kept), None, 0, None) == gsmi.GS_ERR_WORKSPACE
    assert L.gs_prune_opacity(None, 0, 0.005, None, C.byref(kept), None, 0, None) == 0 and kept.value == 0
    assert L.gs_gather_planes(1, 10, 70000, 1, 5, 2, None) == 1  # too many planes
    assert L.gs_gather_planes(1, 10, 2, 1, 5, 1, None) == 1      # in place
    assert L.gs_lr_decay(1, None, 10, 0.0, None) == 1
    assert L.gs_lr_decay(1, None, 10, 1.5, None) == 1
    sz = C.c_size_t()
    sizes = []
    for n in (1, 1000, 2_000_000):
        assert L.gs_prune_workspace(n, C.byref(sz)) == 0
        sizes.append(sz.value)
    assert sizes == sorted(sizes) and sizes[-1] >= 8 * 2_000_000


def test_probe_validation(lib):
    from paper_2506_05558_amd import gsmi
    L = gsmi._lib
    assert L.gs_probe_copy(16, 32, 24, None) == 1          # not a 16-byte multiple
    assert L.gs_probe_copy(16, 16, 32, None) == 1          # in place
    assert L.gs_probe_copy(None, None, 0, None) == 0
    assert L.gs_probe_valu(2, 8, 8, 16, None) == 1         # unknown kind
    assert L.gs_probe_valu(0, 0, 8, 16, None) == 1         # no blocks
    assert L.gs_probe_valu(1, 8, 8, None, None) == 1       # no output


def test_guided_depth_validation(lib):
    from paper_2506_05558_amd import gsmi
    L = gsmi._lib
    ptrs = (C.c_void_p * 1)(16)
    pose = (C.c_float * 12)()
    args = lambda **kw: dict(dict(w=64, h=32, c=32, nb=1, n=32, r=0.1, fi=16), **kw)

    def call(a):
        return L.gs_guided_depth(a["w"], a["h"], a["c"], 50.0, 50.0, 31.5, 15.5, a["fi"], a["nb"], ptrs, pose, 16,
                                 a["n"], a["r"], 16, None, None, None)
    assert call(args(c=24)) == 1      # channels not 8/16/32/64
    assert call(args(nb=5)) == 1      # at most four neighbours
    assert call(args(n=2)) == 1       # at least three candidates
    assert call(args(r=0.0)) == 1     # empty range
    assert call(args(fi=8)) == 1      # features not 16-byte aligned
    assert call(args(w=0)) == 1


def test_anchor_blend_weight_equals_the_oracle(lib):
    # host-only: the blending weight of two anchors
    from oracle import anchors as an
    from paper_2506_05558_amd import gsmi
    for d1, d2, o in [(1.0, 3.0, 0.1), (0.95, 1.0, 0.1), (1.0, 1.0, 0.2), (0.7, 1.0, 0.4), (0.0, 2.0, 0.25)]:
        assert abs(gsmi.anchor_blend_weight(d1, d2, o) - an.blend_weight(d1, d2, o)) < 1e-6
    w = C.c_float()
    L = gsmi._lib
    assert L.gs_anchor_blend_weight(2.0, 1.0, 0.1, C.byref(w)) == 1    # d1 > d2
    assert L.gs_anchor_blend_weight(1.0, 2.0, 0.5, C.byref(w)) == 1    # overlap not below 0.5
    assert L.gs_scale_opacity(1, 10, 1.5, 1, None) == 1                # w > 1
    assert L.gs_anchor_sizes(1, 1, 10, None, 1.0, 1.0, None, 1, None) == 1  # no pose


def test_adjoint_adam_validation(lib):
    """gs_project_bwd_views_adam rejects bad settings on the host, before
    anything is launched, and the projection rejects a misaligned binning
    plane (no GPU needed: every call below fails its checks)."""
    from paper_2506_05558_amd import gsmi as g
    L = g._lib
    L.gs_last_error.restype = C.c_char_p
    fake = [16 * (k + 1) for k in range(5)]  # non-NULL planes: validation fails before they are used
    gau = g._Gauss(10, 0, *fake, None)
    m1 = g._Gauss(10, 0, *fake, None)
    m2 = g._Gauss(10, 0, *fake, None)
    short = g._Gauss(9, 0, *fake, None)
    prm = g._Params(0.3, 0.99, 1 / 255, 1e-4, 1.3, 0)
    ok = dict(lr_means=1e-3, lr_log_scales=1e-3, lr_quats=1e-3, lr_opacity=1e-2, lr_sh_dc=1e-3, lr_sh_rest=1e-4,
              beta1=0.9, beta2=0.999, eps=1e-15, step=1, lr_decay=0.99)

    def call(opt, gm=gau, a=m1, b=m2, visible=64):
        o = None if opt is None else C.byref(g._AdamGroups(**opt))
        return L.gs_project_bwd_views_adam(0, None, C.byref(prm), C.byref(gm), C.byref(a), C.byref(b), None, o,
                                           C.byref(gau), None, 0, visible, None)

    assert call(None) == g.GS_ERR_INVALID_ARG and b"optimiser" in L.gs_last_error()
    assert call(dict(ok, step=0)) == g.GS_ERR_INVALID_ARG and b"step" in L.gs_last_error()
    assert call(dict(ok, beta1=1.0)) == g.GS_ERR_INVALID_ARG
    assert call(dict(ok, eps=-1.0)) == g.GS_ERR_INVALID_ARG
    assert call(dict(ok, lr_decay=0.0)) == g.GS_ERR_INVALID_ARG and b"lr_decay" in L.gs_last_error()
    assert call(dict(ok, lr_decay=1.5)) == g.GS_ERR_INVALID_ARG
    assert call(ok, a=short) == g.GS_ERR_INVALID_ARG and b"moment" in L.gs_last_error()
    assert call(ok, visible=None) == g.GS_ERR_INVALID_ARG and b"visible" in L.gs_last_error()
    # the binning plane of a projection must be 16-byte aligned
    cam = g._Camera(10, 10, 1.0, 1.0, 0.0, 0.0, 0.2, (C.c_float * 3)(0, 0, 0), 16)
    prj = g._Proj(16, 32, 48, 8)
    assert L.gs_project(C.byref(cam), C.byref(prm), C.byref(gau), C.byref(prj), None) == g.GS_ERR_INVALID_ARG
    assert b"16-byte" in L.gs_last_error()
