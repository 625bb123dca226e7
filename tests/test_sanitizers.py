"""The FP64 oracle (C) built with AddressSanitizer and UndefinedBehaviourSanitizer
runs the rasterizer's forward, adjoint and crop renders on small scenes
(degree 0 and 3, the screen-space filter, a posed camera, Gaussians behind
the camera and off-image) without a sanitizer report, and its results equal
the normal build's bit for bit."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "gs_oracle.c")

SCRIPT = r"""
import hashlib, sys
import numpy as np
sys.path.insert(0, sys.argv[1])
from oracle import raster as orc
from paper_2506_05558_amd import synth
h = hashlib.sha256()
view, scene, target = synth.tiny_scene(3, n=400, size=48)
m = scene.means.copy(); m[2, :40] *= -1; m[0, 40:60] += 30.0   # behind the camera, off the image
scene = synth.Scene(m, scene.log_scales, scene.quats, scene.opacity_logits, scene.sh, 0)
for kw in (dict(), dict(eps2d=0.1, mip_filter=1)):
    cam, g = orc.Camera.from_view(view, **kw), orc.Gaussians.from_scene(scene)
    op, ref = orc.forward(cam, g, flag_rel=1e-5)
    gi = np.sign(ref["image"] - target) / target.size
    gr = orc.backward(cam, g, op, g_image=gi)
    for k in ("image", "depth", "alpha"):
        h.update(np.ascontiguousarray(ref[k]).tobytes())
    for k in sorted(gr):
        h.update(np.ascontiguousarray(gr[k]).tobytes())
v2, s2 = synth.single_view(5, width=96, height=64, n=3000)
cam, g = orc.Camera.from_view(v2), orc.Gaussians.from_scene(s2)
op = orc.project(cam, g)
r = orc.render(cam, op, crop=(40, 20, 17, 13), flag_rel=1e-5)
h.update(np.ascontiguousarray(r["image"]).tobytes())
print("digest", h.hexdigest())
"""


def _run(env):
    r = subprocess.run([sys.executable, "-c", SCRIPT, ROOT], capture_output=True, text=True, env=env, timeout=600)
    return r


@pytest.mark.slow
def test_oracle_under_asan_and_ubsan(tmp_path):
    so = str(tmp_path / "libgs_oracle_asan.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-fno-fast-math",
                           "-ffp-contract=off", "-o", so, SRC, "-lm", "-lpthread"])
    libasan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    assert os.path.exists(libasan), libasan
    base = dict(os.environ)
    base.pop("GS_ORACLE_LIB", None)
    plain = _run(base)
    assert plain.returncode == 0, plain.stderr[-2000:]
    env = dict(base, GS_ORACLE_LIB=so, LD_PRELOAD=libasan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    san = _run(env)
    assert san.returncode == 0, san.stderr[-4000:]
    assert "AddressSanitizer" not in san.stderr and "runtime error" not in san.stderr, san.stderr[-4000:]
    # -O1 and -O2 builds of the same C with contraction off give the same bits
    d_plain = [l for l in plain.stdout.splitlines() if l.startswith("digest")]
    d_san = [l for l in san.stdout.splitlines() if l.startswith("digest")]
    assert d_plain and d_plain == d_san


@pytest.mark.slow
def test_library_host_code_under_asan(tmp_path):
    """The HIP library with its host code (argument checks, workspace
    carving, error text) built with AddressSanitizer: the ABI's host-side
    tests run clean (no device work happens in them)."""
    import glob
    csrc = os.path.join(ROOT, "paper_2506_05558_amd", "csrc")
    inc = os.path.join(ROOT, "include")
    objs = []
    procs = []
    for src in sorted(glob.glob(os.path.join(csrc, "*.hip"))):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        objs.append(obj)
        procs.append(subprocess.Popen(
            ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", inc, "-c", src, "-o", obj],
            stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL))
    assert all(p.wait() == 0 for p in procs)
    so = str(tmp_path / "libgsmi_asan.so")
    subprocess.check_call(["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host",
                           "-fsanitize=address", "-o", so, *objs])
    rt = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    assert rt, "clang's ASan runtime is missing"
    env = dict(os.environ, GSMI_LIB=so, LD_PRELOAD=rt[0], ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_abi.py"), "-q", "-x",
                        "-p", "no:cacheprovider"], capture_output=True, text=True, env=env, cwd=ROOT, timeout=600)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
