"""C-ABI contract checks that need no GPU: the library loads, exports every
entry point include/bh.h declares, fills defaults, and rejects bad arguments
before touching the device."""
import ctypes as C
import os
import re

import pytest

from paper_2507_16165_amd import api, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]*?\b(bh_\w+)\s*\(", txt, flags=re.M))
    return names


def test_library_exports_every_declared_symbol():
    L = api.lib()
    names = declared_symbols()
    assert {"bh_trace_rays", "bh_render", "bh_default_options", "bh_last_error"} <= names
    for n in sorted(names):
        assert hasattr(L, n), f"{n} declared in include/ but not exported"


def test_defaults():
    o = api.options()
    assert o.precision == api.FP64 and o.rtol == 1e-10 and o.atol == 0.0
    assert o.rtol_fp32 == 1e-6 and o.band_halfwidth == 0.05 and o.max_steps == 1000000
    assert o.rtol_fp32_growth == 50.0 and o.rtol_band == 1e-9
    assert o.h0 == 1e-2 and o.h0_fp32 == 0.2
    assert abs(o.max_phi - 8 * 3.141592653589793) < 1e-12 and o.analytic_capture == 1


def _render(cam, sc, opt=None, rgba=1):
    L = api.lib()
    c = api.camera_struct(cam)
    s = api.scene_struct(sc)
    o = opt or api.options()
    return L.bh_render(C.byref(c), C.byref(s), C.byref(o), C.c_void_p(rgba), None, None)


@pytest.mark.parametrize("cam,sc,msg", [
    (inputs.Camera(2.5, 90, 0, 60, 8, 8), inputs.Scene(M=1.0), "photon sphere"),
    (inputs.Camera(30, 90, 0, 0.0, 8, 8), inputs.Scene(M=1.0), "fov"),
    (inputs.Camera(30, 90, 0, 180.0, 8, 8), inputs.Scene(M=1.0), "fov"),
    (inputs.Camera(30, 90, 0, 60, 0, 8), inputs.Scene(M=1.0), "width"),
    (inputs.Camera(30, 90, 0, 60, 8, 8), inputs.Scene(M=-1.0), "M must"),
    (inputs.Camera(30, 90, 0, 60, 8, 8), inputs.Scene(M=1.0, disk=(20.0, 6.0)), "disk"),
    (inputs.Camera(3000, 90, 0, 60, 8, 8), inputs.Scene(M=1.0), "sky"),
])
def test_render_rejects_bad_arguments(cam, sc, msg):
    st = _render(cam, sc)
    assert st == api.BH_ERR_ARG
    assert msg in api.lib().bh_last_error().decode()


def test_render_rejects_null_and_bad_options():
    cam, sc = inputs.Camera(30, 90, 0, 60, 8, 8), inputs.Scene(M=1.0)
    assert _render(cam, sc, rgba=0) == api.BH_ERR_ARG
    assert _render(cam, sc, api.options(precision=7)) == api.BH_ERR_ARG
    assert _render(cam, sc, api.options(rtol=-1.0)) == api.BH_ERR_ARG
    assert _render(cam, sc, api.options(chunk=100)) == api.BH_ERR_ARG
    assert _render(cam, sc, api.options(max_steps=0)) == api.BH_ERR_ARG
    assert _render(cam, sc, api.options(h0_fp32=0.0)) == api.BH_ERR_ARG
    assert _render(cam, sc, api.options(samples_side=17)) == api.BH_ERR_ARG
    assert _render(cam, sc, api.options(samples_side=-1)) == api.BH_ERR_ARG
    assert _render(cam, sc, api.options(batch_groups=-1)) == api.BH_ERR_ARG
    assert _render(cam, sc, api.options(fixed_eps=-1.0)) == api.BH_ERR_ARG
    assert _render(cam, sc, api.options(refill_fp32=65)) == api.BH_ERR_ARG
    assert _render(cam, sc, api.options(refill_fp64=-1)) == api.BH_ERR_ARG
    assert _render(cam, sc, api.options(rtol_fp32_growth=0.5)) == api.BH_ERR_ARG
    assert _render(cam, sc, api.options(rtol_fp32_growth=2e4)) == api.BH_ERR_ARG
    assert _render(cam, sc, api.options(rtol_fp32_growth=float("nan"))) == api.BH_ERR_ARG
    assert _render(cam, sc, api.options(rtol_band=0.0)) == api.BH_ERR_ARG
    assert _render(cam, sc, api.options(rtol_band=float("inf"))) == api.BH_ERR_ARG
    assert _render(cam, sc, api.options(fixed_eps=0.5, precision=api.FP32)) == api.BH_ERR_UNSUPPORTED
    L = api.lib()
    assert L.bh_render(None, None, None, None, None, None) == api.BH_ERR_ARG
    assert L.bh_default_options(None) == api.BH_ERR_ARG


def test_trace_rays_argument_checks():
    L = api.lib()
    s = api.scene_struct(inputs.Scene(M=1.0))
    o = api.options()
    out = api.RayOut()
    # no cls output
    assert L.bh_trace_rays(None, None, 4, C.byref(s), C.byref(o), C.byref(out), None) == api.BH_ERR_ARG
    # n = 0 is a no-op that touches nothing, even with no outputs
    assert L.bh_trace_rays(None, None, 0, C.byref(s), C.byref(o), C.byref(out), None) == api.BH_OK
    out.cls = 1
    assert L.bh_trace_rays(None, None, -1, C.byref(s), C.byref(o), C.byref(out), None) == api.BH_ERR_ARG
    assert L.bh_trace_rays(None, None, 4, C.byref(s), C.byref(o), C.byref(out), None) == api.BH_ERR_ARG
    # n = 0 is a no-op that touches nothing
    assert L.bh_trace_rays(None, None, 0, C.byref(s), C.byref(o), C.byref(out), None) == api.BH_OK


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(api, "_lib", None)
    monkeypatch.setattr(api, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(RuntimeError, match="missing"):
        api.lib()


def test_output_marshalling_on_host_tensors():
    """The binding's output allocation and pointer packing (host tensors)."""
    t, ro = api._alloc_out(10, api.ALL_FIELDS, "cpu")
    assert t["exit_dir"].shape == (10, 3) and t["cls"].dtype.itemsize == 1
    assert ro.exit_dir == t["exit_dir"].data_ptr() and ro.steps == t["steps"].data_ptr()
    t, ro = api._alloc_out(4, ("cls",), "cpu")
    assert ro.b is None and ro.cls == t["cls"].data_ptr()


def test_batch_argument_checks():
    """Batch creation rejects bad arguments before touching the device."""
    L = api.lib()
    h = C.c_void_p()
    o = api.options()
    assert L.bh_batch_create(None, 0, C.byref(o), 0, C.byref(h)) == api.BH_ERR_ARG
    reqs = (api.Request * 1)()
    reqs[0] = api.Request(api.camera_struct(inputs.Camera(2.0, 90, 0, 60, 8, 8)),
                          api.scene_struct(inputs.Scene(M=1.0)), 1)
    assert L.bh_batch_create(reqs, 1, C.byref(o), 0, C.byref(h)) == api.BH_ERR_ARG
    assert "request 0" in L.bh_last_error().decode()
    reqs[0] = api.Request(api.camera_struct(inputs.Camera(30.0, 90, 0, 60, 8, 8)),
                          api.scene_struct(inputs.Scene(M=1.0)), None)
    assert L.bh_batch_create(reqs, 1, C.byref(o), 0, C.byref(h)) == api.BH_ERR_ARG
    o2 = api.options(samples_side=2)
    assert L.bh_batch_create(reqs, 1, C.byref(o2), 0, C.byref(h)) == api.BH_ERR_UNSUPPORTED
    o3 = api.options(fixed_eps=0.5)
    assert L.bh_batch_create(reqs, 1, C.byref(o3), 0, C.byref(h)) == api.BH_ERR_UNSUPPORTED
    o4 = api.options(collect_stats=1)
    assert L.bh_batch_create(reqs, 1, C.byref(o4), 0, C.byref(h)) == api.BH_ERR_UNSUPPORTED
    assert L.bh_last_stats(None, None) == api.BH_ERR_ARG
    assert L.bh_batch_launch(None, None) == api.BH_ERR_ARG
    assert L.bh_batch_destroy(None) == api.BH_OK


def test_bench_refuses_more_than_one_gpu():
    """bench.py on N > 1 GPUs exits with status 2 and says why, before it
    touches a device."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_ctypes_structs_match_the_c_layout(tmp_path):
    """The binding's ctypes structures have the field offsets and sizes the C
    compiler gives the structs of include/bh.h (a field added on one side
    only would shift every later field)."""
    import subprocess
    structs = {"bh_scene": api.Scene, "bh_camera": api.Camera, "bh_options": api.Options,
               "bh_ray_out": api.RayOut, "bh_request": api.Request,
               "bh_batch_summary": api.BatchSummary, "bh_adam": api.Adam}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "bh.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    for line in filter(None, out):
        cname, field, val = line.split()
        py = structs[cname]
        want = C.sizeof(py) if field == "size" else getattr(py, field).offset
        assert int(val) == want, (cname, field, int(val), want)


def test_render_noalloc_rejects_frames_beyond_its_workspace():
    """bh_render_noalloc has a fixed workspace of BH_NOALLOC_MAX_RAYS rays:
    larger frames (samples included) are refused before any device call,
    with the same argument checks as bh_render first."""
    L = api.lib()
    sc = api.scene_struct(inputs.Scene(M=1.0))

    def call(cam, opt=None, rgba=1):
        c = api.camera_struct(cam)
        o = opt or api.options()
        return L.bh_render_noalloc(C.byref(c), C.byref(sc), C.byref(o), C.c_void_p(rgba), None, None)

    assert api.NOALLOC_MAX_RAYS == 1 << 20
    assert call(inputs.Camera(30, 90, 0, 60, 1025, 1024)) == api.BH_ERR_ARG
    assert "fixed workspace" in L.bh_last_error().decode()
    assert call(inputs.Camera(30, 90, 0, 60, 512, 512), api.options(samples_side=3)) == api.BH_ERR_ARG
    assert "fixed workspace" in L.bh_last_error().decode()
    assert call(inputs.Camera(2.5, 90, 0, 60, 8, 8)) == api.BH_ERR_ARG
    assert "photon sphere" in L.bh_last_error().decode()
    assert call(inputs.Camera(30, 90, 0, 60, 8, 8), rgba=0) == api.BH_ERR_ARG
    assert L.bh_render_noalloc(None, None, None, None, None, None) == api.BH_ERR_ARG


def test_size_limits_are_checked_before_any_device_call():
    """Frames, sample grids, ray counts and batches beyond the 32-bit ray
    index the kernels use are refused with BH_ERR_ARG (no device needed)."""
    L = api.lib()
    sc = api.scene_struct(inputs.Scene(M=1.0))
    o = api.options()
    big = api.camera_struct(inputs.Camera(30, 90, 0, 60, 65536, 32768))   # 2^31 pixels
    assert L.bh_render(C.byref(big), C.byref(sc), C.byref(o), C.c_void_p(1), None, None) == api.BH_ERR_ARG
    assert "2^31" in L.bh_last_error().decode()
    cam = api.camera_struct(inputs.Camera(30, 90, 0, 60, 16384, 16384))   # 2^28 pixels x 16 samples
    o16 = api.options(samples_side=4)
    assert L.bh_render(C.byref(cam), C.byref(sc), C.byref(o16), C.c_void_p(1), None, None) == api.BH_ERR_ARG
    assert "samples" in L.bh_last_error().decode()
    out = api.RayOut()
    out.cls = 1
    assert L.bh_trace_rays(C.c_void_p(1), C.c_void_p(1), 1 << 31, C.byref(sc), C.byref(o),
                           C.byref(out), None) == api.BH_ERR_ARG
    assert L.bh_reserve(-1) == api.BH_ERR_ARG and L.bh_reserve(1 << 31) == api.BH_ERR_ARG
    reqs = (api.Request * 2)()
    for k in range(2):
        reqs[k] = api.Request(api.camera_struct(inputs.Camera(30, 90, 0, 60, 32768, 32768)), sc, 1)
    h = C.c_void_p()
    assert L.bh_batch_create(reqs, 2, C.byref(o), 0, C.byref(h)) == api.BH_ERR_ARG
    assert "2^31" in L.bh_last_error().decode()
