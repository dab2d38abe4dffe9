"""ctypes wrapper of the CPU FP64 oracle (``libbhref.so``).

TEST INFRASTRUCTURE ONLY.  Imported by the test suite, the smoke check and
the CPU-baseline leg of the benchmark; the product path never imports it.
It shares no code with the GPU library.  See ``bh_ref.h`` for what each
entry point computes and which passage of the paper it follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbhref.so")

SKY, CAPTURED, DISK, UNRESOLVED, INVALID = 0, 1, 2, 3, 4


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc: FP64, no contraction, no fast-math."""
    cmd = [
        "gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
        "-ffp-contract=off", "-fno-fast-math",
        os.path.join(HERE, "bh_ref.c"), "-o", LIB_PATH + ".tmp", "-lm",
    ]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class Scene(C.Structure):
    _fields_ = [("M", C.c_double), ("r_sky", C.c_double), ("has_disk", C.c_int),
                ("disk_rin", C.c_double), ("disk_rout", C.c_double),
                ("disk_power", C.c_double), ("checker_deg", C.c_double),
                ("sky_tex", C.c_void_p), ("tex_w", C.c_int), ("tex_h", C.c_int)]


class Camera(C.Structure):
    _fields_ = [("r", C.c_double), ("incl_deg", C.c_double), ("azim_deg", C.c_double),
                ("fov_deg", C.c_double), ("width", C.c_int), ("height", C.c_int)]


class Options(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol", C.c_double), ("h0", C.c_double),
                ("hmax", C.c_double), ("max_phi", C.c_double), ("max_steps", C.c_int),
                ("fixed_eps", C.c_double)]


class Out(C.Structure):
    _fields_ = [("cls", C.c_void_p), ("b", C.c_void_p), ("phi_end", C.c_void_p),
                ("exit_dir", C.c_void_p), ("r_hit", C.c_void_p), ("n_acc", C.c_void_p),
                ("n_rej", C.c_void_p), ("e_drift", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        L.bhr_max_threads.argtypes = []
        L.bhr_max_threads.restype = C.c_int
        L.bhr_default_options.argtypes = [C.POINTER(Options)]
        L.bhr_camera_ray.argtypes = [C.POINTER(Camera), C.c_int, C.c_int,
                                     C.c_void_p, C.c_void_p]
        L.bhr_trace_rays.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(Scene),
                                     C.POINTER(Options), C.POINTER(Out)]
        L.bhr_render_rows.argtypes = [C.POINTER(Camera), C.POINTER(Scene), C.POINTER(Options),
                                      C.c_int, C.c_int, C.c_void_p, C.POINTER(Out)]
        L.bhr_render_row_list.argtypes = [C.POINTER(Camera), C.POINTER(Scene), C.POINTER(Options),
                                          C.c_void_p, C.c_int, C.c_void_p, C.POINTER(Out)]
        L.bhr_set_threads.argtypes = [C.c_int]
        L.bhr_set_threads.restype = None
        L.bhr_shade.argtypes = [C.POINTER(Scene), C.c_int, C.c_void_p, C.c_double, C.c_void_p]
        L.bhr_sky_sample.argtypes = [C.POINTER(Scene), C.c_double, C.c_double, C.c_void_p]
        L.bhr_sky_sample.restype = None
        L.bhr_shade.restype = None
        L.bhr_dopri5_step.argtypes = [C.c_double, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p]
        L.bhr_dopri5_step.restype = None
        L.bhr_dphi_flat.argtypes = [C.c_double] * 4
        L.bhr_dphi_flat.restype = C.c_double
        _lib = L
    return _lib


def scene(M=1.0, r_sky=None, disk=None, disk_power=-3.0, checker_deg=10.0, sky_tex=None) -> Scene:
    """``r_sky`` defaults to 1000 M; ``disk`` is ``(r_in, r_out)`` or None;
    ``sky_tex`` an optional (tex_h, tex_w, 4) float32 equirectangular image
    (kept alive on the returned struct)."""
    if r_sky is None:
        r_sky = 1000.0 * M if M > 0 else 1000.0
    rin, rout = disk if disk is not None else (0.0, 0.0)
    s = Scene(M, r_sky, 1 if disk is not None else 0, rin, rout, disk_power, checker_deg, None, 0, 0)
    if sky_tex is not None:
        t = np.ascontiguousarray(sky_tex, dtype=np.float32)
        assert t.ndim == 3 and t.shape[2] == 4
        s.sky_tex, s.tex_h, s.tex_w = t.ctypes.data, t.shape[0], t.shape[1]
        s._tex = t
    return s


def sky_sample(sc: Scene, theta: float, varphi: float) -> np.ndarray:
    out = np.zeros(4)
    lib().bhr_sky_sample(C.byref(sc), C.c_double(theta), C.c_double(varphi), out.ctypes.data)
    return out


def camera(r, incl_deg, azim_deg, fov_deg, width, height) -> Camera:
    return Camera(r, incl_deg, azim_deg, fov_deg, int(width), int(height))


def options(rtol=1e-10, atol=0.0, h0=1e-2, hmax=1.0, max_phi=None, max_steps=1000000,
            fixed_eps=0.0) -> Options:
    o = Options()
    lib().bhr_default_options(C.byref(o))
    o.rtol, o.atol, o.h0, o.hmax, o.max_steps = rtol, atol, h0, hmax, max_steps
    o.fixed_eps = fixed_eps
    if max_phi is not None:
        o.max_phi = max_phi
    return o


@dataclass
class Rays:
    cls: np.ndarray
    b: np.ndarray
    phi_end: np.ndarray
    exit_dir: np.ndarray
    r_hit: np.ndarray
    n_acc: np.ndarray
    n_rej: np.ndarray
    e_drift: np.ndarray


def _alloc(n: int) -> tuple[Rays, Out]:
    r = Rays(np.zeros(n, np.uint8), np.zeros(n), np.zeros(n), np.zeros((n, 3)), np.zeros(n),
             np.zeros(n, np.int32), np.zeros(n, np.int32), np.zeros(n))
    out = Out(*[a.ctypes.data for a in (r.cls, r.b, r.phi_end, r.exit_dir, r.r_hit,
                                        r.n_acc, r.n_rej, r.e_drift)])
    return r, out


def trace_rays(origin, direction, sc: Scene, opt: Options | None = None) -> Rays:
    origin = np.ascontiguousarray(origin, dtype=np.float64).reshape(-1, 3)
    direction = np.ascontiguousarray(direction, dtype=np.float64).reshape(-1, 3)
    n = origin.shape[0]
    assert direction.shape[0] == n
    opt = opt or options()
    r, out = _alloc(n)
    rc = lib().bhr_trace_rays(origin.ctypes.data, direction.ctypes.data, n,
                              C.byref(sc), C.byref(opt), C.byref(out))
    if rc != 0:
        raise ValueError("bhr_trace_rays rejected its arguments")
    return r


def render(cam: Camera, sc: Scene, opt: Options | None = None, rows=None):
    """Render rows ``[row0, row1)`` (all by default).  Returns (rgba HxWx4 float32, Rays
    flattened over the full image; rows outside the range are zero)."""
    opt = opt or options()
    W, H = cam.width, cam.height
    row0, row1 = rows if rows is not None else (0, H)
    rgba = np.zeros((H, W, 4), np.float32)
    r, out = _alloc(W * H)
    rc = lib().bhr_render_rows(C.byref(cam), C.byref(sc), C.byref(opt), row0, row1,
                               rgba.ctypes.data, C.byref(out))
    if rc != 0:
        raise ValueError("bhr_render_rows rejected its arguments")
    return rgba, r


def render_row_list(cam: Camera, sc: Scene, rows, opt: Options | None = None):
    """Render the listed rows in one call (OpenMP over the list).  Returns
    (rgba HxWx4 float32, Rays over the full image; unlisted rows are zero)."""
    opt = opt or options()
    W, H = cam.width, cam.height
    rows = np.ascontiguousarray(rows, dtype=np.int32).ravel()
    rgba = np.zeros((H, W, 4), np.float32)
    r, out = _alloc(W * H)
    rc = lib().bhr_render_row_list(C.byref(cam), C.byref(sc), C.byref(opt), rows.ctypes.data,
                                   int(rows.size), rgba.ctypes.data, C.byref(out))
    if rc != 0:
        raise ValueError("bhr_render_row_list rejected its arguments")
    return rgba, r


def set_threads(n: int) -> None:
    """OpenMP threads of the oracle's batch loops from now on."""
    lib().bhr_set_threads(int(n))


def camera_rays(cam: Camera, pixels=None):
    """Origins and directions of the camera rays for the given flat pixel indices
    (all pixels by default)."""
    W, H = cam.width, cam.height
    idx = np.arange(W * H) if pixels is None else np.asarray(pixels).ravel()
    o = np.zeros((idx.size, 3))
    d = np.zeros((idx.size, 3))
    L = lib()
    for k, p in enumerate(idx):
        L.bhr_camera_ray(C.byref(cam), int(p % W), int(p // W),
                         o[k].ctypes.data, d[k].ctypes.data)
    return o, d


def shade(sc: Scene, cls: int, s, r_hit: float) -> np.ndarray:
    s = np.ascontiguousarray(s, dtype=np.float64)
    px = np.zeros(4, np.float32)
    lib().bhr_shade(C.byref(sc), int(cls), s.ctypes.data, float(r_hit), px.ctypes.data)
    return px


def dopri5_step(M: float, y, h: float):
    y = np.ascontiguousarray(y, dtype=np.float64)
    yo = np.zeros(2)
    e = np.zeros(2)
    lib().bhr_dopri5_step(M, y.ctypes.data, h, yo.ctypes.data, e.ctypes.data)
    return yo, e


def dphi_flat(M: float, b: float, r0: float, r_sky: float) -> float:
    return lib().bhr_dphi_flat(M, b, r0, r_sky)


def max_threads() -> int:
    """OpenMP threads the oracle's batch loops use."""
    return int(lib().bhr_max_threads())
