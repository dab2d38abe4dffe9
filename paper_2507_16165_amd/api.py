"""ctypes binding of libbh (include/bh.h).  Argument marshalling only: every
step of the path runs in the library's HIP kernels.  Tensors are torch CUDA
(HIP) tensors; work goes on torch's current stream unless one is given.
"""
from __future__ import annotations

import ctypes as C
import os

from . import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbh.so")

BH_OK, BH_ERR_ARG, BH_ERR_DEVICE, BH_ERR_NOMEM, BH_ERR_UNSUPPORTED, BH_ERR_STATE = 0, -1, -2, -3, -4, -5
SKY, CAPTURED, DISK, UNRESOLVED, INVALID = 0, 1, 2, 3, 4
PATH_NONE, PATH_FP64, PATH_FP32, PATH_SURROGATE = 0, 1, 2, 3
FP64, FP32 = 0, 1


class BhError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"bh status {status}: {msg}")
        self.status = status


class Scene(C.Structure):
    _fields_ = [("M", C.c_double), ("r_sky", C.c_double), ("has_disk", C.c_int),
                ("disk_rin", C.c_double), ("disk_rout", C.c_double),
                ("disk_power", C.c_double), ("checker_deg", C.c_double),
                ("sky_tex", C.c_void_p), ("tex_w", C.c_int), ("tex_h", C.c_int)]


class Camera(C.Structure):
    _fields_ = [("r", C.c_double), ("incl_deg", C.c_double), ("azim_deg", C.c_double),
                ("fov_deg", C.c_double), ("width", C.c_int), ("height", C.c_int)]


class Options(C.Structure):
    _fields_ = [("precision", C.c_int), ("rtol", C.c_double), ("atol", C.c_double),
                ("rtol_fp32", C.c_double), ("band_halfwidth", C.c_double), ("h0", C.c_double),
                ("h0_fp32", C.c_double),
                ("hmax", C.c_double), ("max_phi", C.c_double), ("max_steps", C.c_int),
                ("analytic_capture", C.c_int), ("grid_blocks", C.c_int), ("chunk", C.c_int),
                ("samples_side", C.c_int), ("batch_groups", C.c_int), ("fixed_eps", C.c_double),
                ("surrogate", C.c_void_p), ("refill_fp32", C.c_int), ("refill_fp64", C.c_int),
                ("collect_stats", C.c_int), ("rtol_fp32_growth", C.c_double),
                ("rtol_band", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("rays", C.c_int64), ("cls", C.c_int64 * 5), ("path", C.c_int64 * 4),
                ("step_evals", C.c_int64), ("accepted", C.c_int64 * 2),
                ("rejected", C.c_int64 * 2), ("newton", C.c_int64 * 2),
                ("capped", C.c_int64 * 2), ("sur_listed", C.c_int64),
                ("sur_fallback", C.c_int64), ("sur_untrusted", C.c_int64),
                ("timeline_waves", C.c_int64), ("wave_enter_us", C.c_double * 3),
                ("queue_dry_us", C.c_double * 3), ("wave_exit_us", C.c_double * 3)]


class Request(C.Structure):
    _fields_ = [("cam", Camera), ("scene", Scene), ("rgba", C.c_void_p)]


class BatchSummary(C.Structure):
    _fields_ = [("requests", C.c_int64), ("rays", C.c_int64), ("makespan_ms", C.c_double),
                ("p50_ms", C.c_double), ("p99_ms", C.c_double), ("min_ms", C.c_double),
                ("mrays_per_s", C.c_double)]


class Adam(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float)]


class RayOut(C.Structure):
    _fields_ = [("cls", C.c_void_p), ("b", C.c_void_p), ("phi_end", C.c_void_p),
                ("exit_dir", C.c_void_p), ("r_hit", C.c_void_p), ("steps", C.c_void_p),
                ("path", C.c_void_p)]


_lib = None


def lib():
    """Loads libbh.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = C.CDLL(LIB_PATH)
    st = C.c_int
    L.bh_default_options.argtypes = [C.POINTER(Options)]
    L.bh_default_options.restype = st
    L.bh_trace_rays.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(Scene),
                                C.POINTER(Options), C.POINTER(RayOut), C.c_void_p]
    L.bh_trace_rays.restype = st
    L.bh_render.argtypes = [C.POINTER(Camera), C.POINTER(Scene), C.POINTER(Options), C.c_void_p,
                            C.POINTER(RayOut), C.c_void_p]
    L.bh_render.restype = st
    L.bh_render_noalloc.argtypes = L.bh_render.argtypes
    L.bh_render_noalloc.restype = st
    L.bh_reserve.argtypes = [C.c_int64]
    L.bh_reserve.restype = st
    L.bh_last_counts.argtypes = [C.POINTER(C.c_int64), C.c_void_p]
    L.bh_last_counts.restype = st
    L.bh_last_stats.argtypes = [C.POINTER(Stats), C.c_void_p]
    L.bh_last_stats.restype = st
    L.bh_timing_enable.argtypes = [C.c_int]
    L.bh_timing_enable.restype = st
    L.bh_timing_read.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    L.bh_timing_read.restype = st
    vp, i64 = C.c_void_p, C.c_int64
    sigs = {
        "bh_surrogate_create": [vp, i64, i64, C.POINTER(C.c_void_p)],
        "bh_surrogate_destroy": [vp],
        "bh_surrogate_params": [vp, C.c_int, vp, i64],
        "bh_surrogate_set_params": [vp, vp, vp, vp, C.c_int],
        "bh_surrogate_train_step": [vp, vp, vp, vp, vp, i64, C.POINTER(Adam), vp, vp],
        "bh_surrogate_infer": [vp, vp, vp, i64, vp, vp, vp],
        "bh_surrogate_labels": [vp, vp, vp, i64, vp, vp, vp],
        "bh_surrogate_build_trust": [vp, vp, vp, vp, i64, C.c_float, C.c_int, vp, vp, vp],
        "bh_surrogate_trust": [vp, vp, i64],
        "bh_surrogate_set_trust": [vp, vp, i64],
    }
    sigs.update({
        "bh_batch_create": [C.POINTER(Request), C.c_int, C.POINTER(Options), C.c_int,
                            C.POINTER(C.c_void_p)],
        "bh_batch_launch": [vp, vp],
        "bh_batch_stats": [vp, C.POINTER(BatchSummary)],
        "bh_batch_latencies": [vp, vp, C.c_int],
        "bh_batch_destroy": [vp],
    })
    for name, args in sigs.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = st
    L.bh_shutdown.argtypes = []
    L.bh_shutdown.restype = st
    L.bh_last_error.argtypes = []
    L.bh_last_error.restype = C.c_char_p
    _lib = L
    return L


def check(status: int) -> None:
    if status != BH_OK:
        raise BhError(status, lib().bh_last_error().decode(errors="replace"))


def options(**overrides) -> Options:
    o = Options()
    check(lib().bh_default_options(C.byref(o)))
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise AttributeError(f"bh_options has no field {k!r}")
        setattr(o, k, v)
    return o


_tex_cache = {}  # id(host image) -> (host image, device copy): the device copy lives as long


def sky_texture_device(tex):
    """Device copy (cached) of a (tex_h, tex_w, 4) float32 sky image; a torch
    CUDA tensor is used as it is."""
    import numpy as np
    import torch
    if isinstance(tex, torch.Tensor):
        assert tex.is_cuda and tex.dtype == torch.float32 and tex.is_contiguous()
        return tex
    hit = _tex_cache.get(id(tex))
    if hit is None or hit[0] is not tex:
        hit = (tex, torch.from_numpy(np.ascontiguousarray(tex, dtype=np.float32)).cuda())
        _tex_cache[id(tex)] = hit
    return hit[1]


def scene_struct(s: inputs.Scene) -> Scene:
    rin, rout = s.disk if s.disk is not None else (0.0, 0.0)
    sc = Scene(s.M, s.r_sky, 1 if s.disk is not None else 0, rin, rout, s.disk_power,
               s.checker_deg, None, 0, 0)
    if s.sky_tex is not None:
        t = sky_texture_device(s.sky_tex)
        sc.sky_tex, sc.tex_h, sc.tex_w = t.data_ptr(), t.shape[0], t.shape[1]
    return sc


def camera_struct(c: inputs.Camera) -> Camera:
    return Camera(c.r, c.incl_deg, c.azim_deg, c.fov_deg, int(c.width), int(c.height))


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


ALL_FIELDS = ("cls", "b", "phi_end", "exit_dir", "r_hit", "steps", "path")


def _alloc_out(n: int, fields, device):
    import torch
    shapes = {"cls": ((n,), torch.uint8), "b": ((n,), torch.float64),
              "phi_end": ((n,), torch.float64), "exit_dir": ((n, 3), torch.float64),
              "r_hit": ((n,), torch.float64), "steps": ((n,), torch.int32),
              "path": ((n,), torch.uint8)}
    t = {f: torch.empty(shapes[f][0], dtype=shapes[f][1], device=device) for f in fields}
    ro = RayOut(*[t[f].data_ptr() if f in t else None for f in ALL_FIELDS])
    return t, ro


def trace_rays(origin, direction, scene: inputs.Scene, opt: Options | None = None,
               fields=ALL_FIELDS, stream=None) -> dict:
    """origin, direction: float64 CUDA tensors of shape (n, 3)."""
    import torch
    assert origin.dtype == torch.float64 and direction.dtype == torch.float64
    origin = origin.contiguous()
    direction = direction.contiguous()
    n = origin.shape[0]
    assert direction.shape[0] == n
    if "cls" not in fields:
        fields = ("cls",) + tuple(fields)
    out, ro = _alloc_out(n, fields, origin.device)
    sc = scene_struct(scene)
    opt = opt or options()
    check(lib().bh_trace_rays(origin.data_ptr(), direction.data_ptr(), n, C.byref(sc),
                              C.byref(opt), C.byref(ro), _stream(stream)))
    return out


def render(camera: inputs.Camera, scene: inputs.Scene, opt: Options | None = None, rgba=None,
           fields=None, stream=None, device="cuda"):
    """Renders one frame.  Returns (rgba (H, W, 4) float32 tensor, per-pixel
    dict or None).  ``fields`` selects per-pixel outputs (None: none)."""
    import torch
    H, W = camera.height, camera.width
    if rgba is None:
        rgba = torch.empty((H, W, 4), dtype=torch.float32, device=device)
    assert rgba.dtype == torch.float32 and rgba.is_contiguous() and rgba.numel() == H * W * 4
    out, ro = (None, None)
    opt = opt or options()
    n = max(1, int(opt.samples_side))
    if fields:
        out, ro = _alloc_out(H * W * n * n, fields, rgba.device)  # one record per sample
    cam = camera_struct(camera)
    sc = scene_struct(scene)
    check(lib().bh_render(C.byref(cam), C.byref(sc), C.byref(opt), rgba.data_ptr(),
                          C.byref(ro) if ro is not None else None, _stream(stream)))
    return rgba, out


NOALLOC_MAX_RAYS = 1048576   # BH_NOALLOC_MAX_RAYS


def render_noalloc(camera: inputs.Camera, scene: inputs.Scene, rgba, opt: Options | None = None,
                   out=None, stream=None) -> None:
    """bh_render_noalloc: renders into the caller's ``rgba`` (H, W, 4) float32
    tensor and, if given, the per-pixel tensors of ``out`` (a dict as
    ``alloc_out`` returns); the library allocates nothing for the call."""
    H, W = camera.height, camera.width
    assert rgba.dtype.itemsize == 4 and rgba.is_contiguous() and rgba.numel() == H * W * 4
    ro = None
    if out is not None:
        ro = RayOut(*[out[f].data_ptr() if f in out else None for f in ALL_FIELDS])
    opt = opt or options()
    cam = camera_struct(camera)
    sc = scene_struct(scene)
    check(lib().bh_render_noalloc(C.byref(cam), C.byref(sc), C.byref(opt), rgba.data_ptr(),
                                  C.byref(ro) if ro is not None else None, _stream(stream)))


def alloc_out(n: int, fields=ALL_FIELDS, device="cuda") -> dict:
    """Per-ray output tensors of length n (caller-owned), keyed by field."""
    return _alloc_out(n, fields, device)[0]


def reserve(n: int) -> None:
    check(lib().bh_reserve(int(n)))


def last_counts(stream=None) -> dict:
    arr = (C.c_int64 * 4)()
    check(lib().bh_last_counts(arr, _stream(stream)))
    return {"setup": arr[0], "fp64": arr[1], "fp32": arr[2], "surrogate": arr[3]}


def last_stats(stream=None) -> dict:
    """bh_last_stats of the last render/trace (which must have run with
    collect_stats=1), as a dict; the FP64/FP32 pairs as {'fp64': .., 'fp32': ..}."""
    s = Stats()
    check(lib().bh_last_stats(C.byref(s), _stream(stream)))
    pair = lambda a: {"fp64": int(a[0]), "fp32": int(a[1])}
    return {"rays": s.rays, "cls": dict(zip(("sky", "captured", "disk", "unresolved", "invalid"),
                                            (int(x) for x in s.cls))),
            "path": dict(zip(("none", "fp64", "fp32", "surrogate"), (int(x) for x in s.path))),
            "step_evals": s.step_evals, "accepted": pair(s.accepted), "rejected": pair(s.rejected),
            "newton": pair(s.newton), "capped": pair(s.capped), "sur_listed": s.sur_listed,
            "sur_fallback": s.sur_fallback, "sur_untrusted": s.sur_untrusted,
            "timeline_waves": s.timeline_waves,
            "timeline_us": {k: [round(x, 2) for x in getattr(s, k)]
                            for k in ("wave_enter_us", "queue_dry_us", "wave_exit_us")}}


KERNEL_CLASSES = ("setup", "integrate", "shade", "surrogate")


def timing_enable(on: bool = True) -> None:
    check(lib().bh_timing_enable(1 if on else 0))


def timing_read() -> dict:
    """{class: (summed ms, launches)} since the previous read."""
    ms = (C.c_double * 4)()
    n = (C.c_int64 * 4)()
    check(lib().bh_timing_read(ms, n))
    return {k: (ms[i], n[i]) for i, k in enumerate(KERNEL_CLASSES)}


def shutdown() -> None:
    check(lib().bh_shutdown())


# -- surrogate -------------------------------------------------------------

NPARAM = 33666
TRUST_SHAPE = (256, 64)


class Surrogate:
    """Owner of a bh_surrogate handle (the network, its Adam state, its
    training scratch and trust map live on the device)."""

    def __init__(self, params, max_batch: int = 4096):
        import numpy as np
        p = np.ascontiguousarray(params, dtype=np.float32).ravel()
        h = C.c_void_p()
        check(lib().bh_surrogate_create(p.ctypes.data, p.size, int(max_batch), C.byref(h)))
        self.handle = h
        self.max_batch = int(max_batch)

    def close(self):
        if self.handle:
            check(lib().bh_surrogate_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get(self, which: int = 0):
        """0 params, 1 last gradient, 2 Adam m, 3 Adam v (host float32)."""
        import numpy as np
        out = np.empty(NPARAM, np.float32)
        check(lib().bh_surrogate_params(self.handle, which, out.ctypes.data, NPARAM))
        return out

    def set(self, params, m=None, v=None, step: int = 0):
        import numpy as np
        arrs = [None if a is None else np.ascontiguousarray(a, np.float32) for a in (params, m, v)]
        ptrs = [None if a is None else a.ctypes.data for a in arrs]
        check(lib().bh_surrogate_set_params(self.handle, ptrs[0], ptrs[1], ptrs[2], int(step)))

    def train_step(self, b, r0, phi, cap, lr, loss=None, beta1=0.9, beta2=0.999, eps=1e-8,
                   stream=None):
        hp = Adam(lr, beta1, beta2, eps)
        check(lib().bh_surrogate_train_step(self.handle, b.data_ptr(), r0.data_ptr(), phi.data_ptr(),
                                            cap.data_ptr(), b.numel(), C.byref(hp),
                                            loss.data_ptr() if loss is not None else None,
                                            _stream(stream)))

    def infer(self, b, r0, stream=None):
        import torch
        n = b.numel()
        y = torch.empty((n, 2), dtype=torch.float32, device=b.device)
        phi = torch.empty(n, dtype=torch.float64, device=b.device)
        check(lib().bh_surrogate_infer(self.handle, b.data_ptr(), r0.data_ptr(), n, y.data_ptr(),
                                       phi.data_ptr(), _stream(stream)))
        return y, phi

    def labels(self, b, r0, stream=None):
        import torch
        n = b.numel()
        phi = torch.empty(n, dtype=torch.float64, device=b.device)
        cap = torch.empty(n, dtype=torch.uint8, device=b.device)
        check(lib().bh_surrogate_labels(self.handle, b.data_ptr(), r0.data_ptr(), n, phi.data_ptr(),
                                        cap.data_ptr(), _stream(stream)))
        return phi, cap

    def build_trust(self, b, r0, phi, max_err: float, min_count: int = 3, stream=None):
        import torch
        n = b.numel()
        y = torch.empty((n, 2), dtype=torch.float32, device=b.device)
        pp = torch.empty(n, dtype=torch.float64, device=b.device)
        check(lib().bh_surrogate_build_trust(self.handle, b.data_ptr(), r0.data_ptr(), phi.data_ptr(),
                                             n, float(max_err), int(min_count), y.data_ptr(),
                                             pp.data_ptr(), _stream(stream)))

    def trust(self):
        import numpy as np
        m = np.empty(TRUST_SHAPE, np.uint8)
        check(lib().bh_surrogate_trust(self.handle, m.ctypes.data, m.size))
        return m

    def set_trust(self, m):
        import numpy as np
        m = np.ascontiguousarray(m, np.uint8)
        assert m.shape == TRUST_SHAPE
        check(lib().bh_surrogate_set_trust(self.handle, m.ctypes.data, m.size))


# -- batched rendering --------------------------------------------------------

class Batch:
    """A set of render requests traced together (one persistent integrator
    launch for all of them), optionally replayed from a captured hipGraph.
    ``frames`` are inputs.Frame; ``images`` the matching (H, W, 4) float32
    device tensors (allocated if None)."""

    def __init__(self, frames, opt: Options | None = None, use_graph: bool = True, images=None,
                 device="cuda"):
        import torch
        self.frames = list(frames)
        if images is None:
            images = [torch.empty((f.camera.height, f.camera.width, 4), dtype=torch.float32,
                                  device=device) for f in self.frames]
        self.images = images
        reqs = (Request * len(self.frames))()
        for k, (f, img) in enumerate(zip(self.frames, images)):
            assert img.dtype == torch.float32 and img.is_contiguous()
            assert img.numel() == f.camera.width * f.camera.height * 4
            reqs[k] = Request(camera_struct(f.camera), scene_struct(f.scene), img.data_ptr())
        self.opt = opt or options()
        h = C.c_void_p()
        check(lib().bh_batch_create(reqs, len(self.frames), C.byref(self.opt), 1 if use_graph else 0,
                                    C.byref(h)))
        self.handle = h

    @property
    def rays(self) -> int:
        return sum(f.camera.width * f.camera.height for f in self.frames)

    def launch(self, stream=None):
        check(lib().bh_batch_launch(self.handle, _stream(stream)))

    def stats(self) -> dict:
        st = BatchSummary()
        check(lib().bh_batch_stats(self.handle, C.byref(st)))
        return {k: getattr(st, k) for k, _ in BatchSummary._fields_}

    def latencies(self):
        import numpy as np
        out = np.empty(len(self.frames), np.float64)
        check(lib().bh_batch_latencies(self.handle, out.ctypes.data, len(self.frames)))
        return out

    def close(self):
        if self.handle:
            check(lib().bh_batch_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
