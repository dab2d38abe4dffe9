"""Autotuner for the batched path's launch shape and schedule.

Knobs: resident blocks per CU of the persistent integrator (its grid), the
queue chunk a wavefront takes per grab, the refill threshold of the main
queue (idle lanes a wavefront waits for before it starts new rays; the
FP32 threshold in FP32 mode, the FP64 one in FP64 mode), and the number of
consecutive request groups a batch is split into.  Every candidate computes
bit-identical images (a ray's arithmetic does not depend on the schedule);
only the time changes.

Search: coordinate descent from the library's defaults, one knob at a time,
two passes.  Each candidate is timed with device events around whole batch
launches on the launch stream: one warm-up launch, then the median of
``reps`` (>= 3) launches.  Results are cached in a JSON file keyed by GPU
architecture, precision and workload name.
"""
from __future__ import annotations

import json
import os

from . import api

BLOCKS_PER_CU = (4, 6, 8)
CHUNKS = (128, 256, 512, 1024)
REFILLS_FP32 = (1, 8, 14, 20, 28, 36)
REFILLS_FP64 = (1, 3, 6, 10)
GROUPS = (1, 2, 4, 8)
KNOBS = ("grid_blocks", "chunk", "refill", "batch_groups")


def _key(precision: int, workload: str) -> str:
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    return f"{arch}/{'fp32' if precision == api.FP32 else 'fp64'}/{workload}"


def _options(precision: int, cand: dict):
    kw = dict(precision=precision, grid_blocks=cand["grid_blocks"], chunk=cand["chunk"],
              batch_groups=cand["batch_groups"])
    kw["refill_fp32" if precision == api.FP32 else "refill_fp64"] = cand["refill"]
    return api.options(**kw)


def time_batch(frames, opt, images, reps: int = 3) -> float:
    """Median milliseconds of `reps` launches of one batch (after one warm-up),
    from device events recorded on the launch stream."""
    import torch
    b = api.Batch(frames, opt, use_graph=False, images=images)
    try:
        stream = torch.cuda.current_stream()
        b.launch(stream)
        times = []
        for _ in range(max(3, reps)):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            b.launch(stream)
            e1.record(stream)
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
    finally:
        b.close()
    times.sort()
    return times[len(times) // 2]


def tune_batch(frames, precision: int, workload: str, cache_path: str | None = None,
               reps: int = 3, cus: int | None = None, log=None, passes: int = 2) -> dict:
    """Best {'grid_blocks', 'chunk', 'refill', 'batch_groups', 'ms'} for a
    batch of frames; the cached entry is returned if present."""
    import torch
    key = _key(precision, workload)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            return cache[key]
    cus = cus or torch.cuda.get_device_properties(0).multi_processor_count
    images = [torch.empty((f.camera.height, f.camera.width, 4), dtype=torch.float32, device="cuda")
              for f in frames]
    space = {
        "grid_blocks": [cus * k for k in BLOCKS_PER_CU],
        "chunk": list(CHUNKS),
        "refill": list(REFILLS_FP32 if precision == api.FP32 else REFILLS_FP64),
        "batch_groups": [g for g in GROUPS if g <= len(frames)],
    }
    best = {"grid_blocks": cus * 8, "chunk": 512 if precision == api.FP32 else 256,
            "refill": 28 if precision == api.FP32 else 6,
            "batch_groups": 0}
    best["ms"] = time_batch(frames, _options(precision, best), images, reps)
    seen = {tuple(best[k] for k in KNOBS): best["ms"]}
    if log:
        log(f"autotune {key}: start {best}")
    for _ in range(passes):
        changed = False
        for knob in KNOBS:
            for v in space[knob]:
                cand = dict(best, **{knob: v})
                sig = tuple(cand[k] for k in KNOBS)
                if sig in seen:
                    continue
                ms = time_batch(frames, _options(precision, cand), images, reps)
                seen[sig] = ms
                if log:
                    log(f"autotune {key}: {knob}={v}: {ms:.3f} ms")
                if ms < best["ms"]:
                    best = dict(cand, ms=ms)
                    changed = True
        if not changed:
            break
    best["candidates_timed"] = len(seen)
    if cache_path:
        cache[key] = best
        os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return best


def options_for(best: dict, precision: int):
    """bh_options of a tuned entry."""
    return _options(precision, best)
