"""Autotuner for the persistent integrator's launch shape.

Times the library on a workload for each candidate (resident blocks per CU,
queue chunk) and keeps the fastest; results are cached in a JSON file keyed by
GPU architecture, precision and workload name.  Only launch parameters are
tuned: every candidate computes bit-identical results (each ray's arithmetic
does not depend on the schedule).
"""
from __future__ import annotations

import json
import os
import time

from . import api

BLOCKS_PER_CU = (4, 6, 8)
CHUNKS = (128, 256, 512, 1024)


def _key(precision: int, workload: str) -> str:
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    return f"{arch}/{'fp32' if precision == api.FP32 else 'fp64'}/{workload}"


def tune_batch(frames, precision: int, workload: str, cache_path: str | None = None,
               reps: int = 2, cus: int | None = None, log=None) -> dict:
    """Best {'grid_blocks', 'chunk', 'ms'} for a batch of frames."""
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
    best = None
    for bpc in BLOCKS_PER_CU:
        for chunk in CHUNKS:
            opt = api.options(precision=precision, grid_blocks=cus * bpc, chunk=chunk)
            b = api.Batch(frames, opt, use_graph=False, images=images)
            b.launch()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                b.launch()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / reps
            b.close()
            if log:
                log(f"autotune {key}: blocks/CU {bpc} chunk {chunk}: {ms:.3f} ms")
            if best is None or ms < best["ms"]:
                best = {"grid_blocks": cus * bpc, "chunk": chunk, "ms": ms}
    if cache_path:
        cache[key] = best
        os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return best
