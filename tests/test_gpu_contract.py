"""Library and benchmark contract on the GPU: device memory does not grow over
many calls, and the benchmark prints one JSON line with every field."""
import json
import os
import subprocess
import sys

import pytest

from paper_2507_16165_amd import inputs

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bh():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2507_16165_amd import api
    api.lib()
    return api


def test_no_device_memory_growth_over_many_calls(bh):
    """10^4 bh_render calls (FP32 and FP64 alternating) and 200 batches
    created, launched and destroyed leave device memory where it was."""
    import torch
    f = inputs.Frame(inputs.Camera(30.0, 80.0, 20.0, 60.0, 8, 8), inputs.scene_in_m(1.0, (6.0, 20.0)))
    opts = (bh.options(precision=bh.FP64), bh.options(precision=bh.FP32))
    rgba = torch.empty((8, 8, 4), dtype=torch.float32, device="cuda")

    def renders(n):
        for i in range(n):
            bh.render(f.camera, f.scene, opts[i % 2], rgba=rgba)
        torch.cuda.synchronize()

    def batches(n):
        for i in range(n):
            b = bh.Batch([f, f, f], opts[1], use_graph=(i % 2 == 0))
            b.launch()
            torch.cuda.synchronize()
            b.close()

    renders(100)
    batches(2)
    free0 = torch.cuda.mem_get_info()[0]
    renders(10000)
    batches(200)
    free1 = torch.cuda.mem_get_info()[0]
    assert free0 - free1 < (8 << 20), (free0, free1)


def test_bench_prints_one_line_with_every_field():
    """bench.py on one 4K frame with a small CPU sample: exit status 0 and one
    JSON line on stdout carrying the contract's fields."""
    cmd = [sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--frames", "1", "--steps", "2",
           "--warmup", "1", "--fp64-steps", "1", "--no-surrogate", "--no-batch", "--no-paper",
           "--no-accuracy", "--cpu-row-stride", "540"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1 and lines[0].startswith("{"), r.stdout[-2000:]
    j = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
              "roofline", "cpu_baseline"):
        assert k in j, k
    assert j["n_gpus"] == 1 and j["steps"] == 2 and j["warmup"] == 1
    assert j["value"] > 0 and j["higher_is_better"] is True and j["config"]["workload"]
    assert j["config"]["rays_per_step"] == 3840 * 2160
    rf = j["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in rf, k
    assert rf["bound"] == "alu" and rf["unit"] == "TFLOP/s" and 0.0 < rf["frac"] < 1.0
    assert rf["traffic"] is None  # the committed counters are for the 16-frame workload
    cb = j["cpu_baseline"]
    for k in ("value", "unit", "cores", "kind", "sample"):
        assert k in cb, k
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["cores"] >= 1
