"""bh_render_noalloc (the allocation-free variant of bh_render) against
bh_render through the C ABI: two calls in a row on the same GPU, the second
on a smaller frame, each bit-identical to bh_render of the same frame (image
and every per-pixel record), and device memory unchanged over further calls.
"""
import numpy as np
import pytest

from paper_2507_16165_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bh():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2507_16165_amd import api
    api.lib()
    return api


def _both(bh, frame, opt):
    """(bh_render result, bh_render_noalloc result), each as numpy arrays."""
    import torch
    H, W = frame.camera.height, frame.camera.width
    n = H * W * max(1, int(opt.samples_side)) ** 2
    ref_rgba, ref_out = bh.render(frame.camera, frame.scene, opt, fields=bh.ALL_FIELDS)
    rgba = torch.full((H, W, 4), -7.0, dtype=torch.float32, device="cuda")
    out = bh.alloc_out(n)
    for v in out.values():
        v.fill_(0x5A if v.dtype.itemsize == 1 else -3)
    bh.render_noalloc(frame.camera, frame.scene, rgba, opt, out=out)
    torch.cuda.synchronize()
    np_ = lambda d: {k: v.cpu().numpy() for k, v in d.items()}
    return (ref_rgba.cpu().numpy(), np_(ref_out)), (rgba.cpu().numpy(), np_(out))


def _same(a, b, what):
    (ra, oa), (rb, ob) = a, b
    assert ra.tobytes() == rb.tobytes(), f"{what}: images differ"
    for k in oa:
        assert oa[k].tobytes() == ob[k].tobytes(), f"{what}: per-pixel {k} differs"


def test_noalloc_equals_render_on_two_calls_in_a_row(bh):
    import torch
    # call 1: the largest frame the fixed workspace takes (1024 x 1024 rays),
    # disk scene, FP32 with the FP64 critical band
    big = inputs.disk_1024(1024)
    assert big.camera.width * big.camera.height == bh.NOALLOC_MAX_RAYS
    print(f"noalloc call 1: {big.camera.width}x{big.camera.height} fp32", flush=True)
    a, b = _both(bh, big, bh.options(precision=bh.FP32))
    _same(a, b, "1024x1024 FP32")
    assert (a[1]["path"] == bh.PATH_FP64).sum() > 0  # the band queue ran
    # call 2: a smaller, ragged frame with another camera, FP64, 2x2 samples
    # per pixel (the workspace still holds call 1's rays beyond it)
    small = inputs.Frame(inputs.Camera(25.0, 60.0, 40.0, 50.0, 151, 97),
                         inputs.scene_in_m(1.3, (6.0, 18.0)))
    print("noalloc call 2: 151x97 fp64, 2x2 samples", flush=True)
    a, b = _both(bh, small, bh.options(precision=bh.FP64, samples_side=2))
    _same(a, b, "151x97 FP64 2x2 samples")
    assert (a[1]["cls"] == bh.DISK).sum() > 0 and (a[1]["cls"] == bh.SKY).sum() > 0
    # call 3: smaller still, FP32, no disk
    tiny = inputs.Frame(inputs.Camera(40.0, 90.0, 0.0, 60.0, 37, 5), inputs.scene_in_m(0.7, None))
    print("noalloc call 3: 37x5 fp32", flush=True)
    a, b = _both(bh, tiny, bh.options(precision=bh.FP32))
    _same(a, b, "37x5 FP32")
    # further calls take no device memory
    rgba = torch.empty((97, 151, 4), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for i in range(50):
        bh.render_noalloc(small.camera, small.scene, rgba, bh.options(precision=i % 2))
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0


def test_noalloc_refuses_more_rays_than_its_workspace(bh):
    import torch
    f = inputs.Frame(inputs.Camera(30.0, 90.0, 0.0, 60.0, 1025, 1024), inputs.scene_in_m(1.0, None))
    rgba = torch.empty((1024, 1025, 4), dtype=torch.float32, device="cuda")
    with pytest.raises(bh.BhError) as e:
        bh.render_noalloc(f.camera, f.scene, rgba)
    assert e.value.status == bh.BH_ERR_ARG and "fixed workspace" in str(e.value)
