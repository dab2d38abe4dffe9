"""Batched rendering (one persistent integrator launch for many requests,
optionally replayed from a hipGraph) against per-request bh_render, which the
parity tests pin to the oracle; graph replays; latency statistics; autotuner."""
import json

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


def mixed_frames():
    """Ragged sizes (not multiples of the block or chunk), with and without a
    disk, different masses and distances, one 1x1 request."""
    out = []
    sizes = [(33, 17), (64, 64), (1, 1), (128, 96), (200, 150), (57, 301), (96, 96), (250, 250)]
    rng = np.random.default_rng(12)
    tex = inputs.sky_texture(128, 64, seed=9)
    for k, (w, h) in enumerate(sizes):
        M = float(rng.uniform(0.5, 2.0))
        rho = float(rng.uniform(15.0, 120.0))
        disk = (6.0, 20.0) if k % 2 == 0 else None
        cam = inputs.Camera(rho * M, float(rng.uniform(0, 90)), float(rng.uniform(0, 360)), 60.0, w, h)
        sc = inputs.scene_in_m(M, disk)
        if k in (3, 6):  # two requests with a sky image instead of the checker
            sc = inputs.Scene(M=sc.M, r_sky=sc.r_sky, disk=sc.disk, sky_tex=tex)
        out.append(inputs.Frame(cam, sc, f"m{k}"))
    return out


def _single(bh, frames, precision):
    import torch
    imgs = []
    for f in frames:
        rgba, _ = bh.render(f.camera, f.scene, bh.options(precision=precision))
        imgs.append(rgba)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in imgs]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("graph", [False, True])
def test_batch_equals_per_request_renders(bh, precision, graph):
    import torch
    p = bh.FP64 if precision == "fp64" else bh.FP32
    frames = mixed_frames()
    want = _single(bh, frames, p)
    b = bh.Batch(frames, bh.options(precision=p), use_graph=graph)
    b.launch()
    torch.cuda.synchronize()
    for k, (img, ref) in enumerate(zip(b.images, want)):
        np.testing.assert_array_equal(img.cpu().numpy(), ref, err_msg=f"request {k}")
    st = b.stats()
    assert st["requests"] == len(frames) and st["rays"] == b.rays
    assert 0 <= st["min_ms"] <= st["p50_ms"] <= st["p99_ms"] <= st["makespan_ms"]
    lat = b.latencies()
    assert np.all(lat >= 0) and abs(lat.max() - st["makespan_ms"]) < 1e-9
    b.close()


@pytest.mark.parametrize("precision,graph", [("fp32", True), ("fp64", False)])
def test_batch_matches_oracle(bh, ref, precision, graph):
    """Batched images against the CPU oracle directly: the 8 mixed small
    requests (every pixel) and every 32nd request of the 512-request serving
    mix at its real resolution (128^2 .. 2048^2; 12 rows spread over each
    image), traced together as one batch.  Batches return images only, so
    the comparison is by colour outside the ambiguity zones (critical band
    within 1e-3 M of b_c, checker edges, disk edges read back from the disk
    colour); elsewhere a class or exit error beyond the path's bound changes
    the colour and fails."""
    import torch
    from parity import compare_image
    from test_gpu_parity import ref_camera, ref_scene
    frames = mixed_frames() + inputs.serving_batch(512)[::32]
    p = bh.FP64 if precision == "fp64" else bh.FP32
    b = bh.Batch(frames, bh.options(precision=p), use_graph=graph)
    b.launch()
    torch.cuda.synchronize()
    compared = 0
    for k, (f, img) in enumerate(zip(frames, b.images)):
        W, H = f.camera.width, f.camera.height
        small = W * H <= 250 * 250
        rows = list(range(H)) if small else sorted(set(np.linspace(0, H - 1, 12).astype(int)))
        r_rgba, r_rays = ref.render_row_list(ref_camera(ref, f.camera), ref_scene(ref, f.scene), rows)
        mask = np.zeros(W * H, bool)
        for r0 in rows:
            mask[r0 * W:(r0 + 1) * W] = True
        compared += compare_image(r_rgba, r_rays, img.cpu().numpy(), f.scene, precision, mask=mask,
                                  sky_tex=f.scene.sky_tex)
    b.close()
    print(f"{len(frames)} requests, {compared} pixels compared with the oracle")
    assert compared > 100_000


def edge_frames():
    """Requests at the edges of the scene constants: flat space (M = 0: no
    horizon, an infinite FP32 horizon threshold), a camera at 400 M with a
    disk out to 300 M, one just outside the photon sphere, a 150-degree field
    of view, and a frame larger than one shading chunk."""
    return [
        inputs.Frame(inputs.Camera(30.0, 90.0, 0.0, 60.0, 48, 32),
                     inputs.Scene(M=0.0, r_sky=1000.0, disk=(2.0, 12.0)), "flat"),
        inputs.Frame(inputs.Camera(400.0, 63.0, 17.0, 70.0, 72, 40), inputs.scene_in_m(1.0, (6.0, 300.0)), "far"),
        inputs.Frame(inputs.Camera(3.5, 63.0, 17.0, 90.0, 72, 40), inputs.scene_in_m(1.0, (6.0, 20.0)), "near"),
        inputs.Frame(inputs.Camera(40.0, 63.0, 17.0, 150.0, 72, 40), inputs.scene_in_m(1.0, None), "wide"),
        inputs.Frame(inputs.Camera(25.0, 80.0, 5.0, 60.0, 300, 200), inputs.scene_in_m(2.0, (6.0, 30.0)), "big"),
    ]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("graph", [False, True])
def test_batch_edge_requests_equal_single_renders(bh, precision, graph):
    """FP32 batches keep FP32 start and result records; their pixels must
    still equal single renders bit for bit at the extremes of the scene
    constants, FP64 batches likewise."""
    import torch
    p = bh.FP64 if precision == "fp64" else bh.FP32
    frames = edge_frames()
    want = _single(bh, frames, p)
    b = bh.Batch(frames, bh.options(precision=p), use_graph=graph)
    for _ in range(2):
        b.launch()
        torch.cuda.synchronize()
        for k, (img, ref) in enumerate(zip(b.images, want)):
            np.testing.assert_array_equal(img.cpu().numpy(), ref, err_msg=f"request {frames[k].name}")
    b.close()


def test_image_only_fp32_renders_equal_renders_with_outputs(bh):
    """An FP32 render that returns only the image keeps FP32 start and result
    records (as FP32 batches do), whose r_hit also carries the end class; one
    that also returns per-pixel outputs keeps FP64 records and the class word.
    The pixels must be the same bit for bit: ragged and 1x1 frames, disks, sky
    images, flat space, distant and close cameras, with and without the
    per-call statistics (the instrumented integrator), and with a step cap of
    6 that leaves many rays unresolved (black, where a misread class would
    give sky or disk), in single renders and in an FP32 batch."""
    import torch
    frames = mixed_frames() + edge_frames()
    capped = bh.options(precision=bh.FP32, max_steps=6)
    n_unresolved = 0
    refs = []
    for opt, tag in ((bh.options(precision=bh.FP32), "plain"),
                     (bh.options(precision=bh.FP32, collect_stats=1), "stats"),
                     (capped, "capped")):
        for f in frames:
            img, _ = bh.render(f.camera, f.scene, opt)
            ref, out = bh.render(f.camera, f.scene, opt, fields=("cls",))
            torch.cuda.synchronize()
            assert out is not None and "cls" in out
            np.testing.assert_array_equal(img.cpu().numpy(), ref.cpu().numpy(),
                                          err_msg=f"{f.name} {tag}")
            if tag == "capped":
                n_unresolved += int((out["cls"] == bh.UNRESOLVED).sum().item())
                refs.append(ref.cpu().numpy())
    assert n_unresolved > 1000, n_unresolved
    b = bh.Batch(frames, capped, use_graph=False)
    b.launch()
    torch.cuda.synchronize()
    for f, img, ref in zip(frames, b.images, refs):
        np.testing.assert_array_equal(img.cpu().numpy(), ref, err_msg=f"{f.name} batch capped")
    b.close()


def test_request_groups_must_fit_one_blocks_lds(bh):
    """A group's integrator stages its requests' FP32 constants in LDS, 32
    bytes each: 6000 one-pixel requests in one group (192 KB) are refused at
    creation, and in two groups (96 KB each) they render as single renders."""
    import torch
    rng = np.random.default_rng(5)
    frames = []
    for k in range(6000):
        cam = inputs.Camera(float(rng.uniform(15.0, 90.0)), float(rng.uniform(0, 90)),
                            float(rng.uniform(0, 360)), 40.0, 1, 1)
        frames.append(inputs.Frame(cam, inputs.scene_in_m(1.0, (6.0, 20.0) if k % 2 else None), f"p{k}"))
    with pytest.raises(bh.BhError) as err:
        bh.Batch(frames, bh.options(precision=bh.FP32, batch_groups=1), use_graph=False)
    assert err.value.status == bh.BH_ERR_ARG and "batch_groups" in str(err.value)
    b = bh.Batch(frames, bh.options(precision=bh.FP32, batch_groups=2), use_graph=False)
    b.launch()
    torch.cuda.synchronize()
    assert b.stats()["requests"] == 6000
    for k in range(0, 6000, 997):
        want = _single(bh, [frames[k]], bh.FP32)[0]
        np.testing.assert_array_equal(b.images[k].cpu().numpy(), want, err_msg=f"request {k}")
    b.close()


@pytest.mark.parametrize("graph", [False, True])
def test_batch_groups(bh, graph):
    """Requests split into up to 3 consecutive groups traced one after another:
    pixels still equal the per-request renders, every request completes, and a
    later group's requests complete after every request of an earlier group."""
    import torch
    frames = mixed_frames()
    want = _single(bh, frames, bh.FP32)
    b = bh.Batch(frames, bh.options(precision=bh.FP32, batch_groups=3), use_graph=graph)
    b.launch()
    torch.cuda.synchronize()
    for k, (img, ref) in enumerate(zip(b.images, want)):
        np.testing.assert_array_equal(img.cpu().numpy(), ref, err_msg=f"request {k}")
    lat = b.latencies()
    assert np.all(lat >= 0)
    # group boundaries: consecutive requests, about equal ray counts
    rays = np.array([f.camera.pixels for f in frames], dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(rays)])
    bounds = [0]
    for r in range(1, len(frames)):
        if len(bounds) < 3 and off[r] * 3 >= off[-1] * len(bounds):
            bounds.append(r)
    bounds.append(len(frames))
    assert len(bounds) >= 3  # the last request holds 46% of the rays: 2 groups here
    for g in range(len(bounds) - 2):
        assert lat[bounds[g]:bounds[g + 1]].max() <= lat[bounds[g + 1]:bounds[g + 2]].min()
    b.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_orbit4k_batch_equals_per_frame_renders(bh, precision):
    """The benchmark's launch configuration: the 16 orbit frames at 3840x2160
    as one batch in one group.  Its pixels equal those of one bh_render call
    per frame bit for bit (and test_orbit4k_frame_sampled_rows holds those to
    the oracle at this size)."""
    import torch
    p = bh.FP64 if precision == "fp64" else bh.FP32
    frames = inputs.orbit_4k()
    opt = bh.options(precision=p, batch_groups=1)
    want = []
    for f in frames:
        rgba, _ = bh.render(f.camera, f.scene, opt)
        want.append(rgba)
    b = bh.Batch(frames, opt, use_graph=False)
    b.launch()
    torch.cuda.synchronize()
    for k, (img, ref) in enumerate(zip(b.images, want)):
        assert torch.equal(img, ref), f"frame {k}"
    assert b.stats()["requests"] == 16
    b.close()


@pytest.mark.parametrize("groups", [1, 3])
def test_batch_launches_are_timed(bh, groups):
    """With bh_timing enabled, an eager batch launch records one set-up, one
    integrator and one shading launch per group, each with a positive time; a
    replay of the captured graph records none."""
    import torch
    frames = mixed_frames()
    opt = bh.options(precision=bh.FP32, batch_groups=groups)
    b = bh.Batch(frames, opt, use_graph=False)
    bg = bh.Batch(frames, opt, use_graph=True)
    b.launch()
    bg.launch()
    torch.cuda.synchronize()
    bh.timing_enable(True)
    try:
        bh.timing_read()
        b.launch()
        torch.cuda.synchronize()
        t = bh.timing_read()
        n = t["setup"][1]
        assert 1 <= n <= groups
        for k in ("setup", "integrate", "shade"):
            assert t[k][1] == n and t[k][0] > 0.0, (k, t[k])
        assert t["surrogate"][1] == 0
        bg.launch()
        torch.cuda.synchronize()
        t = bh.timing_read()
        assert all(v[1] == 0 for v in t.values()), t
    finally:
        bh.timing_enable(False)
        b.close()
        bg.close()


def test_graph_replays_are_identical(bh):
    """The captured graph replayed several times, with eager work and
    synchronisation in between, reproduces the eager result every time."""
    import torch
    frames = mixed_frames()
    want = _single(bh, frames, bh.FP32)
    b = bh.Batch(frames, bh.options(precision=bh.FP32), use_graph=True)
    for rep in range(4):
        for img in b.images:
            img.fill_(-1.0)
        torch.cuda.synchronize()
        b.launch()
        torch.cuda.synchronize()
        for k, (img, ref) in enumerate(zip(b.images, want)):
            np.testing.assert_array_equal(img.cpu().numpy(), ref, err_msg=f"replay {rep} request {k}")
        # eager work between replays on the same device
        bh.render(frames[0].camera, frames[0].scene, bh.options(precision=bh.FP64))
        torch.cuda.synchronize()
    b.close()


def test_serving_batch_runs_and_reports(bh):
    """The 512-request serving mix at reduced resolution (sizes / 8): every
    pixel is written, and per-request completion times are recorded."""
    import torch
    frames = inputs.serving_batch(512, sizes=(16, 32, 64, 128, 256))
    b = bh.Batch(frames, bh.options(precision=bh.FP32), use_graph=True)
    b.launch()
    st = b.stats()
    assert st["requests"] == 512 and st["mrays_per_s"] > 0
    for img in b.images[:64]:
        a = img.cpu().numpy()
        assert np.all(a[..., 3] == 1.0)
    b.close()


def test_autotune_returns_a_candidate(bh, tmp_path):
    """The tuner times every knob (grid, chunk, refill threshold, groups)
    with device events, caches its pick, reuses the cache, and its pick
    renders the same pixels as the defaults."""
    import torch
    from paper_2507_16165_amd import autotune
    frames = mixed_frames()
    path = tmp_path / "tune.json"
    best = autotune.tune_batch(frames, bh.FP32, "mixed_small", cache_path=str(path), reps=3)
    assert best["chunk"] in autotune.CHUNKS and best["grid_blocks"] > 0
    assert best["refill"] in autotune.REFILLS_FP32 or best["refill"] == 20
    assert best["batch_groups"] in autotune.GROUPS or best["batch_groups"] == 0
    assert best["candidates_timed"] >= len(autotune.BLOCKS_PER_CU) + len(autotune.CHUNKS)
    cached = json.loads(path.read_text())
    assert list(cached.values())[0] == best
    # the cached entry is reused
    assert autotune.tune_batch(frames, bh.FP32, "mixed_small", cache_path=str(path)) == best
    want = _single(bh, frames, bh.FP32)
    b = bh.Batch(frames, autotune.options_for(best, bh.FP32), use_graph=True)
    b.launch()
    torch.cuda.synchronize()
    for k, (img, ref) in enumerate(zip(b.images, want)):
        np.testing.assert_array_equal(img.cpu().numpy(), ref, err_msg=f"request {k}")
    b.close()
