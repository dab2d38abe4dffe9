"""GPU path (through the C ABI) against the CPU FP64 oracle, element by element.

Workloads: the 64x64 plain frame, the 1024x1024 disk frame (FP64 and FP32 +
FP64 band), 4K orbit frames (sampled rows at full size, in the default launch
shape the benchmark times), random ray sets, and edge cases.
"""
import math

import numpy as np
import pytest

from paper_2507_16165_amd import inputs
from parity import B_CRIT, compare, compare_rgba

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bh():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2507_16165_amd import api
    api.lib()
    return api


def ref_scene(ref, s: inputs.Scene):
    return ref.scene(s.M, r_sky=s.r_sky, disk=s.disk, disk_power=s.disk_power,
                     checker_deg=s.checker_deg, sky_tex=s.sky_tex)


def ref_camera(ref, c: inputs.Camera):
    return ref.camera(c.r, c.incl_deg, c.azim_deg, c.fov_deg, c.width, c.height)


def np_out(d):
    return {k: v.cpu().numpy() for k, v in d.items()}


def gpu_render(bh, frame, precision, **kw):
    import torch
    opt = bh.options(precision=precision, **kw)
    rgba, out = bh.render(frame.camera, frame.scene, opt, fields=bh.ALL_FIELDS)
    torch.cuda.synchronize()
    return rgba.cpu().numpy(), np_out(out)


def oracle_rows(ref, frame, rows, rtol=1e-10):
    """Oracle on a set of image rows, one call over the list (OpenMP across
    the rows); full-image arrays, other rows zero."""
    cam, sc = ref_camera(ref, frame.camera), ref_scene(ref, frame.scene)
    W, H = frame.camera.width, frame.camera.height
    rows = sorted(set(int(r) for r in rows))
    rgba, rays = ref.render_row_list(cam, sc, rows, ref.options(rtol=rtol))
    mask = np.zeros(H * W, bool)
    for r0 in rows:
        mask[r0 * W:(r0 + 1) * W] = True
    return rgba, rays, mask


# ---------------------------------------------------------------------------
def test_plain64_fp64_full_image(bh, ref):
    f = inputs.plain_64()
    rgba, out = gpu_render(bh, f, bh.FP64)
    r_rgba, r_rays = ref.render(ref_camera(ref, f.camera), ref_scene(ref, f.scene))
    s = compare(r_rays, out, f.scene, "fp64")
    assert s["n"] == 4096 and s["captured"] >= 290
    compare_rgba(r_rgba, r_rays, rgba, out["cls"], f.scene, "fp64")
    assert (out["cls"] == bh.CAPTURED).sum() == 300  # closed-form shadow count


@pytest.mark.parametrize("size", [200, 1024])
def test_disk_frame_fp64(bh, ref, size):
    f = inputs.disk_1024(size)
    rgba, out = gpu_render(bh, f, bh.FP64)
    H = f.camera.height
    rows = range(H) if size <= 200 else sorted(set(np.linspace(0, H - 1, 40).astype(int)) | {H // 2})
    r_rgba, r_rays, mask = oracle_rows(ref, f, list(rows))
    s = compare(r_rays, out, f.scene, "fp64", mask=mask)
    assert s["disk"] > 0 and s["sky"] > 0
    compare_rgba(r_rgba, r_rays, rgba, out["cls"], f.scene, "fp64", mask=mask)


@pytest.mark.parametrize("size", [200, 1024])
def test_disk_frame_fp32_band(bh, ref, size):
    f = inputs.disk_1024(size)
    rgba, out = gpu_render(bh, f, bh.FP32)
    H = f.camera.height
    rows = range(H) if size <= 200 else sorted(set(np.linspace(0, H - 1, 40).astype(int)) | {H // 2})
    r_rgba, r_rays, mask = oracle_rows(ref, f, list(rows))
    s = compare(r_rays, out, f.scene, "fp32", mask=mask)
    compare_rgba(r_rgba, r_rays, rgba, out["cls"], f.scene, "fp32", mask=mask)
    # the critical band went through the FP64 integrator, the rest through FP32
    band = np.abs(out["b"] - B_CRIT * f.scene.M) < 0.05 * f.scene.M
    assert np.all(out["path"][band] == bh.PATH_FP64)
    assert np.all(out["path"][~band & (out["path"] != bh.PATH_NONE)] == bh.PATH_FP32)
    assert s["max_angle"] <= 1e-4


@pytest.mark.parametrize("growth", [1.0, 50.0, 100.0])
def test_fp32_tolerance_growth(bh, ref, growth):
    """FP32 rays' tolerance grows with |b - b_c| up to `growth` times the
    base (50 by default).  Every setting is held to the oracle at the FP32
    bounds on a 400x400 disk frame (every 8th row), growth 100 as a stress of
    the schedule; the grown tolerance takes fewer step evaluations per FP32
    ray."""
    f = inputs.disk_1024(400)
    rgba, out = gpu_render(bh, f, bh.FP32, rtol_fp32_growth=growth)
    rows = list(range(0, f.camera.height, 8))
    r_rgba, r_rays, mask = oracle_rows(ref, f, rows)
    s = compare(r_rays, out, f.scene, "fp32", mask=mask)
    compare_rgba(r_rgba, r_rays, rgba, out["cls"], f.scene, "fp32", mask=mask)
    fp32 = out["path"] == bh.PATH_FP32
    steps = float(out["steps"][fp32].mean())
    base = gpu_render(bh, f, bh.FP32, rtol_fp32_growth=1.0)[1]["steps"][fp32].mean()
    print(f"growth {growth}: {steps:.2f} step evaluations per FP32 ray (growth 1: {base:.2f}), "
          f"max exit angle {s['max_angle']:.3g} rad")
    if growth > 1.0:
        assert steps < 0.85 * base


def test_band_tolerance_applies_to_fp32_mode_only(bh):
    """rtol_band sets the FP64 integrator's tolerance for the critical band of
    FP32 mode: FP64 renders are bit-identical whatever its value, while FP32
    renders change their band rays (and only them)."""
    f = inputs.Frame(inputs.Camera(30.0, 75.0, 20.0, 21.0, 256, 256), inputs.scene_in_m(1.0, (6.0, 20.0)))
    a64, o64 = gpu_render(bh, f, bh.FP64)
    b64, p64 = gpu_render(bh, f, bh.FP64, rtol_band=1e-4)
    np.testing.assert_array_equal(a64, b64)
    np.testing.assert_array_equal(o64["phi_end"], p64["phi_end"])
    _, o32 = gpu_render(bh, f, bh.FP32)
    _, p32 = gpu_render(bh, f, bh.FP32, rtol_band=1e-6)
    band = o32["path"] == bh.PATH_FP64
    assert band.sum() > 1000
    np.testing.assert_array_equal(o32["phi_end"][~band], p32["phi_end"][~band])
    assert np.any(o32["phi_end"][band] != p32["phi_end"][band])
    assert o32["steps"][band].mean() > p32["steps"][band].mean()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("disk", [None, (6.0, 20.0)])
def test_band_rays_match_oracle(bh, ref, precision, disk):
    """A 512x512 frame framed on the shadow edge (camera at 30 M, FOV 21 deg):
    about 7,000 rays lie in the critical band 1e-3 M <= |b - b_c| < 0.05 M.
    They go through the FP64 integrator in both modes (in FP32 mode through
    its separate band queue), and each is held to the oracle: classes agree
    (outside a disk-edge zone widened by the band bound), end azimuths and
    exit directions within 1e-8 + b D / |b - b_c| (D = 1e-10; FP32 mode, whose
    band runs at rtol_band 1e-9: D = 1.1e-9, and exit directions are mapped in
    FP32, so within 1e-4 plus that), disk radii likewise, colours outside the
    checker-edge zone."""
    f = inputs.Frame(inputs.Camera(30.0, 75.0, 20.0, 21.0, 512, 512), inputs.scene_in_m(1.0, disk))
    rgba, out = gpu_render(bh, f, bh.FP64 if precision == "fp64" else bh.FP32)
    r_rgba, r_rays = ref.render(ref_camera(ref, f.camera), ref_scene(ref, f.scene))
    s = compare(r_rays, out, f.scene, precision)
    assert s["band_compared"] > 6000, s
    compare_rgba(r_rgba, r_rays, rgba, out["cls"], f.scene, precision)
    band = np.abs(r_rays.b - B_CRIT) < 0.05
    assert np.all(out["path"][band] == bh.PATH_FP64)
    print(f"band rays compared {s['band_compared']}, max end-azimuth difference {s['max_band_phi']:.3g} rad")


@pytest.mark.parametrize("k", [0, 7])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_orbit4k_frame_sampled_rows(bh, ref, k, precision):
    """Full 3840x2160 frames of the 16-frame orbit, default launch shape;
    the oracle checks 12 rows spread over the frame."""
    f = inputs.orbit_4k()[k]
    rgba, out = gpu_render(bh, f, bh.FP64 if precision == "fp64" else bh.FP32)
    H = f.camera.height
    rows = sorted(set(np.linspace(0, H - 1, 11).astype(int)) | {H // 2})
    r_rgba, r_rays, mask = oracle_rows(ref, f, rows)
    compare(r_rays, out, f.scene, precision, mask=mask)
    compare_rgba(r_rgba, r_rays, rgba, out["cls"], f.scene, precision, mask=mask)
    # whole-frame properties: every pixel written, alpha 1, classes valid
    assert np.all(rgba[..., 3] == 1.0)
    assert np.all(out["cls"] <= 3)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("r_cam,fov,disk", [(400.0, 70.0, (6.0, 300.0)), (3.5, 90.0, (6.0, 20.0)),
                                            (40.0, 150.0, None)])
def test_extreme_cameras(bh, ref, precision, r_cam, fov, disk):
    """Cameras far out (rays reaching the sky sphere with b up to ~340 M, where
    the FP32 Newton stop leaves its largest residual), just outside the photon
    sphere, and with a 150-degree field of view: classes, exit directions,
    disk radii and colours against the oracle."""
    f = inputs.Frame(inputs.Camera(r_cam, 63.0, 17.0, fov, 72, 40), inputs.scene_in_m(1.0, disk))
    rgba, out = gpu_render(bh, f, bh.FP64 if precision == "fp64" else bh.FP32)
    r_rgba, r_rays = ref.render(ref_camera(ref, f.camera), ref_scene(ref, f.scene))
    s = compare(r_rays, out, f.scene, precision)
    compare_rgba(r_rgba, r_rays, rgba, out["cls"], f.scene, precision)
    assert s["n"] == 72 * 40


@pytest.mark.parametrize("M,disk", [(1.0, (6.0, 30.0)), (0.5, None), (0.0, (2.0, 40.0))])
def test_trace_rays_random(bh, ref, M, disk):
    import torch
    sc = inputs.Scene(M=M, r_sky=1000.0, disk=disk)
    o, d = inputs.random_rays(20000, seed=int(10 + 3 * M), r_min=max(3.5 * M, 5.0), r_max=200.0,
                              aim_scale=15.0)
    out = np_out(bh.trace_rays(torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda(), sc))
    r = ref.trace_rays(o, d, ref_scene(ref, sc))
    compare(r, out, sc, "fp64")
    out32 = np_out(bh.trace_rays(torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda(), sc,
                                 bh.options(precision=bh.FP32)))
    compare(r, out32, sc, "fp32")


def test_trace_rays_degenerate(bh, ref):
    import torch
    sc = inputs.Scene(M=1.0, r_sky=1000.0)
    o = np.array([[50.0, 0, 0], [50.0, 0, 0], [2.9, 0, 0], [2000.0, 0, 0], [np.nan, 0, 0],
                  [50.0, 0, 0], [0, 0, 40.0]])
    d = np.array([[-1.0, 0, 0], [1.0, 0, 0], [0, 1.0, 0], [0, 1.0, 0], [0, 1.0, 0], [0, 0, 0],
                  [0.1, 0, -1]])
    out = np_out(bh.trace_rays(torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda(), sc))
    r = ref.trace_rays(o, d, ref_scene(ref, sc))
    np.testing.assert_array_equal(out["cls"], r.cls)
    np.testing.assert_allclose(out["exit_dir"][:2], r.exit_dir[:2], atol=1e-15)
    # empty batch
    e = torch.zeros((0, 3), dtype=torch.float64, device="cuda")
    assert bh.trace_rays(e, e, sc)["cls"].numel() == 0


@pytest.mark.parametrize("W,H", [(1, 1), (67, 13), (5, 300)])
def test_ragged_and_tiny_images(bh, ref, W, H):
    f = inputs.Frame(inputs.Camera(25.0, 63.0, 30.0, 70.0, W, H), inputs.scene_in_m(1.0, (6.0, 20.0)))
    rgba, out = gpu_render(bh, f, bh.FP64)
    r_rgba, r_rays = ref.render(ref_camera(ref, f.camera), ref_scene(ref, f.scene))
    compare(r_rays, out, f.scene, "fp64")
    compare_rgba(r_rgba, r_rays, rgba, out["cls"], f.scene, "fp64")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_flat_space_render(bh, ref, precision):
    f = inputs.Frame(inputs.Camera(30.0, 90.0, 0.0, 60.0, 48, 32),
                     inputs.Scene(M=0.0, r_sky=1000.0, disk=(2.0, 12.0)))
    rgba, out = gpu_render(bh, f, bh.FP64 if precision == "fp64" else bh.FP32)
    r_rgba, r_rays = ref.render(ref_camera(ref, f.camera), ref_scene(ref, f.scene))
    compare(r_rays, out, f.scene, precision)
    compare_rgba(r_rgba, r_rays, rgba, out["cls"], f.scene, precision)
    assert not np.any(out["cls"] == bh.CAPTURED)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_schedule_invariance(bh, precision):
    """Each ray's arithmetic is independent of the launch shape, the queue
    order and the refill threshold: results are bit-identical across grid
    sizes, chunk sizes and refill thresholds 1 (every finished lane restarts
    at once: the stress case for the queue), 6, 20 and 32 (the race test for
    the work queue)."""
    f = inputs.disk_1024(256)
    p = bh.FP64 if precision == "fp64" else bh.FP32
    base_rgba, base = gpu_render(bh, f, p)
    shapes = [dict(grid_blocks=g, chunk=c) for g, c in [(1, 64), (7, 64), (64, 1024), (3, 192)]]
    shapes += [dict(refill_fp32=r, refill_fp64=r) for r in (1, 6, 20, 32)]
    shapes += [dict(grid_blocks=5, chunk=64, refill_fp32=1, refill_fp64=1)]
    for kw in shapes:
        rgba, out = gpu_render(bh, f, p, **kw)
        np.testing.assert_array_equal(rgba, base_rgba, err_msg=str(kw))
        for k in ("cls", "phi_end", "r_hit", "steps", "path"):
            np.testing.assert_array_equal(out[k], base[k], err_msg=f"{kw} {k}")


def test_schedule_invariance_at_4k(bh):
    """A 4K FP32 render takes its queue chunk from its size (384 rays); the
    pixels and per-ray records equal those of 256- and 512-ray chunks bit for
    bit."""
    f = inputs.orbit_4k()[0]
    base_rgba, base = gpu_render(bh, f, bh.FP32)
    for c in (256, 512):
        rgba, out = gpu_render(bh, f, bh.FP32, chunk=c)
        np.testing.assert_array_equal(rgba, base_rgba, err_msg=f"chunk {c}")
        for k in ("cls", "phi_end", "r_hit", "steps", "path"):
            np.testing.assert_array_equal(out[k], base[k], err_msg=f"chunk {c} {k}")


def test_step_caps(bh, ref):
    """max_steps and max_phi caps give UNRESOLVED, as in the oracle."""
    f = inputs.plain_64()
    _, out = gpu_render(bh, f, bh.FP64, max_steps=5, analytic_capture=0)
    assert np.all(out["cls"] == bh.UNRESOLVED)
    assert np.all(out["steps"] == 5)
    _, r = ref.render(ref_camera(ref, f.camera), ref_scene(ref, f.scene), ref.options(max_phi=1.0))
    _, out = gpu_render(bh, f, bh.FP64, max_phi=1.0, analytic_capture=0)
    # Whether an event in the step that crosses the cap fires first depends
    # on where that step ends; rays ending clear of the cap must agree.
    clear = (r.phi_end < 0.9) & (out["phi_end"] < 0.9) | (r.cls == 3) & (out["cls"] == 3)
    np.testing.assert_array_equal(out["cls"][clear], r.cls[clear])
    near = ~clear
    assert near.sum() < 0.01 * near.size
    assert np.all(np.maximum(r.phi_end[near], out["phi_end"][near]) >= 0.9)


def test_step_counts_track_oracle(bh, ref):
    """Same controller: mean step evaluations per ray within 8% of the
    oracle's accepted + rejected count (the GPU count also includes the <= 3
    sky-crossing refinement steps)."""
    f = inputs.disk_1024(128)
    _, out = gpu_render(bh, f, bh.FP64, analytic_capture=0)
    _, r = ref.render(ref_camera(ref, f.camera), ref_scene(ref, f.scene))
    g = out["steps"].mean()
    o = (r.n_acc + r.n_rej).mean()
    assert abs(g / o - 1.0) < 0.08, (g, o)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_stats_account_for_every_ray_and_step(bh, ref, precision):
    """bh_last_stats (collect_stats = 1): the instrumented integrator gives the
    same image and records as the plain one; the per-class and per-path ray
    counts match the per-ray records; accepted + rejected + Newton steps add
    up to the per-ray step evaluations; capped rays are the UNRESOLVED ones;
    and in FP64 mode the accepted and rejected steps track the oracle's (same
    controller, same tolerance) within 2%."""
    f = inputs.disk_1024(160)
    p = bh.FP64 if precision == "fp64" else bh.FP32
    rgba0, out0 = gpu_render(bh, f, p)
    with pytest.raises(bh.BhError) as e:
        bh.last_stats()
    assert e.value.status == bh.BH_ERR_STATE
    rgba, out = gpu_render(bh, f, p, collect_stats=1)
    np.testing.assert_array_equal(rgba, rgba0)
    for k in ("cls", "phi_end", "r_hit", "steps", "path"):
        np.testing.assert_array_equal(out[k], out0[k])
    st = bh.last_stats()
    n = f.camera.width * f.camera.height
    assert st["rays"] == n
    for c, name in enumerate(("sky", "captured", "disk", "unresolved", "invalid")):
        assert st["cls"][name] == int((out["cls"] == c).sum()), name
    for q, name in enumerate(("none", "fp64", "fp32", "surrogate")):
        assert st["path"][name] == int((out["path"] == q).sum()), name
    assert st["step_evals"] == int(out["steps"].astype(np.int64).sum())
    tot = sum(st[k]["fp64"] + st[k]["fp32"] for k in ("accepted", "rejected", "newton"))
    assert tot == st["step_evals"]
    assert st["capped"]["fp64"] + st["capped"]["fp32"] == st["cls"]["unresolved"]
    # every integrated ray takes at least one accepted step
    integrated = int((out["path"] == bh.PATH_FP64).sum() + (out["path"] == bh.PATH_FP32).sum())
    assert st["accepted"]["fp64"] + st["accepted"]["fp32"] >= integrated
    if precision == "fp32":
        assert st["accepted"]["fp32"] > 0 and st["accepted"]["fp64"] > 0  # the band
    else:
        assert st["accepted"]["fp32"] == 0 and st["newton"]["fp32"] == 0
        _, r = ref.render(ref_camera(ref, f.camera), ref_scene(ref, f.scene))
        integ = (out["path"] == bh.PATH_FP64)
        oa, orj = int(r.n_acc[integ].sum()), int(r.n_rej[integ].sum())
        assert abs(st["accepted"]["fp64"] / oa - 1.0) < 0.02, (st["accepted"], oa)
        assert abs(st["rejected"]["fp64"] - orj) <= 0.02 * oa, (st["rejected"], orj)
    # queue timeline: every main-queue wavefront entered, found the queue dry
    # and left, in that order
    tl = st["timeline_us"]
    assert st["timeline_waves"] > 0
    assert tl["wave_enter_us"][0] == 0.0
    for q in range(3):
        assert tl["wave_enter_us"][q] <= tl["queue_dry_us"][q] <= tl["wave_exit_us"][q], tl
    print(f"{precision}: accepted {st['accepted']}, rejected {st['rejected']}, "
          f"newton {st['newton']} over {integrated} integrated rays; timeline {tl}")


def test_counts(bh):
    import torch
    f = inputs.plain_64()
    bh.render(f.camera, f.scene, bh.options(precision=bh.FP32))
    c = bh.last_counts()
    assert sum(c.values()) == 4096
    assert 250 < c["setup"] <= 300  # analytic captures (below the band)
    assert c["fp64"] > 0 and c["fp32"] > 3000


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_samples_per_pixel(bh, ref, precision):
    """n x n samples per pixel: the per-sample records equal the oracle's
    render of the same camera at n times the resolution, and each pixel is
    the mean of its n*n samples' colours (pixels whose samples are all clear
    of the ambiguity zones)."""
    from parity import TOL, near_cell_boundary
    n = 3
    f = inputs.Frame(inputs.Camera(25.0, 70.0, 40.0, 60.0, 40, 24), inputs.scene_in_m(1.0, (6.0, 20.0)))
    p = bh.FP64 if precision == "fp64" else bh.FP32
    rgba, out = gpu_render(bh, f, p, samples_side=n)
    W, H = f.camera.width, f.camera.height
    sub = inputs.Camera(f.camera.r, f.camera.incl_deg, f.camera.azim_deg, f.camera.fov_deg, W * n, H * n)
    r_rgba, r_rays = ref.render(ref_camera(ref, sub), ref_scene(ref, f.scene))
    compare(r_rays, out, f.scene, precision)
    t = TOL[precision]
    rc, gc = r_rays.cls.astype(int), out["cls"].astype(int)
    ok = (rc == gc) & ~(np.abs(r_rays.b - B_CRIT) < 0.05)
    ok &= ~(near_cell_boundary(r_rays.exit_dir, f.scene.checker_deg, t["tau_theta"]) & (rc == 0))
    blocks = lambda a: a.reshape(H, n, W, n, *a.shape[2:]).swapaxes(1, 2)  # (H, W, n, n, ...)
    ok_px = blocks(ok.reshape(H * n, W * n)).all(axis=(2, 3))
    want = blocks(r_rgba.astype(np.float64)).mean(axis=(2, 3))
    tol = blocks(np.where((rc == 2)[:, None], 4.0 * t["r_rel"] * np.abs(r_rgba.reshape(-1, 4)) + 1e-7,
                          t["rgba"]).reshape(H * n, W * n, 4)).mean(axis=(2, 3))
    d = np.abs(rgba.astype(np.float64) - want)
    assert ok_px.sum() > 0.8 * W * H
    assert np.all((d <= tol + 1e-6)[ok_px]), d[ok_px].max()
    # one sample per pixel is the plain render
    rgba1, _ = gpu_render(bh, f, p, samples_side=1)
    rgba0, _ = gpu_render(bh, f, p)
    np.testing.assert_array_equal(rgba1, rgba0)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_textured_sky(bh, ref, precision):
    """Equirectangular sky image with bilinear filtering: rays as for the
    checker; sky colours within the image's largest texel step times the
    texel displacement that the path's exit-angle bound allows."""
    from parity import TOL
    tex = inputs.sky_texture(256, 128, seed=3)
    sc = inputs.Scene(M=1.0, r_sky=1000.0, disk=(6.0, 20.0), sky_tex=tex)
    f = inputs.Frame(inputs.Camera(30.0, 75.0, 20.0, 60.0, 48, 32), sc)
    p = bh.FP64 if precision == "fp64" else bh.FP32
    rgba, out = gpu_render(bh, f, p)
    r_rgba, r_rays = ref.render(ref_camera(ref, f.camera), ref_scene(ref, sc))
    compare(r_rays, out, sc, precision)
    t = TOL[precision]
    rc, gc = r_rays.cls.astype(int), out["cls"].astype(int)
    R, G = r_rgba.reshape(-1, 4).astype(np.float64), rgba.reshape(-1, 4).astype(np.float64)
    sky = (rc == 0) & (gc == 0) & ~(np.abs(r_rays.b - B_CRIT) < 0.05)
    s_ = r_rays.exit_dir[sky]
    sin_t = np.maximum(np.hypot(s_[:, 0], s_[:, 1]), 1e-3)
    step = max(np.abs(np.diff(tex, axis=1)).max(), np.abs(np.diff(tex, axis=0)).max())
    H_t, W_t = tex.shape[:2]
    tol = step * (W_t / (2 * np.pi) / sin_t + H_t / np.pi) * t["angle"] + 2e-6
    d = np.abs(R[sky] - G[sky]).max(axis=1)
    assert sky.sum() > 500
    assert np.all(d <= tol), (d.max(), d[np.argmax(d / tol)], tol[np.argmax(d / tol)])
    other = (rc == gc) & (rc == 1)
    np.testing.assert_array_equal(G[other], R[other])


@pytest.mark.parametrize("M,disk", [(1.0, (6.0, 20.0)), (0.0, (2.0, 12.0))])
def test_paper_fixed_step_mode(bh, ref, M, disk):
    """The paper's fixed-step mode (points ~eps apart, hits on chords) against
    the oracle's, both FP64: the same classes, exit directions and hit radii
    to the FP64 bounds, and the same number of steps per ray."""
    eps = 0.5
    f = inputs.Frame(inputs.Camera(30.0, 80.0, 10.0, 60.0, 40, 30),
                     inputs.Scene(M=M, r_sky=1000.0, disk=disk))
    rgba, out = gpu_render(bh, f, bh.FP64, fixed_eps=eps)
    r_rgba, r_rays = ref.render(ref_camera(ref, f.camera), ref_scene(ref, f.scene),
                                ref.options(fixed_eps=eps))
    compare(r_rays, out, f.scene, "fp64")
    compare_rgba(r_rgba, r_rays, rgba, out["cls"], f.scene, "fp64")
    integ = r_rays.n_acc > 0
    assert np.abs(out["steps"][integ] - r_rays.n_acc[integ]).max() <= 1
    assert out["steps"][integ].mean() > 100  # many short steps, as the paper takes them
