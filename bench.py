#!/usr/bin/env python3
"""Benchmark: Schwarzschild ray tracing at 4K on one MI355X.

Workload: the 16-frame camera orbit at 3840x2160 (per frame M ~ U[0.5, 2],
camera at U[20, 100] M, inclination U[0, 90] deg, disk 6-30 M, checker sky at
1000 M, FOV 60 deg; seeded).  One step = render all 16 frames through the
whole path as one batch (set-up/routing of every frame's rays, one
persistent FP32 integration launch with the FP64 critical band over all of
them, shading into resident fp32 RGBA buffers).  Value = rays per second of
the step.  Also reported: the same frames rendered one bh_render call at a
time; the plain FP64 kernel on the same frames; the same frames with the
surrogate network (trained here on the GPU first); the 512-request
batched-serving mix in one graph-replayed launch; the roofline of the
dominant kernel (the batch integrator, timed with HIP events on its launch
stream) and of the surrogate's inference kernel; and the CPU FP64 oracle
timed on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                       [--no-surrogate] [--no-batch] [--fp64-steps K64]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FLOP per Dormand-Prince step evaluation (FMA = 2), counted from
# the kernel's Nystrom-form step in the scaled variable v = 3M u: 6 evaluations
# of g(v) = v^2 - v 12, stage sums 35, solution 20, error estimate 22, error
# scale 4, phi update 1.
FLOP_PER_STEP = 94
# The same step written in its standard Dormand-Prince form (every stage's w
# summed explicitly) is the per-step figure first estimated for the method,
# about 150 FLOP; reported beside the kernel's own count.
FLOP_PER_STEP_STANDARD = 150
# MI355X published vector peaks: FP32 157.3 TFLOP/s (it counts packed FP32
# instructions, two FMAs per lane per clock), FP64 78.6 TFLOP/s.  The library
# is built without packed FP32 instructions, so its FP32 code issues at most
# one FMA per lane per clock: 256 CU x 4 SIMD x 16 lanes x 2 FLOP x 2.4 GHz
# = 78.6 TFLOP/s, the ceiling it can reach (reported as a second fraction).
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
SCALAR_FMA_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_integrate_fp32_batch_orbit4k_traffic.txt")
ROOFLINE_KERNEL = "bh::k_integrate_fp32_batch<false>"
# HBM bytes per ray of the batch integrator (FP32 batches keep FP32 records,
# whose result record carries the end class): start record (8 B) and request
# index (4 B) read, result record (8 B) written
BYTES_PER_RAY = 20
KERNEL_SRCS = [os.path.join(ROOT, "paper_2507_16165_amd", "csrc", f)
               for f in ("bh_kernels.hip", "bh_internal.h")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def code_of(text: str) -> str:
    """C/C++ source without comments and with whitespace collapsed: the part
    of the text that can change the compiled kernel."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_hash() -> str:
    """Hash of the integrator's code (comments and layout ignored): the
    traffic figure is only valid for the kernel it was counted on."""
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        with open(f, encoding="utf-8") as fh:
            h.update(code_of(fh.read()).encode())
    return h.hexdigest()[:16]


def read_traffic():
    """HBM bytes per integrator launch from the committed rocprofv3 counter
    summary, or None if it is absent or the kernel source changed since."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != kernel_hash():
        return None
    try:
        return float(kv["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--fp64-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-row-stride", type=int, default=6,
                    help="oracle sample: every n-th row of every frame, all host threads")
    ap.add_argument("--cpu-row-stride-1t", type=int, default=96,
                    help="oracle sample for the one-thread figure: every n-th row of every frame")
    ap.add_argument("--frames", type=int, default=16)
    ap.add_argument("--rtol-fp32", type=float, default=1e-6,
                    help="relative tolerance of the FP32 integrator (the library default is 1e-6)")
    ap.add_argument("--rtol-fp32-growth", type=float, default=50.0,
                    help="largest factor on an FP32 ray's tolerance far from the critical impact "
                         "parameter (the library default is 50; 1 = the same tolerance for every ray)")
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip the surrogate leg (training and the surrogate render)")
    ap.add_argument("--sur-epochs", type=int, default=40)
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-serving leg")
    ap.add_argument("--no-sky-images", action="store_true",
                    help="skip the sky-image size sweep")
    ap.add_argument("--no-paper", action="store_true",
                    help="skip the fixed-step (paper) mode sweep")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the all-pixel comparison of the fast path with the FP64 kernel")
    ap.add_argument("--batch-requests", type=int, default=512)
    ap.add_argument("--batch-reps", type=int, default=3)
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (the reference "
                         "kernel for scaling rocprofv3 FETCH_SIZE/WRITE_SIZE)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(an image would shard over GPUs by interleaved 16x16 pixel tiles, each GPU "
              "running the single-GPU path on its tiles).",
              file=sys.stderr)
        return 2

    import torch

    from paper_2507_16165_amd import api, inputs

    if args.calibrate_copy_mib > 0:
        n = args.calibrate_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {args.calibrate_copy_mib} MiB read + written")
        del src, dst

    frames = inputs.orbit_4k(frames=args.frames)
    W, H = frames[0].camera.width, frames[0].camera.height
    rays_per_step = W * H * len(frames)
    api.reserve(W * H)
    bufs = [torch.empty((H, W, 4), dtype=torch.float32, device="cuda") for _ in frames]
    opt_fast = api.options(precision=api.FP32, batch_groups=1, rtol_fp32=args.rtol_fp32,
                           rtol_fp32_growth=args.rtol_fp32_growth)
    opt_fp64 = api.options(precision=api.FP64, batch_groups=1)
    batches = {}

    def step(opt):
        """All frames as one batch: one group, three launches."""
        key = (opt.precision, opt.rtol, opt.rtol_fp32)
        if key not in batches:
            batches[key] = api.Batch(frames, opt, use_graph=False, images=bufs)
        batches[key].launch()

    def step_frames(opt):
        """The frames one bh_render call each."""
        for f, buf in zip(frames, bufs):
            api.render(f.camera, f.scene, opt, rgba=buf)

    def timed(step_fn, opt, k, warm, events=True):
        """Milliseconds per step over k steps after `warm` untimed ones, and
        the library's per-kernel HIP-event times over the same steps (with
        events=False none are recorded: the rate a caller gets by default)."""
        for _ in range(warm):
            step_fn(opt)
        torch.cuda.synchronize()
        api.timing_enable(events)
        api.timing_read()
        t0 = time.perf_counter()
        for i in range(k):
            step_fn(opt)
            log(f"step {i + 1}/{k} enqueued")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        tim = api.timing_read()
        api.timing_enable(False)
        return (t1 - t0) * 1e3 / k, tim

    log(f"fast path (one batch): warmup {args.warmup}, steps {args.steps}")
    ms_step, tim = timed(step, opt_fast, args.steps, args.warmup)
    log(f"fast path {ms_step:.3f} ms/step")
    log(f"fast path, one render call per frame: steps {args.steps}")
    # The rate without the library's timing events (six event records per
    # frame measured about 6% of a one-frame render), then the same steps
    # with events for the kernel times.
    ms_frames, _ = timed(step_frames, opt_fast, args.steps, 1, events=False)
    _, tim_frames = timed(step_frames, opt_fast, args.steps, 0)
    log(f"per-frame renders {ms_frames:.3f} ms/step")
    if args.fp64_steps > 0:
        log(f"fp64 path (one batch): steps {args.fp64_steps}")
        ms_step64, tim64 = timed(step, opt_fp64, args.fp64_steps, 1)
        log(f"fp64 path {ms_step64:.3f} ms/step")
    else:
        ms_step64, tim64 = float("nan"), None
    for b in batches.values():
        b.close()
    batches.clear()

    # Algorithmic work: step evaluations per ray are independent of the
    # schedule (the batch's pixels equal the per-frame renders), so one
    # instrumented per-frame pass gives the count of the timed launches.
    def step_evals(opt):
        """Summed step evaluations and rays per path over the frames, and the
        controller's split (accepted, rejected, Newton re-steps per path)
        from the instrumented integrator (bh_last_stats)."""
        tot = 0
        per_path = {}
        split = {}
        timeline = []
        opt_s = api.options(precision=opt.precision, rtol=opt.rtol, rtol_fp32=opt.rtol_fp32,
                            rtol_fp32_growth=opt.rtol_fp32_growth, collect_stats=1)
        for f, buf in zip(frames, bufs):
            _, out = api.render(f.camera, f.scene, opt_s, rgba=buf, fields=("steps", "path"))
            tot += int(out["steps"].to(torch.int64).sum().item())
            for p in (api.PATH_NONE, api.PATH_FP64, api.PATH_FP32):
                per_path[p] = per_path.get(p, 0) + int((out["path"] == p).sum().item())
            st = api.last_stats()
            assert st["step_evals"] == int(out["steps"].to(torch.int64).sum().item())
            for k in ("accepted", "rejected", "newton", "capped"):
                for q in ("fp64", "fp32"):
                    split[(k, q)] = split.get((k, q), 0) + st[k][q]
            timeline.append(st["timeline_us"])
        step_evals.timeline = timeline
        return tot, per_path, split

    def controller(split, per_path):
        """Per integrated ray of each path: accepted steps, rejected trial
        steps and Newton re-steps of the sky crossing."""
        out = {}
        for q, p in (("fp32", api.PATH_FP32), ("fp64", api.PATH_FP64)):
            n = max(1, per_path.get(p, 0))
            out[q] = {k + "_per_ray": round(split[(k, q)] / n, 3)
                      for k in ("accepted", "rejected", "newton")}
            out[q]["rays"] = per_path.get(p, 0)
            out[q]["capped"] = split[("capped", q)]
        return out

    def roof(evals, t, k):
        """(FLOP per integrator launch, mean launch ms, TFLOP/s) of k timed steps."""
        ms, n = t["integrate"]
        flop = evals * FLOP_PER_STEP / (n / k)
        return flop, ms / n, flop / (ms / n * 1e-3) / 1e12

    evals, paths, split = step_evals(opt_fast)
    tl = step_evals.timeline

    def tl_mean(key, q):
        return round(sum(t[key][q] for t in tl) / len(tl), 1)
    flop_launch, avg_launch_ms, achieved = roof(evals, tim, args.steps)
    _, avg_launch_frames, achieved_frames = roof(evals, tim_frames, args.steps)
    if tim64 is not None:
        evals64, paths64, split64 = step_evals(opt_fp64)
        _, _, achieved64 = roof(evals64, tim64, args.fp64_steps)
    else:
        evals64, achieved64 = float("nan"), float("nan")
    # the committed counters were taken on the 16 frames at 3840x2160
    traffic = read_traffic() if (len(frames), W, H) == (16, 3840, 2160) else None
    launches_per_step = tim["integrate"][1] // args.steps
    rays_per_launch = rays_per_step // max(launches_per_step, 1)

    value = rays_per_step / (ms_step * 1e-3) / 1e6
    value_frames = rays_per_step / (ms_frames * 1e-3) / 1e6
    value64 = rays_per_step / (ms_step64 * 1e-3) / 1e6

    line = {
        "metric": "Mrays/s at 4K: FP64 RK45 vs FP32+surrogate at <=1e-4 rad err; % FP peak",
        "value": round(value, 2),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {
            "workload": f"orbit_4k: {len(frames)} frames 3840x2160 rendered as one batch, disk 6-30 M, "
                        "checker sky, FP32 integrator + FP64 band |b-3sqrt3 M|<0.05M",
            "frames": len(frames), "width": W, "height": H, "rays_per_step": rays_per_step,
            "rtol_fp32": opt_fast.rtol_fp32, "rtol_fp32_growth": opt_fast.rtol_fp32_growth,
            "rtol_band": opt_fast.rtol_band, "rtol_fp64": opt_fast.rtol,
        },
        "per_frame_renders": {"value": round(value_frames, 2), "unit": "Mrays/s",
                              "ms_per_step": round(ms_frames, 4),
                              "integrator_avg_launch_ms": round(avg_launch_frames, 4),
                              "integrator_tflops": round(achieved_frames, 3),
                              "queue_timeline_us": {
                                  "note": "one frame's main queue (instrumented pass), mean over the "
                                          "frames: when wavefronts found the queue dry and left it",
                                  "dry_first": tl_mean("queue_dry_us", 0),
                                  "dry_median": tl_mean("queue_dry_us", 1),
                                  "exit_median": tl_mean("wave_exit_us", 1),
                                  "exit_last": tl_mean("wave_exit_us", 2)},
                              "kernels_ms_per_step": {k: round(v[0] / args.steps, 4)
                                                      for k, v in tim_frames.items()}},
        "fp64_plain": {"value": round(value64, 2), "unit": "Mrays/s",
                       "ms_per_step": round(ms_step64, 4), "rtol": opt_fp64.rtol,
                       "achieved_tflops": round(achieved64, 3),
                       "frac": round(achieved64 / PEAK_FP64_TFLOPS, 4),
                       "step_evals_per_ray": round(evals64 / rays_per_step, 3),
                       "controller": (controller(split64, paths64)["fp64"]
                                      if tim64 is not None else None)},
        "speedup_vs_fp64": round(value / value64, 3),
        "kernels_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in tim.items()},
        "paths": {"setup_only": paths.get(0, 0), "fp64_band": paths.get(1, 0),
                  "fp32": paths.get(2, 0)},
        "step_evals_per_ray": round(evals / rays_per_step, 3),
        "controller": controller(split, paths),
        "roofline": {
            "kernel": ROOFLINE_KERNEL,
            "bound": "alu",
            "achieved": round(achieved, 3),
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
            "flop_per_step_eval": FLOP_PER_STEP,
            "step_evals_per_launch": evals // max(1, launches_per_step),
            "frac_of_scalar_fma_ceiling": round(achieved / SCALAR_FMA_TFLOPS, 4),
            "scalar_fma_ceiling_tflops": round(SCALAR_FMA_TFLOPS, 2),
            "achieved_at_standard_form_flop": round(achieved * FLOP_PER_STEP_STANDARD / FLOP_PER_STEP, 3),
            "frac_at_standard_form_flop": round(achieved * FLOP_PER_STEP_STANDARD / FLOP_PER_STEP
                                                / PEAK_FP32_TFLOPS, 4),
            "traffic": traffic,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
            "algorithmic_bytes_per_launch": BYTES_PER_RAY * rays_per_launch,
            "launches_per_step": launches_per_step,
            "flop_per_launch": flop_launch,
            "avg_launch_ms": round(avg_launch_ms, 4),
        },
    }

    if not args.no_accuracy:
        line["accuracy_all_pixels"] = accuracy_leg(frames, api, torch, opt_fast)
    sweep = None
    if not args.no_paper:
        # the orbit's nearest and farthest camera: the surrogate serves rays
        # only where the camera sees impact parameters above the disk's rim
        by_dist = sorted(frames, key=lambda f: f.camera.r / f.scene.M)
        sweep = Sweep([by_dist[0], by_dist[-1]], api, torch)
        line["paper_mode_sweep"] = paper_leg(sweep, api)
    if not args.no_surrogate:
        line["surrogate"] = surrogate_leg(args, frames, bufs, api, torch, value_frames, step_frames,
                                         sweep, value)
        if sweep is not None:
            line["paper_mode_sweep"]["adaptive_fp32_band_surrogate"] = line["surrogate"].pop("sweep_point")
    
    if not args.no_sky_images:
        line["sky_image_sweep"] = sky_image_leg(frames, bufs, api, torch, opt_fast)
    if not args.no_batch:
        line["batch_serving"] = batch_leg(args, api, torch)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(frames, args.cpu_row_stride, args.cpu_row_stride_1t, bufs,
                                            opt_fast, api, torch)
    print(json.dumps(line), flush=True)
    return 0


def accuracy_leg(frames, api, torch, opt32):
    """Every pixel of the 16 frames: the FP32 + band path against the FP64
    kernel (itself held to the CPU oracle within 1e-8 rad by the parity
    tests).  Rays in the critical band |b - 3 sqrt(3) M| < 0.05 M are the
    ambiguity zone for the class; sky and disk rays of equal class elsewhere
    give the exit-direction and hit-radius errors; checker-boundary pixels
    (within 1e-4 rad of a cell edge) are left out of the colour count."""
    import math
    W, H = frames[0].camera.width, frames[0].camera.height
    fields = ("cls", "b", "exit_dir", "r_hit", "phi_end")
    opt64 = api.options(precision=api.FP64)
    band_n, band_worst, band_mism = 0, 0.0, 0
    img32 = torch.empty((H, W, 4), dtype=torch.float32, device="cuda")
    img64 = torch.empty_like(img32)
    n = 0
    mism = 0
    edge_n = 0
    pairs = {}
    band = 0
    ang_max = 0.0
    rr_max = 0.0
    hist = torch.zeros(200, dtype=torch.float64, device="cuda")   # log10 bins of the angle
    colour_bad = 0
    colour_n = 0
    log(f"accuracy: all {len(frames)} frames, FP32 + band vs FP64")
    for f in frames:
        _, a = api.render(f.camera, f.scene, opt32, rgba=img32, fields=fields)
        _, b = api.render(f.camera, f.scene, opt64, rgba=img64, fields=fields)
        M = f.scene.M
        bc = 3.0 * math.sqrt(3.0) * M
        in_band = (b["b"] - bc).abs() < 0.05 * M
        same = a["cls"] == b["cls"]
        # disk-edge zone: a DISK / non-DISK disagreement whose DISK side hit
        # within 1e-4 r of an edge (the FP32 radius tolerance)
        one_disk = (a["cls"] == 2) ^ (b["cls"] == 2)
        r_d = torch.where(a["cls"] == 2, a["r_hit"], b["r_hit"])
        rin, rout = f.scene.disk if f.scene.disk is not None else (0.0, 0.0)
        edge_zone = one_disk & (((r_d - rin).abs() < 1e-4 * rin) | ((r_d - rout).abs() < 1e-4 * rout))
        bad = ~same & ~in_band & ~edge_zone
        mism += int(bad.sum().item())
        edge_n += int((~same & ~in_band & edge_zone).sum().item())
        for i in torch.nonzero(bad).flatten()[:8].tolist():
            pairs[f"{int(b['cls'][i])}->{int(a['cls'][i])}"] = pairs.get(
                f"{int(b['cls'][i])}->{int(a['cls'][i])}", 0) + 1
        band += int(in_band.sum().item())
        # band rays 1e-3 M <= |b - b_c| < 0.05 M: both sides FP64-integrated (FP32 mode's
        # band at rtol_band, the FP64 kernel at 1e-10); end azimuths within
        # 1e-8 + b (rtol_band + 1e-10) / |b - b_c| (the parity tests' band bound)
        dist = (b["b"] - bc).abs()
        shallow = in_band & (dist >= 1e-3 * M)
        bsame = shallow & same & ((b["cls"] == 0) | (b["cls"] == 2))
        band_mism += int((shallow & ~same & ~edge_zone).sum().item())
        if bool(bsame.any()):
            lim = 1e-8 + b["b"][bsame] * (opt32.rtol_band + 1e-10) / dist[bsame]
            band_worst = max(band_worst, float(((a["phi_end"][bsame] - b["phi_end"][bsame]).abs()
                                                / lim).max().item()))
            band_n += int(bsame.sum().item())
        ok = same & ~in_band
        sky = ok & (b["cls"] == 0)
        u, v = a["exit_dir"][sky], b["exit_dir"][sky]
        ang = torch.atan2(torch.linalg.cross(u, v).norm(dim=1), (u * v).sum(1))
        if ang.numel():
            ang_max = max(ang_max, float(ang.max().item()))
            idx = ((ang.clamp_min(1e-20).log10() + 20.0) * 10.0).long().clamp(0, 199)
            hist += torch.bincount(idx, minlength=200).double()
        dsk = ok & (b["cls"] == 2)
        if bool(dsk.any()):
            rr_max = max(rr_max, float((a["r_hit"][dsk] / b["r_hit"][dsk] - 1.0).abs().max().item()))
        # colour: checker-edge pixels (exit within 1e-4 rad of a cell boundary) are ambiguous;
        # a direction error of 1e-4 moves the azimuth by up to 1e-4 / sin(theta)
        s = b["exit_dir"]
        th = torch.atan2(torch.hypot(s[:, 0], s[:, 1]), s[:, 2])
        ph = torch.remainder(torch.atan2(s[:, 1], s[:, 0]), 2 * math.pi)
        cell = math.radians(f.scene.checker_deg)
        tph = 1e-4 / torch.sin(th).clamp_min(1e-300)

        def near(x, t):
            fr = x / cell
            return (fr - fr.round()).abs() * cell < t

        edge = (b["cls"] == 0) & (near(th, 1e-4) | near(ph, tph) | (ph < tph) | (2 * math.pi - ph < tph))
        cok = ok & ~edge
        d = (img32.view(-1, 4) - img64.view(-1, 4)).abs().amax(1)
        tol = torch.where(b["cls"] == 2, 4e-4 * img64.view(-1, 4).abs().amax(1) + 1e-7,
                          torch.full_like(d, 1e-6))
        colour_bad += int(((d > tol) & cok).sum().item())
        colour_n += int(cok.sum().item())
        n += W * H
    cum = torch.cumsum(hist, 0)
    p99_bin = int(torch.searchsorted(cum, 0.99 * cum[-1]).item())
    return {"rays": n, "reference": "FP64 kernel (rtol 1e-10)", "band_rays": band,
            "class_mismatch_in_disk_edge_zone": edge_n,
            "class_mismatch_outside_zones": mism, "mismatch_pairs_fp64_to_fp32": pairs,
            "band_rays_compared": band_n, "band_class_mismatch_beyond_1e-3M": band_mism,
            "band_max_end_azimuth_err_over_bound": band_worst,
            "max_exit_angle_rad": ang_max,
            "p99_exit_angle_rad_upper": 10 ** ((p99_bin + 1) / 10.0 - 20.0),
            "max_disk_r_rel": rr_max,
            "colour_mismatch_fraction": colour_bad / max(colour_n, 1)}


class Sweep:
    """Accuracy against throughput on a few 4K frames (one render call per
    frame): each point renders the frames with some options, times them, and
    compares per-ray records with an adaptive FP64 reference at rtol 1e-12
    (rays of equal class outside the critical band |b - b_c| < 0.05 M).  Exit directions of sky rays are
    compared by angle; disk radii relative, outside a 1% zone at either disk
    edge where a chord or a loose step can miss an edge hit."""

    REF_RTOL = 1e-12
    FIELDS = ("cls", "b", "exit_dir", "r_hit", "steps", "path")

    def __init__(self, frames, api, torch):
        self.frames, self.api, self.torch = frames, api, torch
        W, H = frames[0].camera.width, frames[0].camera.height
        self.buf = torch.empty((H, W, 4), dtype=torch.float32, device="cuda")
        self.refs = [api.render(f.camera, f.scene, api.options(precision=api.FP64, rtol=self.REF_RTOL),
                                fields=self.FIELDS)[1] for f in frames]

    def point(self, opt_of):
        import math
        api, torch, frames, buf = self.api, self.torch, self.frames, self.buf
        W, H = frames[0].camera.width, frames[0].camera.height
        for f in frames:
            api.render(f.camera, f.scene, opt_of(f), rgba=buf)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for f in frames:
            api.render(f.camera, f.scene, opt_of(f), rgba=buf)
        torch.cuda.synchronize()
        mrays = len(frames) * W * H / (time.perf_counter() - t0) / 1e6
        ang_max, rr_max, rr_far, worst_db, steps, edge_diff, cls_diff = 0.0, 0.0, 0.0, None, 0, 0, 0
        n_sur = 0
        for f, b in zip(frames, self.refs):
            _, a = api.render(f.camera, f.scene, opt_of(f), rgba=buf, fields=self.FIELDS)
            steps += int(a["steps"].to(torch.int64).sum().item())
            n_sur += int((a["path"] == api.PATH_SURROGATE).sum().item())
            band = (b["b"] - 3.0 * math.sqrt(3.0) * f.scene.M).abs() < 0.05 * f.scene.M
            cls_diff += int(((a["cls"] != b["cls"]) & ~band).sum().item())
            same = (a["cls"] == b["cls"]) & ~band
            sky = same & (b["cls"] == 0)
            u, v = a["exit_dir"][sky], b["exit_dir"][sky]
            ang = torch.atan2(torch.linalg.cross(u, v).norm(dim=1), (u * v).sum(1))
            ang_max = max(ang_max, float(ang.max().item()))
            dsk = same & (b["cls"] == 2)
            rin, rout = f.scene.disk
            edge = ((b["r_hit"] - rin).abs() < 0.01 * rin) | ((b["r_hit"] - rout).abs() < 0.01 * rout)
            edge_diff += int((dsk & edge & ((a["r_hit"] / b["r_hit"] - 1).abs() > 1e-2)).sum().item())
            dsk = dsk & ~edge
            if bool(dsk.any()):
                rr = (a["r_hit"][dsk] / b["r_hit"][dsk] - 1).abs()
                db = (b["b"][dsk] - 3.0 * math.sqrt(3.0) * f.scene.M) / f.scene.M
                k = int(rr.argmax().item())
                if float(rr[k].item()) > rr_max:
                    rr_max, worst_db = float(rr[k].item()), float(db[k].item())
                far = db.abs() >= 0.5
                if bool(far.any()):
                    rr_far = max(rr_far, float(rr[far].max().item()))
        return {"mrays_per_s": round(mrays, 1), "max_exit_angle_rad": ang_max,
                "max_disk_r_rel": rr_max, "worst_disk_ray_b_minus_bc_M": worst_db,
                "max_disk_r_rel_beyond_0.5M": rr_far,
                "edge_zone_rays_hitting_another_crossing": edge_diff,
                "class_differences_outside_band": cls_diff,
                "surrogate_share": round(n_sur / (len(frames) * W * H), 4),
                "steps_per_ray": round(steps / (len(frames) * W * H), 1)}


def paper_leg(sweep, api):
    """The paper's own scheme (points eps*M apart, one step each, hits on
    chords; FP64) for a few eps, beside the adaptive FP64 path at three rtol,
    FP32 + band at three rtol_fp32 (the same tolerance for every ray) and at
    the library's default (rtol_fp32 1e-6 growing 50x away from the critical
    impact parameter): the accuracy/throughput trade-off."""
    out = {"frames": len(sweep.frames),
           "reference": f"adaptive FP64 kernel (rtol {sweep.REF_RTOL:g})"}
    for eps in (8.0, 2.0, 0.5):
        log(f"paper mode: eps = {eps} M")
        out[f"eps_{eps:g}M"] = sweep.point(lambda f, e=eps: api.options(precision=api.FP64,
                                                                      fixed_eps=e * f.scene.M))
    for rt in (1e-6, 1e-8, 1e-10):
        log(f"sweep: adaptive FP64 rtol {rt:g}")
        out[f"adaptive_fp64_rtol_{rt:g}"] = sweep.point(
            lambda f, r=rt: api.options(precision=api.FP64, rtol=r))
    for rt in (1e-4, 1e-5, 1e-6):
        log(f"sweep: adaptive FP32 + band rtol_fp32 {rt:g}")
        out[f"adaptive_fp32_band_rtol_{rt:g}"] = sweep.point(
            lambda f, r=rt: api.options(precision=api.FP32, rtol_fp32=r, rtol_fp32_growth=1.0))
    log("sweep: adaptive FP32 + band, rtol_fp32 1e-6 growing to 5e-5")
    out["adaptive_fp32_band_rtol_1e-06_growth_50"] = sweep.point(
        lambda f: api.options(precision=api.FP32, rtol_fp32=1e-6, rtol_fp32_growth=50.0))
    return out


FLOP_PER_SUR_RAY = 66560     # 2 x (2*128 + 128*128 + 128*128 + 128*2) multiply-adds
PEAK_BF16_TFLOPS = 2500.0    # dense BF16 matrix-core peak


def surrogate_leg(args, frames, bufs, api, torch, value_fast, step, sweep=None, value_batch=None):
    """Trains the network on the GPU (4M escape-side + 1M capture-side FP64
    labels, Adam), builds its trust map, then renders the same frames with
    FP32 + band + surrogate.  Reports the throughput, the gain over the
    integrator alone, the share of rays the network served, its exit error
    against the FP64 integrator on those rays, and the inference kernel's
    matrix-core roofline."""
    from paper_2507_16165_amd import surrogate as S

    log(f"surrogate: labels + training ({args.sur_epochs} epochs)")
    t0 = time.perf_counter()
    sur, rep = S.fit(n_escape=4_000_000, n_capture=1_000_000, n_val=1_000_000,
                     epochs=args.sur_epochs,
                     log=lambda m: log(m) if m.startswith("epoch") and
                     m.split()[1].split("/")[0] in ("1", str(args.sur_epochs)) else None)
    fit_s = time.perf_counter() - t0
    opt = api.options(precision=api.FP32, rtol_fp32=args.rtol_fp32,
                      rtol_fp32_growth=args.rtol_fp32_growth)
    opt.surrogate = sur.handle
    for _ in range(args.warmup):
        step(opt)
    torch.cuda.synchronize()
    # the rate without timing events (as the per-frame leg it is compared
    # with), then the same steps with events for the kernel times
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(opt)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    api.timing_enable(True)
    api.timing_read()
    for _ in range(args.steps):
        step(opt)
    torch.cuda.synchronize()
    tim = api.timing_read()
    api.timing_enable(False)
    W, H = frames[0].camera.width, frames[0].camera.height
    rays = W * H * len(frames)
    # share and exit error of the surrogate-served rays against the FP64 integrator
    n_sur = 0
    max_err = 0.0
    opt64 = api.options(precision=api.FP64)
    for f, buf in zip(frames, bufs):
        _, o = api.render(f.camera, f.scene, opt, rgba=buf, fields=("cls", "exit_dir", "path"))
        _, o64 = api.render(f.camera, f.scene, opt64, rgba=buf, fields=("cls", "exit_dir"))
        on = o["path"] == api.PATH_SURROGATE
        n_sur += int(on.sum().item())
        if bool(on.any()):
            a, b = o["exit_dir"][on], o64["exit_dir"][on]
            ang = torch.atan2(torch.linalg.cross(a, b).norm(dim=1), (a * b).sum(1))
            max_err = max(max_err, float(ang.max().item()))
    sur_ms, sur_n = tim.get("surrogate", (0.0, 0))
    sur_rays_launch = n_sur / len(frames)
    ach = (sur_rays_launch * FLOP_PER_SUR_RAY / (sur_ms / sur_n * 1e-3) / 1e12) if sur_n else 0.0
    value = rays / (ms * 1e-3) / 1e6
    point = sweep.point(lambda f: opt) if sweep is not None else None
    # the same frames as one batch with the network (one inference launch
    # over every frame's listed rays), against the FP32 + band batch
    opt_b = api.options(precision=api.FP32, rtol_fp32=args.rtol_fp32,
                        rtol_fp32_growth=args.rtol_fp32_growth, batch_groups=1)
    opt_b.surrogate = sur.handle
    bt = api.Batch(frames, opt_b, use_graph=False, images=bufs)
    for _ in range(args.warmup):
        bt.launch()
    torch.cuda.synchronize()
    api.timing_enable(True)
    api.timing_read()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        bt.launch()
    torch.cuda.synchronize()
    ms_b = (time.perf_counter() - t0) * 1e3 / args.steps
    tim_b = api.timing_read()
    api.timing_enable(False)
    bt.close()
    value_b = rays / (ms_b * 1e-3) / 1e6
    bsur_ms, bsur_n = tim_b.get("surrogate", (0.0, 0))
    ach_b = (n_sur * FLOP_PER_SUR_RAY / (bsur_ms / bsur_n * 1e-3) / 1e12) if bsur_n else 0.0
    sur.close()
    res = {
        "value": round(value, 2), "unit": "Mrays/s", "ms_per_step": round(ms, 4),
        "gain_vs_fp32_band_per_frame": round(value / value_fast, 4),
        "share": round(n_sur / rays, 4),
        "max_exit_err_rad_vs_fp64": max_err,
        "kernels_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in tim.items()},
        "batch": {"value": round(value_b, 2), "unit": "Mrays/s", "ms_per_step": round(ms_b, 4),
                  "gain_vs_fp32_band_batch": (round(value_b / value_batch, 4)
                                              if value_batch else None),
                  "kernels_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in tim_b.items()},
                  "sur_render_tflops": round(ach_b, 2),
                  "sur_render_frac_of_bf16_peak": round(ach_b / PEAK_BF16_TFLOPS, 4)},
        "fit": {"seconds": round(fit_s, 1), "train_samples": rep["train_samples"],
                "epochs": rep["epochs"], "final_loss": rep["final_loss"],
                "trusted_bins": rep["trusted_bins"],
                "val_p99_err_b30_100": rep["val"].get("p99_err_b30_100"),
                "val_p99_err_b100_1000": rep["val"].get("p99_err_b100_1000"),
                "capture_agreement": rep["val"]["capture_agreement"]},
        "roofline": {"kernel": "bh::k_sur_render", "bound": "mfma", "achieved": round(ach, 2),
                     "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(ach / PEAK_BF16_TFLOPS, 4),
                     "flop_per_launch": sur_rays_launch * FLOP_PER_SUR_RAY,
                     "avg_launch_ms": round(sur_ms / sur_n, 4) if sur_n else None},
    }
    if point is not None:
        res["sweep_point"] = point
    return res


def sky_image_leg(frames, bufs, api, torch, opt, reps=3):
    """The background-image size axis: the step's frames as one batch with the
    procedural checker sky and with equirectangular sky images of growing
    size (seeded random texels generated on the device; the timing does not
    depend on their values).  Each sky ray reads its four bilinear taps from
    the image during shading; reported per size: the step time and the
    shading time per frame."""
    from dataclasses import replace

    gen = torch.Generator(device="cuda")
    gen.manual_seed(11)
    rays = sum(f.camera.width * f.camera.height for f in frames)
    out = {}
    for size in (None, (1024, 512), (4096, 2048), (16384, 8192)):
        tex = None
        if size is None:
            name, fr = "checker", frames
        else:
            tw, th = size
            tex = torch.rand((th, tw, 4), generator=gen, device="cuda", dtype=torch.float32)
            tex[..., 3] = 1.0
            name = f"{tw}x{th}"
            fr = [replace(f, scene=replace(f.scene, sky_tex=tex)) for f in frames]
        b = api.Batch(fr, opt, use_graph=False, images=bufs)
        b.launch()
        torch.cuda.synchronize()
        api.timing_enable(True)
        api.timing_read()
        t0 = time.perf_counter()
        for _ in range(reps):
            b.launch()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        tim = api.timing_read()
        api.timing_enable(False)
        b.close()
        out[name] = {"texture_mb": round(0.0 if tex is None else tex.numel() * 4 / 1e6, 1),
                     "ms_per_step": round(ms, 4),
                     "mrays_per_s": round(rays / (ms * 1e-3) / 1e6, 1),
                     "shade_ms_per_frame": round(tim["shade"][0] / reps / len(frames), 4)}
        log(f"sky images: {name}: {ms:.3f} ms/step")
        del tex
    return out


def batch_leg(args, api, torch):
    """The serving mix: 512 seeded requests (square sizes 128..2048, half with
    a disk) traced in one persistent FP32 + band launch replayed from a
    captured hipGraph, at the autotuned launch shape.  Reports aggregate
    rays/s and per-request completion latency (device clock, from the start
    of the launch)."""
    from paper_2507_16165_amd import autotune, inputs

    frames = inputs.serving_batch(args.batch_requests)
    log(f"batch: {len(frames)} requests, {sum(f.camera.pixels for f in frames)} rays; autotune")
    cache = os.path.join(ROOT, "_build", "autotune.json")
    best = autotune.tune_batch(frames, api.FP32, f"serving_{len(frames)}", cache_path=cache,
                               reps=3, log=log)
    opt = autotune.options_for(best, api.FP32)
    b = api.Batch(frames, opt, use_graph=True)
    b.launch()
    torch.cuda.synchronize()
    runs = []
    t0 = time.perf_counter()
    for _ in range(args.batch_reps):
        b.launch()
        runs.append(b.stats())
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3 / args.batch_reps
    med = sorted(runs, key=lambda r: r["makespan_ms"])[len(runs) // 2]
    b.close()
    # the same requests as one group: a single persistent integrator launch
    # over all 512 requests (set-up, integration and shading once each)
    one = dict(best, batch_groups=1)
    b1 = api.Batch(frames, autotune.options_for(one, api.FP32), use_graph=True)
    b1.launch()
    torch.cuda.synchronize()
    runs1 = []
    for _ in range(args.batch_reps):
        b1.launch()
        runs1.append(b1.stats())
    med1 = sorted(runs1, key=lambda r: r["makespan_ms"])[len(runs1) // 2]
    b1.close()
    return {"requests": med["requests"], "rays": med["rays"], "graph": True,
            "one_launch": {"mrays_per_s": round(med1["mrays_per_s"], 2),
                           "makespan_ms": round(med1["makespan_ms"], 3),
                           "p50_ms": round(med1["p50_ms"], 3), "p99_ms": round(med1["p99_ms"], 3)},
            "autotuned": {k: best[k] for k in ("grid_blocks", "chunk", "refill", "batch_groups",
                                                "candidates_timed")},
            "mrays_per_s": round(med["mrays_per_s"], 2), "makespan_ms": round(med["makespan_ms"], 3),
            "p50_ms": round(med["p50_ms"], 3), "p99_ms": round(med["p99_ms"], 3),
            "min_ms": round(med["min_ms"], 3), "wall_ms_per_launch": round(wall_ms, 3),
            "reps": args.batch_reps}


def cpu_baseline(frames, stride, stride_1t, bufs, opt_fast, api, torch):
    """The CPU FP64 oracle (rtol 1e-10) as it stands, timed on a bounded
    sample of the step's frames: every stride-th row of every frame, one call
    per frame over the listed rows with OpenMP across them (all host threads);
    beside it the same oracle on one thread, on every stride_1t-th row.  On
    the N-thread sample the GPU fast path is compared with the oracle: class
    mismatches outside the critical band and the disk-edge zone, and the
    largest exit-direction error of sky rays outside the band."""
    import numpy as np

    from oracle import ref

    W, H = frames[0].camera.width, frames[0].camera.height
    bc = 3.0 * np.sqrt(3.0)

    def run(rows_of, threads, compare):
        ref.set_threads(threads)
        n, secs, max_err, mism, cls_n = 0, 0.0, 0.0, 0, 0
        for k, f in enumerate(frames):
            c, s = f.camera, f.scene
            cam = ref.camera(c.r, c.incl_deg, c.azim_deg, c.fov_deg, c.width, c.height)
            sc = ref.scene(s.M, r_sky=s.r_sky, disk=s.disk, disk_power=s.disk_power,
                           checker_deg=s.checker_deg)
            rows = rows_of(k)
            t0 = time.perf_counter()
            _, rr = ref.render_row_list(cam, sc, rows)
            secs += time.perf_counter() - t0
            n += len(rows) * W
            if compare:
                _, out = api.render(c, s, opt_fast, rgba=bufs[k], fields=("cls", "exit_dir", "r_hit"))
                idx = (np.asarray(rows)[:, None] * W + np.arange(W)[None, :]).ravel()
                gcls = out["cls"].cpu().numpy()[idx]
                gdir = out["exit_dir"].cpu().numpy()[idx]
                gr = out["r_hit"].cpu().numpy()[idx]
                rc, rb, rdir, rrh = rr.cls[idx], rr.b[idx], rr.exit_dir[idx], rr.r_hit[idx]
                out_band = np.abs(rb - bc * s.M) >= 0.05 * s.M
                rin, rout = s.disk
                r_d = np.where(rc == 2, rrh, gr)
                edge = ((rc == 2) ^ (gcls == 2)) & ((np.abs(r_d - rin) < 1e-4 * rin) |
                                                    (np.abs(r_d - rout) < 1e-4 * rout))
                mism += int(((rc != gcls) & out_band & ~edge).sum())
                cls_n += int(out_band.sum())
                ok = (rc == gcls) & (rc == 0) & out_band
                a, b = rdir[ok], gdir[ok]
                if a.size:
                    ang = np.arctan2(np.linalg.norm(np.cross(a, b), axis=1), np.sum(a * b, 1))
                    max_err = max(max_err, float(ang.max()))
            del rr
        return n, secs, max_err, mism, cls_n

    threads = ref.max_threads()
    log(f"cpu baseline: oracle on every {stride}th row of {len(frames)} frames, {threads} threads")
    n, secs, max_err, mism, cls_n = run(lambda k: list(range(stride // 2, H, stride)), threads, True)
    log(f"cpu baseline: {n} rays in {secs:.1f} s; one thread on every {stride_1t}th row")
    # the one-thread sample: every stride_1t-th row, offset so that it is not
    # a subset of the rows above
    n1, secs1, _, _, _ = run(lambda k: list(range(stride_1t // 2 + 1, H, stride_1t)), 1, False)
    ref.set_threads(threads)
    return {"value": round(n / secs / 1e6, 4), "unit": "Mrays/s", "cores": threads,
            "kind": "oracle",
            "sample": f"every {stride}th row (offset {stride // 2}) of all {len(frames)} frames: "
                      f"{n} rays, FP64 rtol 1e-10, one call per frame over the listed rows, "
                      f"OpenMP across them on {threads} threads",
            "seconds": round(secs, 2), "cpu_model": cpu_model(),
            "single_thread": {"value": round(n1 / secs1 / 1e6, 4), "unit": "Mrays/s", "cores": 1,
                              "sample": f"every {stride_1t}th row (offset {stride_1t // 2 + 1}) of all "
                                        f"{len(frames)} frames: {n1} rays",
                              "seconds": round(secs1, 2)},
            "gpu_fast_path_on_sample": {"rays_outside_band": cls_n,
                                        "class_mismatch_outside_band_and_disk_edge": mism,
                                        "max_exit_err_rad": max_err}}


def cpu_model() -> str:
    """The host CPU's model name, from /proc/cpuinfo ('' where unavailable)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


if __name__ == "__main__":
    sys.exit(main())
