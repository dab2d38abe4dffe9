"""Element-by-element comparison of the GPU path with the CPU oracle.

Tolerances:
  FP64 path: exit-direction angle <= 1e-8 rad, disk hit radius <= 1e-9 rel,
             RGBA |diff| <= 1e-6 on matching pixels.  Both sides run the same
             method at rtol 1e-10; they differ by rounding and by step
             sequences that rounding perturbs, which stays near 1e-10.
  FP32 path: exit-direction angle <= 1e-4 rad, disk hit radius <= 1e-4 rel:
             the FP32 path's error budget (its rtol is 1e-6).
Classification must agree exactly outside the ambiguity zones where several
answers are correct to the method's accuracy:
  - the critical band |b - 3 sqrt(3) M| < 0.05 M (ill-conditioned sweep),
  - disk edges: a DISK/non-DISK disagreement is allowed only if the DISK
    side's hit radius lies within tau_r of r_in or r_out,
  - checker cell boundaries (colour only): oracle theta or varphi within
    tau_theta of a multiple of the cell size.
"""
from __future__ import annotations

import math

import numpy as np

B_CRIT = 3.0 * math.sqrt(3.0)

TOL = {
    "fp64": dict(angle=1e-8, r_rel=1e-9, tau_r=1e-7, tau_theta=1e-8, rgba=1e-6),
    # r_rel: a radial error dr/r = 1e-4 displaces the hit by 1e-4 rad as seen
    # from the centre, the same bound as the exit direction
    "fp32": dict(angle=1e-4, r_rel=1e-4, tau_r=1e-4, tau_theta=1e-4, rgba=1e-6),
}


def angle_between(a, b):
    a = np.asarray(a, float).reshape(-1, 3)
    b = np.asarray(b, float).reshape(-1, 3)
    return np.arctan2(np.linalg.norm(np.cross(a, b), axis=1), np.sum(a * b, 1))


def near_cell_boundary(s, cell_deg, tau):
    s = np.asarray(s, float).reshape(-1, 3)
    theta = np.arctan2(np.hypot(s[:, 0], s[:, 1]), s[:, 2])
    varphi = np.mod(np.arctan2(s[:, 1], s[:, 0]), 2 * np.pi)
    cell = math.radians(cell_deg)

    def near(x):
        f = x / cell
        return np.abs(f - np.round(f)) * cell < tau

    return near(theta) | near(varphi) | (varphi < tau) | (2 * np.pi - varphi < tau)


def compare(ref_rays, gpu: dict, scene, mode: str, mask=None, band=0.05, check_steps=False):
    """ref_rays: oracle.ref.Rays; gpu: dict of numpy arrays (cls, b, phi_end,
    exit_dir, r_hit).  mask: which rays to compare (default all).  Returns a
    summary dict; raises AssertionError on any violation."""
    t = TOL[mode]
    n = ref_rays.cls.shape[0]
    m = np.ones(n, bool) if mask is None else np.asarray(mask, bool)
    M = scene.M
    rc, gc = ref_rays.cls.astype(int), np.asarray(gpu["cls"]).astype(int)
    b = ref_rays.b
    in_band = (np.abs(b - B_CRIT * M) < band * M) & (M > 0)
    mism = (rc != gc) & m & ~in_band
    if scene.disk is not None and mism.any():
        rin, rout = scene.disk
        r_dsk = np.where(rc == 2, ref_rays.r_hit, np.asarray(gpu["r_hit"]))
        edge = (np.abs(r_dsk - rin) < t["tau_r"] * rin) | (np.abs(r_dsk - rout) < t["tau_r"] * rout)
        one_disk = (rc == 2) ^ (gc == 2)
        mism &= ~(one_disk & edge)
    bad = np.nonzero(mism)[0]
    assert bad.size == 0, (f"{bad.size} class mismatches outside ambiguity zones, first: "
                           f"{[(int(i), int(rc[i]), int(gc[i]), float(b[i])) for i in bad[:5]]}")
    if "b" in gpu:
        ok = m & (rc != 4)
        np.testing.assert_allclose(np.asarray(gpu["b"])[ok], b[ok], rtol=1e-12)
    same = m & (rc == gc) & ~in_band
    sky = same & (rc == 0)
    ang = angle_between(ref_rays.exit_dir[sky], np.asarray(gpu["exit_dir"])[sky])
    max_ang = float(ang.max()) if ang.size else 0.0
    assert max_ang <= t["angle"], f"max exit angle {max_ang} > {t['angle']}"
    dsk = same & (rc == 2)
    max_r = 0.0
    if dsk.any():
        rr = np.abs(np.asarray(gpu["r_hit"])[dsk] / ref_rays.r_hit[dsk] - 1.0)
        max_r = float(rr.max())
        assert max_r <= t["r_rel"], f"max disk radius rel err {max_r} > {t['r_rel']}"
        da = angle_between(ref_rays.exit_dir[dsk], np.asarray(gpu["exit_dir"])[dsk])
        assert da.max() <= t["angle"]
    return dict(n=int(m.sum()), band=int((in_band & m).sum()), sky=int(sky.sum()),
                disk=int(dsk.sum()), captured=int((same & (rc == 1)).sum()),
                mismatch_in_zones=int(((rc != gc) & m).sum()), max_angle=max_ang, max_r_rel=max_r,
                p99_angle=float(np.percentile(ang, 99)) if ang.size else 0.0)


def compare_rgba(ref_rgba, ref_rays, gpu_rgba, gpu_cls, scene, mode, mask=None, band=0.05):
    """Colour parity on pixels whose class agrees, outside the critical band
    and the checker-boundary zone."""
    t = TOL[mode]
    R = np.asarray(ref_rgba).reshape(-1, 4)
    G = np.asarray(gpu_rgba).reshape(-1, 4)
    n = R.shape[0]
    m = np.ones(n, bool) if mask is None else np.asarray(mask, bool)
    rc, gc = ref_rays.cls.astype(int), np.asarray(gpu_cls).astype(int)
    in_band = (np.abs(ref_rays.b - B_CRIT * scene.M) < band * scene.M) & (scene.M > 0)
    zone = near_cell_boundary(ref_rays.exit_dir, scene.checker_deg, t["tau_theta"]) & (rc == 0)
    ok = m & (rc == gc) & ~in_band & ~zone
    d = np.abs(R[ok] - G[ok])
    # disk colour follows (r/r_in)^power: relative error ~ |power| * r_rel
    dsk = (rc[ok] == 2)
    tol = np.where(dsk[:, None], 4.0 * t["r_rel"] * np.abs(R[ok]) + 1e-7, t["rgba"])
    bad = np.nonzero(np.any(d > tol, axis=1))[0]
    assert bad.size == 0, f"{bad.size} colour mismatches, first diffs {d[bad[:3]]}"
    return int(ok.sum())
