"""Element-by-element comparison of the GPU path with the CPU oracle.

Tolerances:
  FP64 path: exit-direction angle <= 1e-8 rad, disk hit radius <= 1e-9 rel,
             RGBA |diff| <= 1e-6 on matching pixels.  Both sides run the same
             method at rtol 1e-10; they differ by rounding and by step
             sequences that rounding perturbs, which stays near 1e-10.
  FP32 path: exit-direction angle <= 1e-4 rad (the stated target), disk hit
             radius <= 1e-4 relative.  The radius bound is set by what a
             radial error does to the image.  The pixel's ray is fixed by the
             camera, so a radial error only changes where on the disk that
             ray samples the emissivity I = (r / r_in)^-3: the relative colour
             error is 3 dr/r <= 3e-4, a twelfth of one 8-bit display level
             (1/255) at the brightest disk pixel, and the disk edges move by
             dr, which the disk-edge ambiguity zone (tau_r = 1e-4 r) covers.
             The FP32 integrator (rtol 1e-6) measured 1.1e-5 to 5e-5 here, so
             the 1e-5 first proposed for this bound is not met; the colour
             argument above is what 1e-4 rests on.
Classification must agree exactly outside the ambiguity zones where several
answers are correct to the method's accuracy:
  - the critical band |b - 3 sqrt(3) M| < 0.05 M (ill-conditioned sweep),
  - disk edges: a DISK/non-DISK disagreement is allowed only if the DISK
    side's hit radius lies within tau_r of r_in or r_out,
  - checker cell boundaries (colour only): oracle theta within tau_theta,
    or varphi within tau_theta / sin(theta), of a multiple of the cell size
    (a direction error of tau_theta moves the azimuth by up to that much).

Band rays.  Inside the band the FP64 integrator still serves the rays (in
FP32 mode too), and rays of equal class are compared with a bound from the
conditioning: near b_c the sweep grows like -ln(b - b_c), so a ray's end
moves by db / |b - b_c| when its impact parameter moves by db.  Integration
error shows up as a drift of the first integral E = w^2 + u^2 - 2 M u^3 =
1/b^2; with each side's relative drift at most D, the two effective impact
parameters differ by at most b D, and the ends by
    b D / |b - b_c|  (radians of azimuth),
on top of the bounds outside the band.  D = 1e-10 at rtol 1e-10 (the oracle's
drift on band rays is a few 1e-11; pinned in test_oracle_pins).  In FP32 mode
the band is integrated at rtol_band = 1e-9, so D = 1e-9 + 1e-10 there.  Rays
within 1e-3 M of b_c are left out: there the bound reaches the size of the
answer.
For a disk hit the same azimuth error moves the radius by r |w| / u per
radian, with w^2 = 1/b^2 - u^2 + 2 M u^3 at u = 1/r.
"""
from __future__ import annotations

import math

import numpy as np

B_CRIT = 3.0 * math.sqrt(3.0)

TOL = {
    "fp64": dict(angle=1e-8, r_rel=1e-9, tau_r=1e-7, tau_theta=1e-8, rgba=1e-6),
    "fp32": dict(angle=1e-4, r_rel=1e-4, tau_r=1e-4, tau_theta=1e-4, rgba=1e-6),
}

# relative drift of the first integral allowed between the two sides' band
# rays: FP64 mode and the oracle integrate at rtol 1e-10; FP32 mode's band at
# rtol_band 1e-9 (the library's default), plus the oracle's 1e-10
BAND_DRIFT = {"fp64": 1e-10, "fp32": 1e-9 + 1e-10}
BAND_MIN = 1e-3         # band rays closer than this to b_c (units of M) are not compared


def angle_between(a, b):
    a = np.asarray(a, float).reshape(-1, 3)
    b = np.asarray(b, float).reshape(-1, 3)
    return np.arctan2(np.linalg.norm(np.cross(a, b), axis=1), np.sum(a * b, 1))


def band_extra(b, M, mode="fp64"):
    """Azimuth bound added for a band ray with impact parameter b (FP64
    integration on both sides): b D / |b - b_c|, D = BAND_DRIFT[mode]."""
    b = np.asarray(b, float)
    d = np.abs(b - B_CRIT * M)
    with np.errstate(divide="ignore"):
        return np.where(d > 0, b * BAND_DRIFT[mode] / d, np.inf)


def radius_per_azimuth(b, r, M):
    """|dr/dphi| / r = |w| / u on the orbit of impact parameter b at radius r
    (0 where r is not a hit radius, r <= 0)."""
    r = np.broadcast_to(np.asarray(r, float), np.shape(b)).copy()
    b = np.asarray(b, float)
    out = np.zeros(r.shape)
    h = (r > 0.0) & (b > 0.0) & np.isfinite(r)
    u = 1.0 / r[h]
    w2 = np.maximum(1.0 / (b[h] * b[h]) - u * u + 2.0 * M * u ** 3, 0.0)
    out[h] = np.sqrt(w2) / u
    return out


def near_cell_boundary(s, cell_deg, tau):
    """Exit directions within tau radians of a checker boundary: a direction
    error of tau moves theta by up to tau and the azimuth varphi by up to
    tau / sin(theta), so the azimuth zone widens toward the poles."""
    s = np.asarray(s, float).reshape(-1, 3)
    theta = np.arctan2(np.hypot(s[:, 0], s[:, 1]), s[:, 2])
    varphi = np.mod(np.arctan2(s[:, 1], s[:, 0]), 2 * np.pi)
    cell = math.radians(cell_deg)
    tau_phi = tau / np.maximum(np.sin(theta), 1e-300)

    def near(x, t):
        f = x / cell
        return np.abs(f - np.round(f)) * cell < t

    return near(theta, tau) | near(varphi, tau_phi) | (varphi < tau_phi) | (2 * np.pi - varphi < tau_phi)


def _zones(ref_rays, scene, band, mode):
    M = scene.M
    b = ref_rays.b
    dist = np.abs(b - B_CRIT * M)
    in_band = (dist < band * M) & (M > 0)
    deep = in_band & (dist < BAND_MIN * M)          # not compared at all
    shallow = in_band & ~deep                       # compared with the band bound
    extra = np.where(shallow, band_extra(b, M, mode), 0.0)
    return in_band, deep, shallow, extra


def _disk_edge(r, scene, tau_rel):
    rin, rout = scene.disk
    return (np.abs(r - rin) < tau_rel * rin) | (np.abs(r - rout) < tau_rel * rout)


def compare(ref_rays, gpu: dict, scene, mode: str, mask=None, band=0.05, check_steps=False):
    """ref_rays: oracle.ref.Rays; gpu: dict of numpy arrays (cls, b, phi_end,
    exit_dir, r_hit).  mask: which rays to compare (default all).  Band rays
    (|b - b_c| in [1e-3, 0.05] M) of equal class are compared with the band
    bound; in FP32 mode their phi_end (FP64-integrated) is held to the FP64
    band bound.  Returns a summary dict; raises AssertionError on any
    violation."""
    t = TOL[mode]
    n = ref_rays.cls.shape[0]
    m = np.ones(n, bool) if mask is None else np.asarray(mask, bool)
    M = scene.M
    rc, gc = ref_rays.cls.astype(int), np.asarray(gpu["cls"]).astype(int)
    b = ref_rays.b
    in_band, deep, shallow, extra = _zones(ref_rays, scene, band, mode)
    g_r = np.asarray(gpu["r_hit"]) if "r_hit" in gpu else np.zeros(n)
    # class: exact outside the band and the disk-edge zone; inside the band
    # (|b - b_c| >= 1e-3 M) exact outside a disk-edge zone widened by the band bound
    mism = (rc != gc) & m & ~deep
    if scene.disk is not None and mism.any():
        r_dsk = np.where(rc == 2, ref_rays.r_hit, g_r)
        one_disk = (rc == 2) ^ (gc == 2)
        tau = t["tau_r"] + np.where(shallow, extra * radius_per_azimuth(b, r_dsk, M), 0.0)
        edge = np.zeros(n, bool)
        nz = r_dsk > 0
        edge[nz] = _disk_edge(r_dsk[nz], scene, tau[nz])
        mism &= ~(one_disk & edge)
    bad = np.nonzero(mism)[0]
    assert bad.size == 0, (f"{bad.size} class mismatches outside ambiguity zones, first: "
                           f"{[(int(i), int(rc[i]), int(gc[i]), float(b[i])) for i in bad[:5]]}")
    if "b" in gpu:
        ok = m & (rc != 4)
        np.testing.assert_allclose(np.asarray(gpu["b"])[ok], b[ok], rtol=1e-12)
    same = m & (rc == gc) & ~deep
    sky = same & (rc == 0)
    ang = angle_between(ref_rays.exit_dir[sky], np.asarray(gpu["exit_dir"])[sky])
    lim = t["angle"] + extra[sky]
    worst = float((ang / lim).max()) if ang.size else 0.0
    assert worst <= 1.0, (f"exit angle over its bound by {worst:.3g}x: "
                          f"{ang[np.argmax(ang / lim)]} vs {lim[np.argmax(ang / lim)]}")
    out_sky = sky & ~in_band
    max_ang = float(angle_between(ref_rays.exit_dir[out_sky], np.asarray(gpu["exit_dir"])[out_sky]).max()) \
        if out_sky.any() else 0.0
    dsk = same & (rc == 2)
    max_r = 0.0
    if dsk.any():
        rr = np.abs(g_r[dsk] / ref_rays.r_hit[dsk] - 1.0)
        rlim = t["r_rel"] + extra[dsk] * radius_per_azimuth(b[dsk], ref_rays.r_hit[dsk], M)
        wr = float((rr / rlim).max())
        assert wr <= 1.0, f"disk radius over its bound by {wr:.3g}x"
        max_r = float(rr[~in_band[dsk]].max()) if (~in_band[dsk]).any() else 0.0
        da = angle_between(ref_rays.exit_dir[dsk], np.asarray(gpu["exit_dir"])[dsk])
        assert (da / (t["angle"] + extra[dsk])).max() <= 1.0
    # band rays' end azimuth: FP64-integrated in both modes
    band_cmp = same & shallow & ((rc == 0) | (rc == 2))
    max_band_phi = 0.0
    if band_cmp.any() and "phi_end" in gpu:
        dphi = np.abs(np.asarray(gpu["phi_end"])[band_cmp] - ref_rays.phi_end[band_cmp])
        plim = TOL["fp64"]["angle"] + extra[band_cmp]
        wp = float((dphi / plim).max())
        assert wp <= 1.0, f"band ray end azimuth over its bound by {wp:.3g}x"
        max_band_phi = float(dphi.max())
    return dict(n=int(m.sum()), band=int((in_band & m).sum()), sky=int(sky.sum()),
                disk=int(dsk.sum()), captured=int((same & (rc == 1)).sum()),
                band_compared=int((same & shallow).sum()),
                mismatch_in_zones=int(((rc != gc) & m).sum()), max_angle=max_ang, max_r_rel=max_r,
                max_band_phi=max_band_phi,
                p99_angle=float(np.percentile(ang, 99)) if ang.size else 0.0)


def compare_rgba(ref_rgba, ref_rays, gpu_rgba, gpu_cls, scene, mode, mask=None, band=0.05):
    """Colour parity on pixels whose class agrees, outside the checker-boundary
    zone (band rays within 1e-3 M of b_c left out; other band rays with their
    zones widened by the band bound)."""
    t = TOL[mode]
    R = np.asarray(ref_rgba).reshape(-1, 4)
    G = np.asarray(gpu_rgba).reshape(-1, 4)
    n = R.shape[0]
    m = np.ones(n, bool) if mask is None else np.asarray(mask, bool)
    rc, gc = ref_rays.cls.astype(int), np.asarray(gpu_cls).astype(int)
    _, deep, shallow, extra = _zones(ref_rays, scene, band, mode)
    zone = np.zeros(n, bool)
    sky = rc == 0
    zone[sky] = near_cell_boundary(ref_rays.exit_dir[sky], scene.checker_deg,
                                   t["tau_theta"] + extra[sky]) if sky.any() else zone[sky]
    ok = m & (rc == gc) & ~deep & ~zone
    d = np.abs(R[ok] - G[ok])
    # disk colour follows (r/r_in)^power: relative error ~ |power| * r_rel
    dsk = (rc[ok] == 2)
    r_tol = t["r_rel"] + extra[ok] * radius_per_azimuth(ref_rays.b[ok], np.where(dsk, ref_rays.r_hit[ok], 0.0), scene.M)
    tol = np.where(dsk[:, None], 4.0 * r_tol[:, None] * np.abs(R[ok]) + 1e-7, t["rgba"])
    bad = np.nonzero(np.any(d > tol, axis=1))[0]
    assert bad.size == 0, f"{bad.size} colour mismatches, first diffs {d[bad[:3]]}"
    return int(ok.sum())


def _decode_class(G, scene):
    """Class of a GPU pixel from its colour alone (batches return images
    only): black is captured/unresolved, equal grey levels are sky, a disk
    colour (I, 0.6 I, 0.2 I) is a disk hit at r = r_in I^(1/power)."""
    G = np.asarray(G, np.float64).reshape(-1, 4)
    cls = np.full(G.shape[0], 0, int)
    black = np.all(G[:, :3] == 0.0, axis=1)
    cls[black] = 1
    disk = (~black) & (np.abs(G[:, 1] - 0.6 * G[:, 0]) <= 1e-5 * G[:, 0] + 1e-12) & (G[:, 0] != G[:, 2])
    cls[disk] = 2
    r = np.zeros(G.shape[0])
    if scene.disk is not None and disk.any():
        r[disk] = scene.disk[0] * np.power(G[disk, 0], 1.0 / scene.disk_power)
    return cls, r


def compare_image(ref_rgba, ref_rays, gpu_rgba, scene, mode, mask=None, band=0.05, sky_tex=None):
    """Pixel parity of an image for which the GPU side returned colours only
    (batched requests).  Outside the ambiguity zones -- band rays within
    1e-3 M of b_c, checker-cell boundaries, and disk edges (the GPU's hit
    radius is read back from its disk colour) -- every pixel must match the
    oracle's colour to the path's bounds; a class difference there changes
    the colour and fails.  With a sky image (sky_tex, (h, w, 4)) sky colours
    are bounded by the image's largest texel step times the texel
    displacement the exit-angle bound allows.  Returns the number of pixels
    compared."""
    t = TOL[mode]
    R = np.asarray(ref_rgba, np.float64).reshape(-1, 4)
    G = np.asarray(gpu_rgba, np.float64).reshape(-1, 4)
    n = R.shape[0]
    m = np.ones(n, bool) if mask is None else np.asarray(mask, bool)
    rc = ref_rays.cls.astype(int).copy()
    rc[rc == 3] = 1      # unresolved shades like captured
    gc, gr = _decode_class(G, scene)
    _, deep, shallow, extra = _zones(ref_rays, scene, band, mode)
    zone = deep.copy()
    sky = rc == 0
    if sky.any() and sky_tex is None:
        zone[sky] |= near_cell_boundary(ref_rays.exit_dir[sky], scene.checker_deg,
                                        t["tau_theta"] + extra[sky])
    if scene.disk is not None:
        r_dsk = np.where(rc == 2, ref_rays.r_hit, gr)
        one_disk = (rc == 2) ^ (gc == 2)
        tau = t["tau_r"] + extra * radius_per_azimuth(ref_rays.b, r_dsk, scene.M)
        nz = r_dsk > 0
        e = np.zeros(n, bool)
        e[nz] = _disk_edge(r_dsk[nz], scene, tau[nz])
        zone |= one_disk & e
    ok = m & ~zone
    tol = np.full(n, t["rgba"])
    dsk = rc == 2
    if dsk.any():
        r_tol = t["r_rel"] + extra[dsk] * radius_per_azimuth(ref_rays.b[dsk], ref_rays.r_hit[dsk], scene.M)
        tol[dsk] = 0.0  # per channel below
    if sky_tex is not None and sky.any():
        tex = np.asarray(sky_tex, np.float64)
        step = max(np.abs(np.diff(tex, axis=1)).max(), np.abs(np.diff(tex, axis=0)).max())
        s_ = ref_rays.exit_dir[sky]
        sin_t = np.maximum(np.hypot(s_[:, 0], s_[:, 1]), 1e-3)
        Ht, Wt = tex.shape[:2]
        tol[sky] = step * (Wt / (2 * np.pi) / sin_t + Ht / np.pi) * (t["angle"] + extra[sky]) + 2e-6
    tol4 = np.repeat(tol[:, None], 4, axis=1)
    if dsk.any():
        tol4[dsk] = 4.0 * r_tol[:, None] * np.abs(R[dsk]) + 1e-7
    d = np.abs(R - G)
    bad = np.nonzero(ok & np.any(d > tol4, axis=1))[0]
    assert bad.size == 0, (f"{bad.size} pixels differ from the oracle outside the zones, first: "
                           f"ref {R[bad[:3]]} gpu {G[bad[:3]]}")
    return int(ok.sum())
