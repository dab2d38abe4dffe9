"""Pins of the CPU FP64 oracle against closed forms, quadrature, invariants and
brute-force references -- never against itself.

Each test names the property of the paper's method it checks (Eq. (1) and the
text after it; the initial-condition and stepping recipe of the section on GSL
ODE approximation).  Plausible mistakes each test would catch are listed in its
docstring.
"""
import math

import mpmath
import numpy as np
import pytest

import quadrature as Q

RNG = np.random.default_rng(20250716)


def _plane_rays(r0, alpha, M=1.0):
    """Rays from (r0, 0, 0) at angle alpha (rad) from the outward radial, in
    the xy-plane."""
    r0 = np.asarray(r0, float)
    alpha = np.asarray(alpha, float)
    o = np.stack([r0, np.zeros_like(r0), np.zeros_like(r0)], -1)
    d = np.stack([np.cos(alpha), np.sin(alpha), np.zeros_like(alpha)], -1)
    return o, d


def _b_geom(M, r0, sin_psi):
    """Impact parameter of the straight-line initial direction, from the
    first integral written with the angle psi to the radial:
    1/b^2 = u0^2 / sin^2 psi - 2 M u0^3."""
    u0 = 1.0 / r0
    return 1.0 / np.sqrt(u0 * u0 / sin_psi**2 - 2.0 * M * u0**3)


# --------------------------------------------------------------------------
# Stepper
# --------------------------------------------------------------------------
def test_dopri5_local_order_against_taylor_reference(ref):
    """One Dormand-Prince step on the nonlinear orbit system (M = 1, u up to
    0.25, near the photon sphere) against a 30-digit Taylor-series solution
    (mpmath.odefun).  The 5th-order solution's local error must scale like
    h^6 and the embedded error estimate like h^5.  A wrong tableau entry
    breaks an order condition and fails the ratio test."""
    mpmath.mp.dps = 30
    M = 1.0
    # states where the leading local-error coefficient is well away from zero
    for y0 in ((0.1, 0.05), (0.15, 0.1), (0.25, -0.1)):
        sol = mpmath.odefun(lambda t, y: [y[1], 3 * M * y[0] ** 2 - y[0]], 0,
                            list(map(mpmath.mpf, y0)))
        errs, ests = [], []
        for h in (0.2, 0.1, 0.05):
            yo, e = ref.dopri5_step(M, y0, h)
            ex = sol(mpmath.mpf(h))
            errs.append(max(abs(yo[0] - float(ex[0])), abs(yo[1] - float(ex[1]))))
            ests.append(max(abs(e[0]), abs(e[1])))
        for a, b in zip(errs, errs[1:]):
            assert 55 < a / b < 95, (y0, errs)  # ~2^6 = 64
        for a, b in zip(ests, ests[1:]):
            assert 28 < a / b < 36, (y0, ests)  # ~2^5 = 32


def test_dopri5_flat_space_rotation(ref):
    """M = 0 makes the system a rotation: the exact step is (cos h, -sin h)
    from (1, 0).  Local error of a 5th-order method is O(h^6)."""
    for h in (0.1, 0.3):
        yo, _ = ref.dopri5_step(0.0, (1.0, 0.0), h)
        assert abs(yo[0] - math.cos(h)) < 2e-3 * h**6
        assert abs(yo[1] + math.sin(h)) < 2e-3 * h**6


# --------------------------------------------------------------------------
# Flat space: straight lines (M = 0)
# --------------------------------------------------------------------------
def test_m0_rays_are_straight_lines(ref):
    """With M = 0 Eq. (1) is u'' + u = 0, whose solutions are straight lines.
    The end point on the sky sphere must be the line/sphere intersection
    C + t d with |C + t d| = R (closed form), within the tolerance-bound error, and b must equal
    |C x d|.  Catches a wrong sign in the u term of Eq. (1), a wrong initial
    slope, or a broken sky-crossing refinement."""
    n = 400
    R = 1000.0
    o = RNG.normal(size=(n, 3))
    o *= (RNG.uniform(1.0, 600.0, n) / np.linalg.norm(o, axis=1))[:, None]
    d = RNG.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    sc = ref.scene(M=0.0, r_sky=R)
    od = np.sum(o * d, 1)
    t = -od + np.sqrt(od**2 - (np.sum(o * o, 1) - R * R))
    p = (o + t[:, None] * d) / R
    # the error bound follows the tolerance: ~rtol at 1e-10, far below at 1e-13
    for rtol, bound in ((1e-10, 2e-10), (1e-13, 1e-12)):
        out = ref.trace_rays(o, d, sc, ref.options(rtol=rtol))
        assert np.all(out.cls == ref.SKY)
        ang = np.arctan2(np.linalg.norm(np.cross(p, out.exit_dir), axis=1), np.sum(p * out.exit_dir, 1))
        assert ang.max() < bound, (rtol, ang.max())
    b = np.linalg.norm(np.cross(o, d), axis=1)
    np.testing.assert_allclose(out.b, b, rtol=1e-12)


def test_m0_disk_hits_match_line_plane_intersection(ref):
    """M = 0 with a disk: the hit is the line's crossing of z = 0 (closed form
    t = -Cz/dz), a DISK hit iff r_in <= |hit| <= r_out.  Catches a wrong
    disk-crossing angle or a missed landing."""
    n = 600
    R, rin, rout = 1000.0, 6.0, 40.0
    o = RNG.normal(size=(n, 3))
    o *= (RNG.uniform(20.0, 80.0, n) / np.linalg.norm(o, axis=1))[:, None]
    # aim near the origin so many rays cross the disk
    tgt = RNG.normal(scale=25.0, size=(n, 3))
    d = tgt - o
    d /= np.linalg.norm(d, axis=1)[:, None]
    sc = ref.scene(M=0.0, r_sky=R, disk=(rin, rout))
    out = ref.trace_rays(o, d, sc)
    t = -o[:, 2] / d[:, 2]
    hit = o + t[:, None] * d
    rh = np.linalg.norm(hit, axis=1)
    expect_disk = (t > 0) & (rh >= rin) & (rh <= rout)
    edge = (np.abs(rh - rin) < 1e-7) | (np.abs(rh - rout) < 1e-7)
    ok = ~edge
    assert expect_disk.sum() > 100
    np.testing.assert_array_equal(out.cls[ok] == ref.DISK, expect_disk[ok])
    m = expect_disk & ok
    np.testing.assert_allclose(out.r_hit[m], rh[m], rtol=1e-10)
    u = hit[m] / rh[m][:, None]
    ang = np.arctan2(np.linalg.norm(np.cross(u, out.exit_dir[m]), axis=1), np.sum(u * out.exit_dir[m], 1))
    assert ang.max() < 1e-10


def test_dphi_flat_is_the_straight_line_sweep(ref):
    """The flat-space sweep used for surrogate labels equals the M = 0 exit
    azimuth of the same ray (any b < r0) and equals its closed form."""
    r0, R = 80.0, 1000.0
    sc = ref.scene(M=0.0, r_sky=R)
    for psi in (0.05, 0.4, 1.2):
        alpha = math.pi - psi
        o, d = _plane_rays([r0], [alpha])
        out = ref.trace_rays(o, d, sc)
        b = r0 * math.sin(psi)
        assert abs(ref.dphi_flat(0.0, b, r0, R) - out.phi_end[0]) < 1e-11
    # closed form: pi - psi - asin(r0 sin psi / R)
    assert abs(ref.dphi_flat(0.0, 40.0, r0, R) - (math.pi - math.pi / 6 - math.asin(0.04))) < 1e-14


# --------------------------------------------------------------------------
# First integral, capture threshold, exit azimuth
# --------------------------------------------------------------------------
def test_first_integral_conserved(ref):
    """E = w^2 + u^2 - 2 M u^3 = 1/b^2 is constant along every solution of
    Eq. (1) with the '+' sign; drift along each ray must stay below 2e-9 at
    rtol 1e-10 (cfg 64x64, r = 30 M)."""
    cam = ref.camera(30.0, 90.0, 0.0, 60.0, 64, 64)
    _, out = ref.render(cam, ref.scene(1.0))
    assert out.e_drift.max() < 2e-9, out.e_drift.max()


def test_capture_exactly_below_critical_impact_parameter(ref):
    """An ingoing ray from r0 > 3M is captured iff b < 3 sqrt(3) M (closed
    form of the effective-potential maximum at u = 1/(3M)); outgoing rays
    always escape.  Rays with |b - b_c| < 1e-3 M are excluded (ill-posed)."""
    for M in (1.0, 2.0):
        n = 3000
        r0 = M * RNG.uniform(3.3, 300.0, n)
        alpha = RNG.uniform(0.0, math.pi, n)
        o, d = _plane_rays(r0, alpha)
        out = ref.trace_rays(o, d, ref.scene(M))
        b = _b_geom(M, r0, np.sin(alpha))
        bc = Q.B_CRIT * M
        ok = np.abs(b - bc) > 1e-3 * M
        ingoing = np.cos(alpha) < 0
        expect = ingoing & (b < bc)
        np.testing.assert_array_equal((out.cls == ref.CAPTURED)[ok], expect[ok])
        assert np.all(out.cls[ok & ~expect] == ref.SKY)
        np.testing.assert_allclose(out.b, b, rtol=1e-12)


def _exit_cases(M, n, seed):
    rng = np.random.default_rng(seed)
    cases = []
    while len(cases) < n:
        r0 = M * rng.uniform(4.0, 300.0)
        alpha = rng.uniform(0.01, math.pi - 0.01)
        b = _b_geom(M, r0, math.sin(alpha))
        ingoing = math.cos(alpha) < 0
        if ingoing and b < Q.B_CRIT * M + 0.05 * M:
            continue
        cases.append((r0, alpha, b, ingoing))
    return cases


@pytest.mark.parametrize("M", [1.0, 0.5])
def test_exit_azimuth_matches_quadrature(ref, M):
    """Exit azimuth of escaping rays against the quadrature of
    dphi = du / sqrt(1/b^2 - u^2 + 2 M u^3) through the turning point:
    within 1e-8 rad at rtol 1e-10 (the method's own tolerance bound).
    Catches any error in the right-hand side (sign, factor 3, power of u)."""
    R = 1000.0 * M
    cases = _exit_cases(M, 60, 7 if M == 1.0 else 8)
    o, d = _plane_rays([c[0] for c in cases], [c[1] for c in cases])
    out = ref.trace_rays(o, d, ref.scene(M, r_sky=R))
    assert np.all(out.cls == ref.SKY)
    for k, (r0, alpha, b, ingoing) in enumerate(cases):
        want = Q.exit_phi(M, b, r0, R, ingoing)
        assert abs(out.phi_end[k] - want) < 1e-8, (r0, alpha, b, out.phi_end[k], want)


def test_error_shrinks_with_tolerance(ref):
    """The paper: a smaller step/tolerance gives a more accurate trajectory.
    Max exit-azimuth error against quadrature must fall by >= 30x per two
    decades of rtol."""
    M, R = 1.0, 1000.0
    cases = _exit_cases(M, 40, 11)
    o, d = _plane_rays([c[0] for c in cases], [c[1] for c in cases])
    want = np.array([Q.exit_phi(M, c[2], c[0], R, c[3]) for c in cases])
    errs = []
    for rtol in (1e-5, 1e-7, 1e-9):
        out = ref.trace_rays(o, d, ref.scene(M), ref.options(rtol=rtol))
        errs.append(np.abs(out.phi_end - want).max())
    assert errs[0] > 30 * errs[1] and errs[1] > 30 * errs[2], errs
    assert errs[0] < 1e-3


def test_weak_field_deflection(ref):
    """Weak field: the sweep matches the first-order solution
    u = sin(phi)/b + (M/b^2)(1 + cos^2 phi) up to O((M/b)^2), and the
    deflection beyond the straight line tends to 4M/b for distant endpoints.
    A wrong coefficient in 3 M u^2 shifts both at first order."""
    M, r0, R = 1.0, 500.0, 1000.0
    for b in (40.0, 80.0, 150.0, 300.0):
        # ingoing ray from r0 with impact parameter b
        sin_psi = (1.0 / r0) / math.sqrt(1.0 / b**2 + 2 * M / r0**3)
        o, d = _plane_rays([r0], [math.pi - math.asin(sin_psi)])
        out = ref.trace_rays(o, d, ref.scene(M, r_sky=R))
        got = out.phi_end[0]
        assert abs(got - Q.weak_field_sweep(M, b, r0, R)) < 3.0 * (15 * math.pi / 4) * (M / b) ** 2
    # far endpoints: deflection -> 4M/b (+ (15 pi/4)(M/b)^2 at second order)
    r0, R, b = 1e6, 1e7, 1000.0
    sin_psi = (1.0 / r0) / math.sqrt(1.0 / b**2 + 2 * M / r0**3)
    psi = math.asin(sin_psi)
    o, d = _plane_rays([r0], [math.pi - psi])
    out = ref.trace_rays(o, d, ref.scene(M, r_sky=R))
    flat = math.pi - psi - math.asin(r0 * sin_psi / R)
    defl = out.phi_end[0] - flat
    assert abs(defl - 4 * M / b) < (15 * math.pi / 4 + 1.0) * (M / b) ** 2, defl


def test_periapsis_approaches_photon_sphere(ref):
    """Closed form: the turning point u2 of a ray with b -> b_c+ tends to
    1/(3M); a ray with b slightly above b_c winds (sweep grows like
    -log(b - b_c)) and still escapes.  Checked through the sweep: the oracle's
    exit azimuth equals the quadrature, whose turning point comes from the
    cubic's roots."""
    M, r0, R = 1.0, 30.0, 1000.0
    for db in (1e-2, 1e-4):
        b = Q.B_CRIT + db
        sin_psi = (1.0 / r0) / math.sqrt(1.0 / b**2 + 2 * M / r0**3)
        o, d = _plane_rays([r0], [math.pi - math.asin(sin_psi)])
        out = ref.trace_rays(o, d, ref.scene(M, r_sky=R))
        assert out.cls[0] == ref.SKY
        assert abs(Q.turning_point(M, b) - 1.0 / 3.0) < 2.0 * math.sqrt(db)
        # the problem is ill-conditioned near b_c: the sweep error grows like
        # rtol / (b - b_c), and falls with the tolerance
        want = Q.exit_phi(M, out.b[0], r0, R, True)
        assert abs(out.phi_end[0] - want) < 1e-10 / db
        tight = ref.trace_rays(o, d, ref.scene(M, r_sky=R), ref.options(rtol=1e-13))
        assert abs(tight.phi_end[0] - want) < 1e-13 / db


def test_band_rays_within_the_conditioning_bound(ref):
    """Rays in the critical band, 1e-3 M <= |b - b_c| <= 0.05 M, from cameras
    at 10-100 M: the first integral drifts by at most 1e-10 relative along
    each ray (rtol 1e-10), and the exit azimuth of the escaping ones matches
    the quadrature within 1e-8 + b 1e-10 / (b - b_c).  That is the bound the
    GPU parity tests apply to band rays: near b_c the sweep behaves like
    -ln(b - b_c), so a drift D of E = 1/b^2 moves the end by about
    b D / (2 (b - b_c)).  A controller that let the drift grow, or a wrong
    coefficient that only shows near the photon sphere, fails here."""
    rng = np.random.default_rng(31)
    M = 1.0
    rows = []
    for _ in range(120):
        delta = math.exp(rng.uniform(math.log(1e-3), math.log(0.05)))
        if rng.uniform() < 0.3:
            delta = -delta
        b = Q.B_CRIT + delta
        r0 = rng.uniform(10.0, 100.0)
        sin_psi = (1.0 / r0) / math.sqrt(1.0 / b**2 + 2 * M / r0**3)
        o, d = _plane_rays([r0], [math.pi - math.asin(sin_psi)])
        out = ref.trace_rays(o, d, ref.scene(M))
        rows.append((delta, r0, out))
    for delta, r0, out in rows:
        assert out.e_drift[0] <= 1e-10, (delta, out.e_drift[0])
        if delta > 0:
            assert out.cls[0] == ref.SKY
            want = Q.exit_phi(M, out.b[0], r0, 1000.0, True)
            bound = 1e-8 + out.b[0] * 1e-10 / (out.b[0] - Q.B_CRIT)
            assert abs(out.phi_end[0] - want) <= bound, (delta, r0, out.phi_end[0] - want, bound)
        else:
            assert out.cls[0] == ref.CAPTURED


def test_disk_hit_radius_matches_quadrature(ref):
    """Camera on the +z axis: every ray's orbital plane contains the z axis,
    so it meets the disk plane exactly at phi = pi/2.  The hit radius must be
    the u with phi(u) = pi/2 from the quadrature (before or after the turning
    point), to 1e-8 relative."""
    from scipy.optimize import brentq
    M, r0, R = 1.0, 40.0, 1000.0
    rin, rout = 2.5, 200.0
    sc = ref.scene(M, r_sky=R, disk=(rin, rout))
    for psi_deg in (3.0, 8.0, 15.0, 25.0, 35.0):
        psi = math.radians(psi_deg)
        o = np.array([[0.0, 0.0, r0]])
        d = np.array([[math.sin(psi), 0.0, -math.cos(psi)]])
        out = ref.trace_rays(o, d, sc)
        b = _b_geom(M, r0, math.sin(psi))
        if b < Q.B_CRIT:
            continue
        u0, u2 = 1.0 / r0, Q.turning_point(M, b)
        target = math.pi / 2
        if Q.psi(M, b, u0) >= target:  # crossing before the turning point
            f = lambda u: Q.phi_at_u(M, b, r0, u, False) - target
            u_hit = brentq(f, u0, u2, xtol=1e-16, rtol=1e-15)
        else:
            f = lambda u: Q.phi_at_u(M, b, r0, u, True) - target
            u_hit = brentq(f, 1.0 / R, u2, xtol=1e-16, rtol=1e-15)
        r_hit = 1.0 / u_hit
        assert out.cls[0] == (ref.DISK if rin <= r_hit <= rout else ref.SKY)
        assert abs(out.r_hit[0] - r_hit) < 1e-8 * r_hit, (psi_deg, out.r_hit[0], r_hit)
        assert abs(out.phi_end[0] - target) < 1e-15


# --------------------------------------------------------------------------
# Images: shadow, symmetry, scale
# --------------------------------------------------------------------------
def test_shadow_pixel_count_cfg1(ref):
    """64x64, r = 30 M, i = 90 deg, FOV 60 deg, no disk: the captured pixels
    are exactly those inside the shadow cone sin^2(alpha) < u0^2 /
    (1/(27 M^2) + 2 M u0^3) (alpha from the forward axis, closed form)."""
    cam = ref.camera(30.0, 90.0, 0.0, 60.0, 64, 64)
    _, out = ref.render(cam, ref.scene(1.0))
    o, d = ref.camera_rays(cam)
    fwd = -o / np.linalg.norm(o, axis=1)[:, None]
    cosa = np.sum(d * fwd, 1)
    sin2 = 1.0 - cosa**2
    thr = Q.shadow_sin2(1.0, 30.0)
    expect = (sin2 < thr) & (cosa > 0)
    ok = np.abs(sin2 - thr) > 1e-9
    np.testing.assert_array_equal((out.cls == ref.CAPTURED)[ok], expect[ok])
    assert expect.sum() == 300


def test_mirror_symmetry_cfg1(ref):
    """Camera in the equatorial plane on the x axis: left/right image
    reflection mirrors y, top/bottom mirrors z of every end vector."""
    W = H = 64
    cam = ref.camera(30.0, 90.0, 0.0, 60.0, W, H)
    _, out = ref.render(cam, ref.scene(1.0))
    e = out.exit_dir.reshape(H, W, 3)
    c = out.cls.reshape(H, W)
    lr = e[:, ::-1] * np.array([1, -1, 1])
    tb = e[::-1, :] * np.array([1, 1, -1])
    np.testing.assert_array_equal(c, c[:, ::-1])
    np.testing.assert_array_equal(c, c[::-1, :])
    sky = c == ref.SKY
    assert np.abs(e - lr)[sky].max() < 1e-11
    assert np.abs(e - tb)[sky].max() < 1e-11


def test_mass_scale_invariance(ref):
    """Eq. (1) is invariant under M -> kM, r -> kr: the image of (M=2, r=60,
    R=2000) equals that of (M=1, r=30, R=1000)."""
    cam1 = ref.camera(30.0, 80.0, 10.0, 40.0, 24, 24)
    cam2 = ref.camera(60.0, 80.0, 10.0, 40.0, 24, 24)
    _, a = ref.render(cam1, ref.scene(1.0, disk=(6.0, 20.0)))
    _, b = ref.render(cam2, ref.scene(2.0, disk=(12.0, 40.0)))
    np.testing.assert_array_equal(a.cls, b.cls)
    assert np.abs(a.exit_dir - b.exit_dir).max() < 1e-9
    np.testing.assert_allclose(2.0 * a.r_hit, b.r_hit, rtol=1e-9)


def test_einstein_ring_visible(ref):
    """Qualitative (the paper's renders show a clear Einstein ring): around
    the shadow, lensed sky pixels are strongly deflected; the ring of pixels
    just outside the shadow sees sky behind the camera's hemisphere."""
    cam = ref.camera(30.0, 90.0, 0.0, 60.0, 64, 64)
    _, out = ref.render(cam, ref.scene(1.0))
    o, d = ref.camera_rays(cam)
    e1 = o / np.linalg.norm(o, axis=1)[:, None]
    back = np.sum(out.exit_dir * e1, 1) > 0  # end point on the camera's side
    assert np.any(back & (out.cls == ref.SKY))


# --------------------------------------------------------------------------
# Camera, shading, edge cases
# --------------------------------------------------------------------------
def test_camera_pixel_directions(ref):
    """Pinhole with vertical FOV: for a 2x2 image with FOV 90 deg the top-left
    pixel centre is at (x, y) = (-0.5, 0.5) on the image plane at distance 1;
    the camera at i = 90 deg, a = 0 has forward -x, right +y, up +z."""
    cam = ref.camera(30.0, 90.0, 0.0, 90.0, 2, 2)
    o, d = ref.camera_rays(cam, [0])
    want = np.array([-1.0, -0.5, 0.5]) / math.sqrt(1.5)
    assert np.abs(d[0] - want).max() < 1e-15
    np.testing.assert_allclose(o[0], [30.0, 0, 0], atol=1e-14)
    # odd-sized image: the centre pixel looks straight at the hole
    cam = ref.camera(50.0, 37.0, 123.0, 30.0, 5, 5)
    o, d = ref.camera_rays(cam, [12])
    assert np.abs(d[0] + o[0] / 50.0).max() < 1e-15


def test_shading_closed_forms(ref):
    """Checker parity (floor(theta/10deg) + floor(varphi/10deg)) mod 2, disk
    emissivity (r/r_in)^-3 times the disk colour, black otherwise."""
    sc = ref.scene(1.0, disk=(6.0, 20.0))
    np.testing.assert_allclose(ref.shade(sc, ref.SKY, [1.0, 0.0, 0.0], 0.0), [0.1, 0.1, 0.1, 1.0])
    th, ph = math.radians(45.0), math.radians(5.0)
    s = [math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)]
    np.testing.assert_allclose(ref.shade(sc, ref.SKY, s, 0.0), [1, 1, 1, 1])
    th, ph = math.radians(15.0), math.radians(-5.0)  # varphi = 355 deg -> cell 35
    s = [math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)]
    np.testing.assert_allclose(ref.shade(sc, ref.SKY, s, 0.0), [1, 1, 1, 1])
    np.testing.assert_allclose(ref.shade(sc, ref.DISK, [1, 0, 0], 12.0), [0.125, 0.075, 0.025, 1.0],
                               rtol=1e-7)
    for c in (ref.CAPTURED, ref.UNRESOLVED, ref.INVALID):
        np.testing.assert_array_equal(ref.shade(sc, c, [1, 0, 0], 0.0), [0, 0, 0, 1])


def test_degenerate_rays(ref):
    """Radial rays, invalid origins and non-finite input (readings: inward
    radial -> captured, outward -> sky along the radial; origin inside the
    photon sphere or outside the sky -> invalid)."""
    sc = ref.scene(1.0)
    o = np.array([[50.0, 0, 0], [50.0, 0, 0], [2.9, 0, 0], [2000.0, 0, 0], [np.nan, 0, 0], [50.0, 0, 0]])
    d = np.array([[-1.0, 0, 0], [1.0, 0, 0], [0, 1.0, 0], [0, 1.0, 0], [0, 1.0, 0], [0, 0, 0]])
    out = ref.trace_rays(o, d, sc)
    assert list(out.cls) == [ref.CAPTURED, ref.SKY, ref.INVALID, ref.INVALID, ref.INVALID, ref.INVALID]
    np.testing.assert_allclose(out.exit_dir[1], [1, 0, 0])
    # flat space: an inward radial ray goes straight through the centre
    out = ref.trace_rays(o[:1], d[:1], ref.scene(0.0))
    assert out.cls[0] == ref.SKY
    np.testing.assert_allclose(out.exit_dir[0], [-1, 0, 0])


def test_caps_give_unresolved(ref):
    """A ray next to the critical impact parameter winds around the photon
    sphere; the sweep cap turns it into UNRESOLVED, as does the step cap."""
    M, r0 = 1.0, 30.0
    b = Q.B_CRIT * (1 + 1e-9)
    sin_psi = (1.0 / r0) / math.sqrt(1.0 / b**2 + 2 * M / r0**3)
    o, d = _plane_rays([r0], [math.pi - math.asin(sin_psi)])
    out = ref.trace_rays(o, d, ref.scene(M), ref.options(max_phi=2 * math.pi))
    assert out.cls[0] == ref.UNRESOLVED
    out = ref.trace_rays(o, d, ref.scene(M), ref.options(max_steps=5))
    assert out.cls[0] == ref.UNRESOLVED
    assert out.n_acc[0] + out.n_rej[0] == 5


# -- equirectangular sky image: bilinear filtering --------------------------

def _tex(W=16, H=8, seed=0):
    return np.random.default_rng(seed).uniform(0, 1, (H, W, 4)).astype(np.float32)


def test_sky_texture_texel_centres(ref):
    """At a texel centre the sample is that texel."""
    t = _tex()
    H, W = t.shape[:2]
    sc = ref.scene(1.0, sky_tex=t)
    for j, i in [(0, 0), (3, 7), (7, 15), (5, 2)]:
        got = ref.sky_sample(sc, math.pi * (j + 0.5) / H, 2 * math.pi * (i + 0.5) / W)
        np.testing.assert_allclose(got, t[j, i], atol=1e-12)


def test_sky_texture_reproduces_bilinear_functions(ref):
    """A texture linear in (column, row) is reproduced exactly between texel
    centres (away from the varphi seam and the clamped pole half-rows)."""
    H, W = 8, 16
    jj, ii = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    a = np.array([0.1, 0.2, -0.3, 1.0]); bi = np.array([0.01, -0.02, 0.03, 0.0])
    cj = np.array([0.05, 0.04, -0.01, 0.0]); dij = np.array([0.002, 0.0, 0.001, 0.0])
    t = (a + bi * ii[..., None] + cj * jj[..., None] + dij * (ii * jj)[..., None]).astype(np.float64)
    t32 = t.astype(np.float32)
    sc = ref.scene(1.0, sky_tex=t32)
    rng = np.random.default_rng(1)
    for _ in range(50):
        u = rng.uniform(0.0, W - 1.0)  # continuous texel coordinates, centres at integers
        v = rng.uniform(0.0, H - 1.0)
        want = a + bi * u + cj * v + dij * u * v
        # the texture holds float32 roundings of the exact values: compare with them
        i0, j0 = int(u), int(v)
        fu, fv = u - i0, v - j0
        q = t32.astype(np.float64)  # the stored texels, interpolated in FP64
        want32 = ((1 - fv) * ((1 - fu) * q[j0, i0] + fu * q[j0, i0 + 1])
                  + fv * ((1 - fu) * q[j0 + 1, i0] + fu * q[j0 + 1, i0 + 1]))
        got = ref.sky_sample(sc, math.pi * (v + 0.5) / H, 2 * math.pi * (u + 0.5) / W)
        np.testing.assert_allclose(got, want32, atol=1e-12)
        np.testing.assert_allclose(got, want, atol=1e-6)


def test_sky_texture_wraps_in_varphi_and_clamps_at_the_poles(ref):
    t = _tex(seed=2)
    H, W = t.shape[:2]
    sc = ref.scene(1.0, sky_tex=t)
    # across the seam: between the last column and the first
    fu, j = 0.3, 4
    got = ref.sky_sample(sc, math.pi * (j + 0.5) / H, 2 * math.pi * (W - 0.5 + fu) / W)
    np.testing.assert_allclose(got, (1 - fu) * t[j, W - 1] + fu * t[j, 0], atol=1e-12)
    # just past varphi = 0 from below is the same point as just below 2 pi
    np.testing.assert_allclose(ref.sky_sample(sc, 1.0, 2 * math.pi - 1e-9),
                               ref.sky_sample(sc, 1.0, 0.0), atol=1e-6)
    # within half a row of a pole only that row contributes
    i, fu = 5, 0.25
    got = ref.sky_sample(sc, 0.1 * math.pi / H, 2 * math.pi * (i + 0.5 + fu) / W)
    np.testing.assert_allclose(got, (1 - fu) * t[0, i] + fu * t[0, i + 1], atol=1e-12)
    got = ref.sky_sample(sc, math.pi * (1 - 0.1 / H), 2 * math.pi * (i + 0.5 + fu) / W)
    np.testing.assert_allclose(got, (1 - fu) * t[H - 1, i] + fu * t[H - 1, i + 1], atol=1e-12)


def test_textured_sky_shading_uses_the_exit_direction(ref):
    t = _tex(seed=3)
    sc = ref.scene(1.0, sky_tex=t)
    th, ph = 1.1, 4.0
    s = [math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)]
    np.testing.assert_allclose(ref.shade(sc, ref.SKY, s, 0.0), ref.sky_sample(sc, th, ph), atol=1e-6)
    # disk and captured rays ignore the sky image
    sc_d = ref.scene(1.0, disk=(6.0, 20.0), sky_tex=t)
    np.testing.assert_allclose(ref.shade(sc_d, ref.CAPTURED, s, 0.0), [0, 0, 0, 1])


# -- the paper's fixed-step mode: points ~eps apart, hits on chords ----------

def _paper_errors(ref, M, disk, eps_list):
    cam = ref.camera(30, 80, 0, 60, 32, 24)
    sc = ref.scene(M, r_sky=1000.0, disk=disk)
    _, a = ref.render(cam, sc, ref.options(rtol=1e-13))
    out = []
    for eps in eps_list:
        _, p = ref.render(cam, sc, ref.options(fixed_eps=eps))
        assert np.array_equal(a.cls, p.cls)
        d = a.cls == 2
        s = a.cls == 0
        ang = np.arctan2(np.linalg.norm(np.cross(a.exit_dir[s], p.exit_dir[s]), axis=1),
                         np.sum(a.exit_dir[s] * p.exit_dir[s], 1))
        out.append((np.abs(p.r_hit[d] / a.r_hit[d] - 1.0).max(), ang.max(), p.n_acc.mean()))
    return out


def test_paper_mode_chords_are_second_order_in_curved_space(ref):
    """With M > 0 the disk-hit radius error comes from the chord's sagitta:
    it falls by ~4 when eps halves; the exit direction converges fast (the
    chord is nearly straight far out); points are ~eps apart, so the number
    of steps doubles."""
    e = _paper_errors(ref, 1.0, (6.0, 20.0), [0.5, 0.25, 0.125])
    for k in range(2):
        assert 3.0 < e[k][0] / e[k + 1][0] < 5.5, e
        assert 1.8 < e[k + 1][2] / e[k][2] < 2.2, e
    assert e[2][1] < 1e-10


def test_paper_mode_chords_are_exact_in_flat_space(ref):
    """With M = 0 the ray is a straight line, so its chords are exact: only
    the integration error of the (large) steps remains, and it falls much
    faster than the sagitta's eps^2."""
    e = _paper_errors(ref, 0.0, (2.0, 12.0), [0.5, 0.25, 0.125])
    for k in range(2):
        assert e[k][0] / e[k + 1][0] > 16.0, e
    assert e[2][0] < 1e-7 and e[2][1] < 1e-10
