"""Pin of the oracle's step-size controller against an independent
Dormand-Prince implementation: scipy's ``RK45``.

The oracle's controller (the adaptive reading of the paper's GSL stepping,
Sec. "Using GSL for ODE approximation") is the elementary one: accept iff the
error ratio err = max_i |e_i| / (atol + rtol max(|y_i|, |y_new,i|)) is at most
1, then scale the step by 0.9 err^(-1/5) clamped to [0.2, 5], with no growth
right after a rejection.  scipy's RK45 (Dormand & Prince 1980, the same
tableau) has the same controller up to two constants: its error norm is the
RMS over components and its growth limit is 10.  With those two set to the
oracle's values (max norm, growth limit 5) scipy must take exactly the
oracle's accepted and rejected steps on the same rays, except where an
error ratio sits on 1 to within rounding.

A dropped safety factor, another exponent, another clamp, growth after a
rejection, an error scale from |y| alone, or a wrong entry of the error
weights changes the step sequence of nearly every ray and fails this test.

Events are checked on the accepted step's end point, as the oracle does
(disk landing, horizon, sky sphere).  Steps that would pass a disk-plane
crossing are shortened to land on it (scipy's ``t_bound``), and a landing
step leaves the step proposal where it was: the oracle's reading of the
landing rule, restated in ``_scipy_counts`` below.
"""
import math

import numpy as np
import pytest
import scipy.integrate._ivp.rk as rk
from scipy.integrate import RK45


def _maxnorm(x):
    return float(np.max(np.abs(x)))


def _initial_conditions(o, d):
    """u0, w0 and the first disk-plane crossing angle of a ray from origin o
    with direction d (plane through the centre spanned by o and d, phi = 0 at
    the origin, increasing along the ray)."""
    r0 = np.linalg.norm(o)
    e1 = o / r0
    d = d / np.linalg.norm(d)
    c = float(d @ e1)
    v = d - c * e1
    s = np.linalg.norm(v)
    e2 = v / s
    u0 = 1.0 / r0
    w0 = -u0 * c / s
    a, bz = e1[2], e2[2]
    if math.hypot(a, bz) <= 1e-15:
        phi1 = math.inf
    else:
        # root of a cos(phi) + bz sin(phi) = 0 in (0, pi]
        phi1 = math.atan2(-a, bz) % math.pi
        if phi1 == 0.0:
            phi1 = math.pi
    return u0, w0, phi1


def _scipy_counts(M, u0, w0, phi1, disk, r_sky, rtol, h0=1e-2, hmax=1.0, max_phi=8 * math.pi,
                  landing_keeps_proposal=True):
    """(accepted, rejected) steps of scipy's RK45 (max norm, growth limit 5)
    on u' = w, w' = 3 M u^2 - u from (u0, w0) until the first event.
    landing_keeps_proposal=False: a landing step sets the next proposal from
    its own shortened length, as any other step (a negative control)."""
    u_sky = 1.0 / r_sky
    atol = rtol * u_sky
    fun = lambda t, y: np.array([y[1], 3.0 * M * y[0] * y[0] - y[0]])
    phik = phi1 if disk is not None else math.inf
    s = RK45(fun, 0.0, np.array([u0, w0]), t_bound=phik, rtol=rtol, atol=atol,
             max_step=hmax, first_step=h0)
    acc = 0
    while True:
        if s.status == "finished":   # landed on a crossing: aim at the next one
            s.status = "running"
        s.t_bound = phik
        h_prop = min(s.h_abs, hmax)
        s.step()
        assert s.status != "failed"
        acc += 1
        landed = s.t == phik
        if landed and landing_keeps_proposal:
            s.h_abs = h_prop         # a landing step keeps the proposal
        u, w = s.y
        if landed:
            r = 1.0 / u
            if disk[0] <= r <= disk[1]:
                break
            phik += math.pi
        if M > 0.0 and 2.0 * M * u >= 1.0:
            break
        if u <= u_sky and w < 0.0:
            break
        if s.t > max_phi:
            break
    attempts = (s.nfev - 1) // 6    # one derivative at the start, six per attempt
    return acc, attempts - acc


def _camera_case(ref, disk, W=20, H=14):
    cam = ref.camera(25.0, 70.0, 30.0, 60.0, W, H)
    sc = ref.scene(1.0, disk=disk)
    o, d = ref.camera_rays(cam)
    out = ref.trace_rays(o, d, sc)
    return o, d, out, sc


@pytest.mark.parametrize("disk", [None, (6.0, 20.0), (60.0, 80.0)])
def test_step_counts_equal_scipy_rk45(ref, monkeypatch, disk):
    """Every integrated ray of a small frame (no disk / disk 6-20 M / a ring
    at 60-80 M that most rays cross without hitting, so that steps after a
    landing matter): the oracle's accepted and rejected step counts equal
    scipy's, on at least 98% of the rays and in total within 0.5%."""
    monkeypatch.setattr(rk, "norm", _maxnorm)
    monkeypatch.setattr(rk, "MAX_FACTOR", 5.0)
    o, d, out, sc = _camera_case(ref, disk)
    same, n, tot_o, tot_s = 0, 0, 0, 0
    for k in range(o.shape[0]):
        if out.n_acc[k] == 0:
            continue  # radial or invalid: no integration
        u0, w0, phi1 = _initial_conditions(o[k], d[k])
        acc, rej = _scipy_counts(1.0, u0, w0, phi1, disk, sc.r_sky, 1e-10)
        n += 1
        same += (acc == out.n_acc[k]) and (rej == out.n_rej[k])
        tot_o += int(out.n_acc[k]) + int(out.n_rej[k])
        tot_s += acc + rej
    assert n > 200
    assert same >= 0.98 * n, (same, n)
    assert abs(tot_o / tot_s - 1.0) < 5e-3, (tot_o, tot_s)


def test_rejections_occur_and_stay_bounded(ref, monkeypatch):
    """The controller is exercised: at rtol 1e-6 (the FP32 path's tolerance,
    where steps are long) rejections happen, scipy agrees on them ray by ray,
    and they stay a minority of the attempts on smooth rays."""
    monkeypatch.setattr(rk, "norm", _maxnorm)
    monkeypatch.setattr(rk, "MAX_FACTOR", 5.0)
    cam = ref.camera(40.0, 60.0, 10.0, 50.0, 16, 10)
    sc = ref.scene(1.0)
    o, d = ref.camera_rays(cam)
    out = ref.trace_rays(o, d, sc, ref.options(rtol=1e-6))
    same = n = 0
    for k in range(o.shape[0]):
        if out.n_acc[k] == 0:
            continue
        u0, w0, phi1 = _initial_conditions(o[k], d[k])
        acc, rej = _scipy_counts(1.0, u0, w0, phi1, None, sc.r_sky, 1e-6)
        n += 1
        same += (acc == out.n_acc[k]) and (rej == out.n_rej[k])
    assert same >= 0.98 * n, (same, n)
    rej_frac = out.n_rej.sum() / max(1, (out.n_acc + out.n_rej).sum())
    assert 0.01 < rej_frac < 0.4, rej_frac


def test_scipy_pin_detects_a_changed_controller(ref, monkeypatch):
    """Negative control: the same comparison with scipy's safety factor
    changed to 0.8 (a plausible slip) disagrees on most rays, so the
    equality above is not vacuous."""
    monkeypatch.setattr(rk, "norm", _maxnorm)
    monkeypatch.setattr(rk, "MAX_FACTOR", 5.0)
    monkeypatch.setattr(rk, "SAFETY", 0.8)
    o, d, out, sc = _camera_case(ref, None, 10, 7)
    same = n = 0
    for k in range(o.shape[0]):
        if out.n_acc[k] == 0:
            continue
        u0, w0, phi1 = _initial_conditions(o[k], d[k])
        acc, rej = _scipy_counts(1.0, u0, w0, phi1, None, sc.r_sky, 1e-10)
        n += 1
        same += (acc == out.n_acc[k]) and (rej == out.n_rej[k])
    assert same < 0.5 * n, (same, n)


def test_scipy_pin_detects_a_changed_landing_rule(ref, monkeypatch):
    """Negative control for the landing reading: if a landing step set the
    next proposal from its own shortened length, the step counts of rays
    that cross the disk plane without hitting (ring at 60-80 M) would differ
    from the oracle's on more than a tenth of the rays."""
    monkeypatch.setattr(rk, "norm", _maxnorm)
    monkeypatch.setattr(rk, "MAX_FACTOR", 5.0)
    disk = (60.0, 80.0)
    o, d, out, sc = _camera_case(ref, disk)
    same = n = 0
    for k in range(o.shape[0]):
        if out.n_acc[k] == 0:
            continue
        u0, w0, phi1 = _initial_conditions(o[k], d[k])
        acc, rej = _scipy_counts(1.0, u0, w0, phi1, disk, sc.r_sky, 1e-10,
                                 landing_keeps_proposal=False)
        n += 1
        same += (acc == out.n_acc[k]) and (rej == out.n_rej[k])
    assert same < 0.9 * n, (same, n)
