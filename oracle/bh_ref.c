/*
 * bh_ref.c -- plain CPU FP64 oracle for Schwarzschild black-hole ray tracing.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product path.  It shares no
 * code with the GPU library.  Written to be read against the paper; speed is
 * not a goal.  Build: gcc -O2 -fopenmp -ffp-contract=off (no fast-math).
 *
 * Paper passages followed (arXiv 2507.16165):
 *   Introduction, Eq. (1) and the two paragraphs after it: the photon-orbit
 *     ODE in u = 1/r against phi, one ray cast through each pixel.
 *   Implementation / "Approximating the trajectory of a light ray as a
 *     piecewise function": the ray is computed as discrete points and
 *     intersected with the scene.
 *   Implementation / "Using GSL for ODE approximation" and Fig. 1: initial
 *     point plus successor from the straight-line direction; step size
 *     trades accuracy for work.
 *   Implementation / "Use of OpenMP": parallel loop over scanlines.
 * Readings (sign of Eq. (1), adaptive stepping, exact event location) are
 * explained in bh_ref.h.
 */
#include "bh_ref.h"

#include <math.h>
#include <omp.h>
#include <stddef.h>

#define PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Photon-orbit equation, Eq. (1) read as u'' + u = 3 M u^2 (Binet form).  */
/* First-order system y = (u, w) with w = du/dphi:                           */
/*   u' = w,   w' = 3 M u^2 - u.                                             */
/* ------------------------------------------------------------------------ */
static void orbit_rhs(double M, double u, double w, double* du, double* dw)
{
    *du = w;
    *dw = 3.0 * M * u * u - u;
}

/* First integral of Eq. (1): E = w^2 + u^2 - 2 M u^3 = 1/b^2. */
static double first_integral(double M, double u, double w)
{
    return w * w + u * u - 2.0 * M * u * u * u;
}

/* ------------------------------------------------------------------------ */
/* Dormand-Prince 5(4) tableau (Dormand & Prince 1980; Hairer, Norsett,      */
/* Wanner, Solving ODEs I, Sec. II.5).  The system is autonomous, so the     */
/* nodes c_i are not needed.  b5 = the 5th-order weights (= last row of A),  */
/* e = b5 - b4 (difference to the embedded 4th-order weights).               */
/* ------------------------------------------------------------------------ */
static const double DP_A[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5.0, 0, 0, 0, 0, 0},
    {3.0 / 40.0, 9.0 / 40.0, 0, 0, 0, 0},
    {44.0 / 45.0, -56.0 / 15.0, 32.0 / 9.0, 0, 0, 0},
    {19372.0 / 6561.0, -25360.0 / 2187.0, 64448.0 / 6561.0, -212.0 / 729.0, 0, 0},
    {9017.0 / 3168.0, -355.0 / 33.0, 46732.0 / 5247.0, 49.0 / 176.0, -5103.0 / 18656.0, 0},
    {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0},
};
static const double DP_E[7] = {
    71.0 / 57600.0, 0.0, -71.0 / 16695.0, 71.0 / 1920.0,
    -17253.0 / 339200.0, 22.0 / 525.0, -1.0 / 40.0,
};

/* One step from y with step h.  The seven stage derivatives are evaluated
 * here from scratch (no first-same-as-last reuse: simpler to check; the
 * numbers are identical).  y_out is the 5th-order solution; err is the
 * difference of the 5th- and 4th-order solutions. */
static void dopri5_step(double M, double u, double w, double h,
                        double* u_out, double* w_out, double* eu, double* ew)
{
    double ku[7], kw[7];
    orbit_rhs(M, u, w, &ku[0], &kw[0]);
    for (int s = 1; s < 7; ++s) {
        double su = 0.0, sw = 0.0;
        for (int j = 0; j < s; ++j) {
            su += DP_A[s][j] * ku[j];
            sw += DP_A[s][j] * kw[j];
        }
        orbit_rhs(M, u + h * su, w + h * sw, &ku[s], &kw[s]);
    }
    /* 5th-order solution: the weights equal row 7 of A (stage 7 is y_out). */
    double su = 0.0, sw = 0.0, tu = 0.0, tw = 0.0;
    for (int j = 0; j < 6; ++j) {
        su += DP_A[6][j] * ku[j];
        sw += DP_A[6][j] * kw[j];
    }
    for (int j = 0; j < 7; ++j) {
        tu += DP_E[j] * ku[j];
        tw += DP_E[j] * kw[j];
    }
    *u_out = u + h * su;
    *w_out = w + h * sw;
    *eu = h * tu;
    *ew = h * tw;
}

void bhr_dopri5_step(double M, const double y[2], double h, double y_out[2], double err[2])
{
    dopri5_step(M, y[0], y[1], h, &y_out[0], &y_out[1], &err[0], &err[1]);
}

int bhr_max_threads(void) { return omp_get_max_threads(); }

void bhr_default_options(bhr_options* opt)
{
    opt->rtol = 1e-10;
    opt->atol = 0.0;
    opt->h0 = 1e-2;
    opt->hmax = 1.0;
    opt->max_phi = 8.0 * PI;
    opt->max_steps = 1000000;
    opt->fixed_eps = 0.0;
}

/* ------------------------------------------------------------------------ */
/* Small vector helpers.                                                     */
/* ------------------------------------------------------------------------ */
static double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static double norm3(const double a[3]) { return sqrt(dot3(a, a)); }

/* ------------------------------------------------------------------------ */
/* Camera: one ray through the centre of each pixel (Introduction, the      */
/* 1920x1080 example).  Pinhole looking at the hole, vertical field of view, */
/* row 0 at the top, "up" = -e_theta of the camera position.                 */
/* ------------------------------------------------------------------------ */
int bhr_camera_ray(const bhr_camera* cam, int px, int py, double origin[3], double dir[3])
{
    if (!cam || !origin || !dir) return -1;
    const double inc = cam->incl_deg * PI / 180.0;
    const double az = cam->azim_deg * PI / 180.0;
    const double pos_hat[3] = {sin(inc) * cos(az), sin(inc) * sin(az), cos(inc)};
    const double fwd[3] = {-pos_hat[0], -pos_hat[1], -pos_hat[2]};
    const double up[3] = {-cos(inc) * cos(az), -cos(inc) * sin(az), sin(inc)};
    const double right[3] = {fwd[1] * up[2] - fwd[2] * up[1],
                             fwd[2] * up[0] - fwd[0] * up[2],
                             fwd[0] * up[1] - fwd[1] * up[0]};
    const double t = tan(0.5 * cam->fov_deg * PI / 180.0);
    const double W = (double)cam->width, H = (double)cam->height;
    const double x = (2.0 * (px + 0.5) / W - 1.0) * t * W / H;
    const double y = (1.0 - 2.0 * (py + 0.5) / H) * t;
    double d[3];
    for (int k = 0; k < 3; ++k) {
        origin[k] = cam->r * pos_hat[k];
        d[k] = fwd[k] + x * right[k] + y * up[k];
    }
    const double n = norm3(d);
    for (int k = 0; k < 3; ++k) dir[k] = d[k] / n;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* One ray.                                                                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int cls;
    double b, phi_end, exit_dir[3], r_hit, e_drift;
    int n_acc, n_rej;
} ray_result;

static void set_end(ray_result* res, int cls, double phi, const double e1[3], const double e2[3])
{
    res->cls = cls;
    res->phi_end = phi;
    for (int k = 0; k < 3; ++k) res->exit_dir[k] = cos(phi) * e1[k] + sin(phi) * e2[k];
}

/* Paper mode (Sec. "Approximating the trajectory of a light ray as a
 * piecewise function", Sec. "Using GSL for ODE approximation", Fig.
 * "nextpoint"): the ray is a sequence of points about eps apart.  From the
 * point at (u, w, phi) the azimuth advances by the angle that a straight
 * segment of length eps along the ray's current direction subtends at the
 * hole -- the direction has radial and tangential components proportional
 * to (-w, u), so dphi = atan2(eps u^2, sqrt(u^2 + w^2) - eps u w) -- with one
 * Dormand-Prince step over dphi and no error control.  The scene is intersected with the straight
 * chord between consecutive points, in order: the disk plane z = 0 (inside
 * r_in <= |Q| <= r_out), the horizon (the new point inside r = 2M), the sky
 * sphere (|Q| = r_sky on the chord).  In-plane coordinates: a point at
 * (r, phi) is r (cos phi e1 + sin phi e2); its height is r zeta(phi) with
 * zeta(phi) = e1z cos(phi) + e2z sin(phi). */
static void trace_paper(const bhr_scene* sc, const bhr_options* opt, const double e1[3],
                        const double e2[3], double u0, double w0, int disk_on, ray_result* res)
{
    const double M = sc->M, R = sc->r_sky, u_sky = 1.0 / R, eps = opt->fixed_eps;
    double u = u0, w = w0, phi = 0.0;
    double x = 1.0 / u0, y = 0.0;        /* current point, in-plane coordinates */
    double z = x * e1[2];                /* its height */
    for (;;) {
        if (res->n_acc >= opt->max_steps || phi > opt->max_phi) {
            set_end(res, BHR_UNRESOLVED, phi, e1, e2);
            return;
        }
        const double h = atan2(eps * u * u, sqrt(u * u + w * w) - eps * u * w);
        double un, wn, eu, ew;
        dopri5_step(M, u, w, h, &un, &wn, &eu, &ew);
        ++res->n_acc;
        const double phin = phi + h;
        const double rn = un > 0.0 ? 1.0 / un : 1e300;
        const double xn = rn * cos(phin), yn = rn * sin(phin);
        const double zn = rn * (e1[2] * cos(phin) + e2[2] * sin(phin));
        if (disk_on && ((z < 0.0 && zn >= 0.0) || (z > 0.0 && zn <= 0.0))) {
            const double t = z / (z - zn);
            const double qx = x + t * (xn - x), qy = y + t * (yn - y);
            const double rq = sqrt(qx * qx + qy * qy);
            if (rq >= sc->disk_rin && rq <= sc->disk_rout) {
                res->r_hit = rq;
                set_end(res, BHR_DISK, phi + atan2(x * qy - y * qx, x * qx + y * qy), e1, e2);
                return;
            }
        }
        if (M > 0.0 && 2.0 * M * un >= 1.0) {
            set_end(res, BHR_CAPTURED, phin, e1, e2);
            return;
        }
        if (un <= u_sky) {
            /* |P + t (Pn - P)| = R with |P| < R: the root t in (0, 1] */
            const double dx = xn - x, dy = yn - y;
            const double qa = dx * dx + dy * dy, qb = 2.0 * (x * dx + y * dy);
            const double qc = x * x + y * y - R * R;
            const double t = (-qb + sqrt(qb * qb - 4.0 * qa * qc)) / (2.0 * qa);
            const double qx = x + t * dx, qy = y + t * dy;
            set_end(res, BHR_SKY, phi + atan2(x * qy - y * qx, x * qx + y * qy), e1, e2);
            return;
        }
        u = un;
        w = wn;
        phi = phin;
        x = xn;
        y = yn;
        z = zn;
    }
}

static void trace_one(const double o[3], const double d_in[3], const bhr_scene* sc,
                      const bhr_options* opt, ray_result* res)
{
    const double M = sc->M;
    const double R = sc->r_sky;
    res->cls = BHR_INVALID;
    res->b = 0.0;
    res->phi_end = 0.0;
    res->exit_dir[0] = res->exit_dir[1] = res->exit_dir[2] = 0.0;
    res->r_hit = 0.0;
    res->e_drift = 0.0;
    res->n_acc = res->n_rej = 0;

    for (int k = 0; k < 3; ++k)
        if (!isfinite(o[k]) || !isfinite(d_in[k])) return;
    const double r0 = norm3(o);
    const double dn = norm3(d_in);
    /* The ray must start outside the photon sphere and inside the sky. */
    if (!(r0 > 3.0 * M) || !(r0 < R) || !(dn > 0.0)) return;

    /* Orbital plane (the hole bends light the same way from every
     * direction, so the ray stays in the plane through the centre spanned by
     * its origin and direction). */
    double e1[3], d[3], v[3], e2[3];
    for (int k = 0; k < 3; ++k) {
        e1[k] = o[k] / r0;
        d[k] = d_in[k] / dn;
    }
    const double c = dot3(d, e1); /* cos of the angle to the outward radial */
    for (int k = 0; k < 3; ++k) v[k] = d[k] - c * e1[k];
    const double s = norm3(v); /* sin of that angle */

    if (s <= 1e-15) {
        /* Radial ray: it never leaves the radial line. */
        double neg[3] = {-e1[0], -e1[1], -e1[2]};
        if (c < 0.0 && M > 0.0) {
            res->cls = BHR_CAPTURED;
            for (int k = 0; k < 3; ++k) res->exit_dir[k] = e1[k];
        } else if (c < 0.0) {
            res->cls = BHR_SKY; /* flat space: straight through the centre */
            res->phi_end = PI;
            for (int k = 0; k < 3; ++k) res->exit_dir[k] = neg[k];
        } else {
            res->cls = BHR_SKY;
            for (int k = 0; k < 3; ++k) res->exit_dir[k] = e1[k];
        }
        return;
    }
    for (int k = 0; k < 3; ++k) e2[k] = v[k] / s;

    /* Initial conditions from the straight-line direction: the successor
     * point in its exact-derivative limit. */
    const double u0 = 1.0 / r0;
    const double w0 = -u0 * c / s;
    const double E0 = first_integral(M, u0, w0);
    res->b = 1.0 / sqrt(E0);

    /* Crossings of the disk plane z = 0: the ray's height is proportional to
     * e1z cos(phi) + e2z sin(phi), so crossings sit at phi_1 + k*pi, with
     * phi_1 the first root in (0, pi]. */
    int disk_on = 0;
    double phi_k = 0.0;
    if (sc->has_disk) {
        const double a = e1[2], bz = e2[2];
        if (hypot(a, bz) > 1e-15) {
            disk_on = 1;
            if (a == 0.0) {
                phi_k = PI;
            } else if (bz == 0.0) {
                phi_k = 0.5 * PI;
            } else {
                phi_k = atan(-a / bz);        /* in (-pi/2, pi/2) */
                if (phi_k <= 0.0) phi_k += PI; /* first root in (0, pi] */
            }
        }
    }

    if (opt->fixed_eps > 0.0) {
        trace_paper(sc, opt, e1, e2, u0, w0, sc->has_disk && hypot(e1[2], e2[2]) > 1e-15, res);
        return;
    }

    const double u_sky = 1.0 / R;
    const double rtol = opt->rtol;
    const double atol = opt->atol > 0.0 ? opt->atol : rtol * u_sky;

    double u = u0, w = w0, phi = 0.0, h = opt->h0;
    int rejected_last = 0;
    int attempts = 0;

    for (;;) {
        if (attempts >= opt->max_steps) {
            set_end(res, BHR_UNRESOLVED, phi, e1, e2);
            return;
        }
        ++attempts;

        /* Trial step; a step that would pass the next disk-plane crossing
         * is shortened to land on it exactly. */
        double ht = h;
        int land = 0;
        if (disk_on && phi + ht >= phi_k) {
            ht = phi_k - phi;
            land = 1;
        }
        double un, wn, eu, ew;
        dopri5_step(M, u, w, ht, &un, &wn, &eu, &ew);
        const double sc_u = atol + rtol * fmax(fabs(u), fabs(un));
        const double sc_w = atol + rtol * fmax(fabs(w), fabs(wn));
        const double err = fmax(fabs(eu) / sc_u, fabs(ew) / sc_w);

        if (!(err <= 1.0)) {
            /* Rejected: shrink and retry from the same state. */
            ++res->n_rej;
            double fac = isfinite(err) ? 0.9 * pow(err, -0.2) : 0.2;
            if (fac < 0.2) fac = 0.2;
            h = ht * fac;
            rejected_last = 1;
            continue;
        }

        /* Accepted. */
        ++res->n_acc;
        const double u_prev = u, w_prev = w, phi_prev = phi;
        u = un;
        w = wn;
        phi = land ? phi_k : phi + ht;
        {
            const double drift = fabs(first_integral(M, u, w) / E0 - 1.0);
            if (drift > res->e_drift) res->e_drift = drift;
        }
        /* Next step size.  A landing step leaves the previous proposal in
         * place; otherwise the elementary controller with safety 0.9 and
         * factor limits [0.2, 5], and no growth right after a rejection. */
        if (!land) {
            double fac = err > 0.0 ? 0.9 * pow(err, -0.2) : 5.0;
            if (fac > 5.0) fac = 5.0;
            if (fac < 0.2) fac = 0.2;
            if (rejected_last && fac > 1.0) fac = 1.0;
            h = ht * fac;
        }
        if (h > opt->hmax) h = opt->hmax;
        rejected_last = 0;

        /* Events, in order: disk crossing, horizon, sky sphere, caps. */
        if (land) {
            const double r = 1.0 / u;
            if (r >= sc->disk_rin && r <= sc->disk_rout) {
                res->r_hit = r;
                set_end(res, BHR_DISK, phi, e1, e2);
                return;
            }
            phi_k += PI;
        }
        if (M > 0.0 && 2.0 * M * u >= 1.0) {
            set_end(res, BHR_CAPTURED, phi, e1, e2);
            return;
        }
        if (u <= u_sky && w < 0.0) {
            /* Locate the sky crossing inside the last step by Newton's
             * method on the step length, redoing the step from the last
             * accepted state: h <- h - (u(h) - u_sky) / u'(h). */
            double hh = ht, uu = u, ww = w;
            for (int it = 0; it < 4; ++it) {
                const double dh = (uu - u_sky) / ww;
                hh -= dh;
                if (fabs(dh) < 1e-15 || it == 3) break;
                double e_u, e_w;
                dopri5_step(M, u_prev, w_prev, hh, &uu, &ww, &e_u, &e_w);
            }
            set_end(res, BHR_SKY, phi_prev + hh, e1, e2);
            return;
        }
        if (phi > opt->max_phi) {
            set_end(res, BHR_UNRESOLVED, phi, e1, e2);
            return;
        }
    }
}

static void store(bhr_out* out, int64_t i, const ray_result* r)
{
    if (!out) return;
    if (out->cls) out->cls[i] = (uint8_t)r->cls;
    if (out->b) out->b[i] = r->b;
    if (out->phi_end) out->phi_end[i] = r->phi_end;
    if (out->exit_dir)
        for (int k = 0; k < 3; ++k) out->exit_dir[3 * i + k] = r->exit_dir[k];
    if (out->r_hit) out->r_hit[i] = r->r_hit;
    if (out->n_acc) out->n_acc[i] = r->n_acc;
    if (out->n_rej) out->n_rej[i] = r->n_rej;
    if (out->e_drift) out->e_drift[i] = r->e_drift;
}

static int scene_ok(const bhr_scene* sc)
{
    if (!sc) return 0;
    if (!(sc->M >= 0.0) || !(sc->r_sky > 0.0) || !(sc->checker_deg > 0.0)) return 0;
    if (sc->has_disk && !(sc->disk_rin > 0.0 && sc->disk_rin < sc->disk_rout)) return 0;
    if (sc->sky_tex && !(sc->tex_w >= 1 && sc->tex_h >= 1)) return 0;
    return 1;
}

int bhr_trace_rays(const double* origin, const double* dir, int64_t n,
                   const bhr_scene* sc, const bhr_options* opt, bhr_out* out)
{
    if (!origin || !dir || n < 0 || !scene_ok(sc) || !opt) return -1;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        ray_result r;
        trace_one(origin + 3 * i, dir + 3 * i, sc, opt, &r);
        store(out, i, &r);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Shading: sky (procedural checker or an equirectangular image), disk       */
/* emissivity, black otherwise.                                              */
/* ------------------------------------------------------------------------ */
void bhr_sky_sample(const bhr_scene* sc, double theta, double varphi, double rgba[4])
{
    const int W = sc->tex_w, H = sc->tex_h;
    /* continuous texel coordinates: centres at integers */
    const double u = varphi / (2.0 * PI) * W - 0.5;
    const double v = theta / PI * H - 0.5;
    const double i0f = floor(u), j0f = floor(v);
    const double fu = u - i0f, fv = v - j0f;
    long i0 = (long)i0f % W;
    if (i0 < 0) i0 += W;
    const long i1 = (i0 + 1) % W;
    long j0 = (long)j0f, j1 = j0 + 1;
    if (j0 < 0) j0 = 0;
    if (j0 > H - 1) j0 = H - 1;
    if (j1 < 0) j1 = 0;
    if (j1 > H - 1) j1 = H - 1;
    for (int c = 0; c < 4; ++c) {
        const double t00 = sc->sky_tex[((size_t)j0 * W + i0) * 4 + c];
        const double t10 = sc->sky_tex[((size_t)j0 * W + i1) * 4 + c];
        const double t01 = sc->sky_tex[((size_t)j1 * W + i0) * 4 + c];
        const double t11 = sc->sky_tex[((size_t)j1 * W + i1) * 4 + c];
        rgba[c] = (1.0 - fv) * ((1.0 - fu) * t00 + fu * t10) + fv * ((1.0 - fu) * t01 + fu * t11);
    }
}

void bhr_shade(const bhr_scene* sc, int cls, const double s[3], double r_hit, float rgba[4])
{
    rgba[0] = rgba[1] = rgba[2] = 0.0f;
    rgba[3] = 1.0f;
    if (cls == BHR_SKY && sc->sky_tex) {
        const double theta = atan2(hypot(s[0], s[1]), s[2]);
        double varphi = atan2(s[1], s[0]);
        if (varphi < 0.0) varphi += 2.0 * PI;
        double t[4];
        bhr_sky_sample(sc, theta, varphi, t);
        for (int c = 0; c < 4; ++c) rgba[c] = (float)t[c];
    } else if (cls == BHR_SKY) {
        const double theta = atan2(hypot(s[0], s[1]), s[2]);
        double varphi = atan2(s[1], s[0]);
        if (varphi < 0.0) varphi += 2.0 * PI;
        const double cell = sc->checker_deg * PI / 180.0;
        const long parity = ((long)floor(theta / cell) + (long)floor(varphi / cell)) & 1L;
        const float g = parity ? 0.1f : 1.0f;
        rgba[0] = rgba[1] = rgba[2] = g;
    } else if (cls == BHR_DISK) {
        const double I = pow(r_hit / sc->disk_rin, sc->disk_power);
        rgba[0] = (float)(1.0 * I);
        rgba[1] = (float)(0.6 * I);
        rgba[2] = (float)(0.2 * I);
    }
}

/* One image row: camera ray, trace and shade of every pixel in it. */
static void render_row(const bhr_camera* cam, const bhr_scene* sc, const bhr_options* opt, int py,
                       float* rgba, bhr_out* out)
{
    const int W = cam->width;
    for (int px = 0; px < W; ++px) {
        double o[3], d[3];
        bhr_camera_ray(cam, px, py, o, d);
        ray_result r;
        trace_one(o, d, sc, opt, &r);
        const int64_t i = (int64_t)py * W + px;
        store(out, i, &r);
        if (rgba) bhr_shade(sc, r.cls, r.exit_dir, r.r_hit, rgba + 4 * i);
    }
}

int bhr_render_rows(const bhr_camera* cam, const bhr_scene* sc, const bhr_options* opt,
                    int row0, int row1, float* rgba, bhr_out* out)
{
    if (!cam || !scene_ok(sc) || !opt) return -1;
    if (cam->width < 1 || cam->height < 1) return -1;
    if (row0 < 0 || row1 > cam->height || row0 > row1) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int py = row0; py < row1; ++py) render_row(cam, sc, opt, py, rgba, out);
    return 0;
}

int bhr_render_row_list(const bhr_camera* cam, const bhr_scene* sc, const bhr_options* opt,
                        const int* rows, int nrows, float* rgba, bhr_out* out)
{
    if (!cam || !scene_ok(sc) || !opt || (!rows && nrows > 0) || nrows < 0) return -1;
    if (cam->width < 1 || cam->height < 1) return -1;
    for (int k = 0; k < nrows; ++k)
        if (rows[k] < 0 || rows[k] >= cam->height) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k < nrows; ++k) render_row(cam, sc, opt, rows[k], rgba, out);
    return 0;
}

void bhr_set_threads(int n)
{
    if (n > 0) omp_set_num_threads(n);
}

/* ------------------------------------------------------------------------ */
/* Flat-space sweep of the straight ray with the same initial direction.     */
/* ------------------------------------------------------------------------ */
double bhr_dphi_flat(double M, double b, double r0, double r_sky)
{
    const double u0 = 1.0 / r0;
    const double sin_psi = u0 / sqrt(1.0 / (b * b) + 2.0 * M * u0 * u0 * u0);
    const double psi = asin(sin_psi);
    return PI - psi - asin(r0 * sin_psi / r_sky);
}
