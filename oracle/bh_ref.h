/*
 * bh_ref.h -- plain CPU FP64 oracle for Schwarzschild black-hole ray tracing.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the correctness reference for
 * the GPU path and is loaded only by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark.  The product path never calls it.  It
 * shares no code, header, table or constant with the GPU library.
 *
 * What it computes (paper: Section "Introduction", Eq. (1) and the text
 * around it; Section "Implementation", subsections on the piecewise ray and
 * on GSL ODE approximation; Fig. 1 caption):
 *   - one ray per pixel of a pinhole camera that looks at the hole;
 *   - each ray is reduced to its orbital plane through the hole's centre
 *     (the Schwarzschild hole bends light independently of the approach
 *     direction, so the orbit stays in one plane);
 *   - the photon-orbit equation in u = 1/r against the azimuth phi is
 *     integrated from the straight-line initial direction until the ray
 *     escapes to the sky sphere, falls through the horizon or hits a thin
 *     equatorial disk;
 *   - the endpoint is mapped back to 3D and shaded.
 *
 * Readings taken where the paper is silent or garbled:
 *   - Eq. (1) is printed with a minus sign on u; the Binet equation of the
 *     cited textbook, and every limit the method must reproduce (straight
 *     lines at M = 0, the critical impact parameter 3*sqrt(3)*M, weak-field
 *     deflection 4M/b), use u'' + u = 3 M u^2 (G = c = 1).
 *   - The paper's fixed-step GSL stepping with chord intersection is replaced
 *     by adaptive Dormand-Prince 5(4) with exact event location.
 *   - The "successor point from the linear direction" is taken in its
 *     exact-derivative limit: w0 = du/dphi = -u0 * cot(alpha).
 *
 * Units: G = c = 1; M, r, b share one length unit.  All arithmetic is IEEE
 * binary64, round to nearest, built without contraction or fast-math.
 *
 * Threading: the batch entry points parallelise with OpenMP over image rows
 * (render) or over rays (trace), mirroring the paper's shared-memory loop over
 * scanlines.  Every ray is computed by one thread with no shared state, so
 * results do not depend on the thread count.
 *
 * Return value of every entry point: 0 on success, -1 on a bad argument.
 */
#ifndef BH_REF_H
#define BH_REF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Per-ray classes. */
enum { BHR_SKY = 0, BHR_CAPTURED = 1, BHR_DISK = 2, BHR_UNRESOLVED = 3, BHR_INVALID = 4 };

typedef struct {
    double M;            /* hole mass (>= 0); M = 0 gives flat space          */
    double r_sky;        /* radius of the sky sphere (absolute units)         */
    int    has_disk;     /* 1: thin opaque disk in the plane z = 0            */
    double disk_rin;     /* inner disk radius                                 */
    double disk_rout;    /* outer disk radius                                 */
    double disk_power;   /* emissivity I = (r / r_in)^power (power = -3)      */
    double checker_deg;  /* checker cell size on the sky sphere, degrees      */
    const float* sky_tex;/* optional equirectangular sky image (host, RGBA floats,
                            tex_h rows from theta = 0 to pi, tex_w columns from
                            varphi = 0 to 2 pi); NULL: the checker             */
    int    tex_w, tex_h;
} bhr_scene;

typedef struct {
    double r;            /* camera distance from the hole                     */
    double incl_deg;     /* polar angle of the camera from +z                 */
    double azim_deg;     /* azimuth of the camera about +z                    */
    double fov_deg;      /* vertical field of view                            */
    int    width, height;
} bhr_camera;

typedef struct {
    double rtol;         /* relative tolerance of the error test              */
    double atol;         /* absolute tolerance; <= 0 means rtol / r_sky       */
    double h0;           /* first trial step in phi (radians)                 */
    double hmax;         /* largest step in phi                               */
    double max_phi;      /* sweep cap -> UNRESOLVED                           */
    int    max_steps;    /* cap on step attempts -> UNRESOLVED                */
    double fixed_eps;    /* > 0: the paper's fixed-step mode -- points about
                            fixed_eps apart (absolute length), one Dormand-Prince
                            step each, scene hits on the chords between them;
                            0: adaptive steps with events on the curve          */
} bhr_options;

/* Structure-of-arrays output, length n; any pointer may be NULL. */
typedef struct {
    uint8_t* cls;        /* class, BHR_*                                      */
    double*  b;          /* impact parameter from the first integral          */
    double*  phi_end;    /* azimuth at the end event                          */
    double*  exit_dir;   /* n*3: unit vector of the end point                 */
    double*  r_hit;      /* disk hit radius (DISK), else 0                    */
    int32_t* n_acc;      /* accepted steps                                    */
    int32_t* n_rej;      /* rejected steps                                    */
    double*  e_drift;    /* max |E/E0 - 1| of the first integral over the ray */
} bhr_out;

/* Number of OpenMP threads the batch entry points use. */
int bhr_max_threads(void);

/* Default options: rtol 1e-10, atol = rtol/r_sky, h0 1e-2, hmax 1,
 * max_phi 8*pi, max_steps 1e6. */
void bhr_default_options(bhr_options* opt);

/* Unit ray direction and origin through the centre of pixel (px, py). */
int bhr_camera_ray(const bhr_camera* cam, int px, int py, double origin[3], double dir[3]);

/* Trace n rays given world-space origins and directions (host arrays, n*3). */
int bhr_trace_rays(const double* origin, const double* dir, int64_t n,
                   const bhr_scene* sc, const bhr_options* opt, bhr_out* out);

/* Render image rows [row0, row1).  rgba is the full W*H*4 float image (rows
 * outside the range are left untouched); out arrays are indexed by pixel
 * y*W + x over the full image as well.  Either may be NULL. */
int bhr_render_rows(const bhr_camera* cam, const bhr_scene* sc, const bhr_options* opt,
                    int row0, int row1, float* rgba, bhr_out* out);

/* Render the listed image rows (each 0 <= rows[k] < height; OpenMP over the
 * list, one row per task).  Same per-pixel computation as bhr_render_rows;
 * arrays are full-image as there. */
int bhr_render_row_list(const bhr_camera* cam, const bhr_scene* sc, const bhr_options* opt,
                        const int* rows, int nrows, float* rgba, bhr_out* out);

/* Number of OpenMP threads later batch calls use (n >= 1). */
void bhr_set_threads(int n);

/* Colour of one ray from its class, end vector and hit radius. */
void bhr_shade(const bhr_scene* sc, int cls, const double exit_dir[3], double r_hit, float rgba[4]);
/* Bilinear sample of the sky image at direction angles (theta, varphi):
 * texel (i, j) covers column i, row j with its centre at
 * varphi = 2 pi (i + 1/2) / tex_w, theta = pi (j + 1/2) / tex_h; columns wrap
 * around in varphi, rows are clamped at the poles.  Computed in FP64. */
void bhr_sky_sample(const bhr_scene* sc, double theta, double varphi, double rgba[4]);

/* One Dormand-Prince 5(4) step of the photon-orbit system from (u, w) with
 * step h: y_out = 5th-order solution, err = 5th minus embedded 4th order. */
void bhr_dopri5_step(double M, const double y[2], double h, double y_out[2], double err[2]);

/* Azimuth swept by a straight (M = 0) ingoing ray with impact parameter b from
 * radius r0 to the sphere of radius r_sky, where the direction angle psi
 * from the inward radial has sin(psi) = u0 / sqrt(1/b^2 + 2 M u0^3). */
double bhr_dphi_flat(double M, double b, double r0, double r_sky);

#ifdef __cplusplus
}
#endif
#endif
