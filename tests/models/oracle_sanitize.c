/* Driver for the oracle's sanitizer run (tests/test_oracle_sanitizers.py):
 * calls every entry point of oracle/bh_ref.h on small inputs that reach all
 * of its branches -- every end class, the disk, both sky kinds, the paper's
 * fixed-step mode, flat space, the step and sweep caps, radial, zero,
 * non-finite and out-of-range rays, single-row and row-list renders -- so
 * that AddressSanitizer and UndefinedBehaviorSanitizer see them.  Exits 0
 * on completion; the sanitizers abort on the first error. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "bh_ref.h"

static void render(const bhr_camera* cam, const bhr_scene* sc, const bhr_options* opt) {
    const int n = cam->width * cam->height;
    float* rgba = (float*)calloc((size_t)n * 4, sizeof(float));
    bhr_out o;
    o.cls = (uint8_t*)calloc((size_t)n, 1);
    o.b = (double*)calloc((size_t)n, sizeof(double));
    o.phi_end = (double*)calloc((size_t)n, sizeof(double));
    o.exit_dir = (double*)calloc((size_t)n * 3, sizeof(double));
    o.r_hit = (double*)calloc((size_t)n, sizeof(double));
    o.n_acc = (int32_t*)calloc((size_t)n, sizeof(int32_t));
    o.n_rej = (int32_t*)calloc((size_t)n, sizeof(int32_t));
    o.e_drift = (double*)calloc((size_t)n, sizeof(double));
    if (bhr_render_rows(cam, sc, opt, 0, cam->height, rgba, &o) != 0) exit(2);
    int rows[3] = {cam->height - 1, 0, cam->height / 2};
    if (bhr_render_row_list(cam, sc, opt, rows, 3, rgba, &o) != 0) exit(3);
    if (bhr_render_rows(cam, sc, opt, 1, 2, NULL, NULL) != 0) exit(4);
    int counts[5] = {0, 0, 0, 0, 0};
    for (int i = 0; i < n; ++i) counts[o.cls[i] < 5 ? o.cls[i] : 4]++;
    printf("render %dx%d M=%g disk=%d: sky %d captured %d disk %d unresolved %d invalid %d\n",
           cam->width, cam->height, sc->M, sc->has_disk, counts[0], counts[1], counts[2],
           counts[3], counts[4]);
    free(rgba); free(o.cls); free(o.b); free(o.phi_end); free(o.exit_dir); free(o.r_hit);
    free(o.n_acc); free(o.n_rej); free(o.e_drift);
}

int main(void) {
    bhr_set_threads(2);
    bhr_options opt;
    bhr_default_options(&opt);
    bhr_scene sc = {1.0, 1000.0, 1, 6.0, 20.0, -3.0, 10.0, NULL, 0, 0};
    bhr_camera cam = {30.0, 80.0, 20.0, 60.0, 23, 17};
    render(&cam, &sc, &opt);                       /* disk, sky, capture */
    bhr_scene nodisk = sc;
    nodisk.has_disk = 0;
    bhr_camera axial = {25.0, 0.0, 0.0, 50.0, 11, 11}; /* odd: a radial centre ray */
    render(&axial, &nodisk, &opt);
    bhr_scene flat = {0.0, 1000.0, 1, 2.0, 12.0, -3.0, 10.0, NULL, 0, 0};
    render(&cam, &flat, &opt);                     /* M = 0 */
    /* textured sky */
    const int tw = 16, th = 8;
    float* tex = (float*)malloc(sizeof(float) * 4 * tw * th);
    for (int k = 0; k < 4 * tw * th; ++k) tex[k] = (float)(k % 7) / 7.0f;
    bhr_scene texsc = sc;
    texsc.sky_tex = tex;
    texsc.tex_w = tw;
    texsc.tex_h = th;
    render(&cam, &texsc, &opt);
    /* caps and the fixed-step mode */
    bhr_options capped = opt;
    capped.max_steps = 3;
    render(&cam, &sc, &capped);
    capped = opt;
    capped.max_phi = 0.5;
    render(&cam, &sc, &capped);
    bhr_options paper = opt;
    paper.fixed_eps = 2.0;
    render(&cam, &sc, &paper);
    render(&cam, &flat, &paper);
    /* explicit rays: ordinary, radial in and out, zero and non-finite
     * direction, origins inside the photon sphere and outside the sky, a ray
     * in the disk plane */
    const double nan = NAN, inf = INFINITY;
    double o[10][3] = {{30, 0, 1}, {30, 0, 0}, {30, 0, 0}, {30, 0, 0}, {30, 0, 0},
                       {2.5, 0, 0}, {2000, 0, 0}, {30, 0, 0}, {nan, 0, 0}, {40, 3, 0}};
    double d[10][3] = {{-1, 0.2, 0}, {-1, 0, 0}, {1, 0, 0}, {0, 0, 0}, {nan, 1, 0},
                       {-1, 0.1, 0}, {-1, 0.1, 0}, {-1, inf, 0}, {-1, 0, 0}, {-1, 0.3, 0}};
    uint8_t cls[10];
    double b[10], pe[10], ed[30], rh[10], drift[10];
    int32_t na[10], nr[10];
    bhr_out out = {cls, b, pe, ed, rh, na, nr, drift};
    if (bhr_trace_rays(&o[0][0], &d[0][0], 10, &sc, &opt, &out) != 0) return 5;
    if (bhr_trace_rays(&o[0][0], &d[0][0], 10, &flat, &paper, &out) != 0) return 6;
    if (bhr_trace_rays(&o[0][0], &d[0][0], 0, &sc, &opt, &out) != 0) return 7;
    for (int k = 0; k < 10; ++k) printf("ray %d: class %d\n", k, cls[k]);
    /* single functions */
    double origin[3], dir[3];
    if (bhr_camera_ray(&cam, 3, 4, origin, dir) != 0) return 8;
    float px[4];
    const double up[3] = {0, 0, 1};
    for (int c = 0; c < 5; ++c) {
        bhr_shade(&sc, c, up, 7.0, px);
        bhr_shade(&texsc, c, up, 7.0, px);
    }
    double s[4];
    bhr_sky_sample(&texsc, 0.0, 0.0, s);
    bhr_sky_sample(&texsc, 3.14159265358979, 6.28318530717958, s);
    bhr_sky_sample(&texsc, 1.0, -0.1, s);
    double y[2] = {0.02, 0.01}, yo[2], err[2];
    bhr_dopri5_step(1.0, y, 0.3, yo, err);
    bhr_dopri5_step(0.0, y, 0.3, yo, err);
    printf("dphi_flat %.6f %.6f\n", bhr_dphi_flat(1.0, 20.0, 50.0, 1000.0),
           bhr_dphi_flat(0.0, 20.0, 50.0, 1000.0));
    printf("threads %d\n", bhr_max_threads());
    free(tex);
    puts("done");
    return 0;
}
