/*
 * bh.h -- C ABI of the MI355X (gfx950) Schwarzschild black-hole ray tracer.
 *
 * Method (arXiv 2507.16165): one ray per pixel of a camera looking at a
 * non-spinning, uncharged hole (Introduction, the 1920x1080 example); each
 * ray stays in its orbital plane through the centre, where the photon-orbit
 * equation Eq. (1) in u = 1/r against the azimuth phi is integrated from the
 * straight-line initial direction (Implementation, "Using GSL for ODE
 * approximation"; Fig. 1) until the ray escapes to the sky sphere, falls
 * through the horizon or hits a thin equatorial disk; the end point is mapped
 * back to 3D and shaded.  Eq. (1) is used as u'' + u = 3 M u^2 (the printed
 * minus sign contradicts the cited Binet equation and the straight-line,
 * critical-parameter and weak-field limits).  Integration is adaptive
 * Dormand-Prince 5(4) with exact event location in place of the paper's
 * fixed step and chord intersection.  Units: G = c = 1.
 *
 * Conventions for every entry point:
 *   - Every array argument is a DEVICE pointer (hipMalloc'd or a torch CUDA
 *     tensor's data_ptr()) allocated and owned by the caller; structs are read
 *     during the call and not retained.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream)
 *     and the call returns without synchronising.  Results are valid after
 *     the caller synchronises that stream.
 *   - The library owns only an internal per-device workspace (per-ray
 *     scratch and queue counters), grown on demand with hipMalloc; growing it
 *     synchronises `stream` first.  bh_reserve() sizes it up front;
 *     bh_shutdown() frees it.  Calls that overlap on one device share the
 *     workspace, so they must be ordered on one stream.
 *   - Argument errors return BH_ERR_ARG at once with nothing enqueued;
 *     bh_last_error() gives a message (thread-local).  A HIP launch error
 *     returns BH_ERR_DEVICE.  Per-ray problems (non-finite input, origin
 *     inside the photon sphere) are a per-ray class BH_INVALID, not an error.
 */
#ifndef BH_H
#define BH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BH_OK = 0,
    BH_ERR_ARG = -1,
    BH_ERR_DEVICE = -2,
    BH_ERR_NOMEM = -3,
    BH_ERR_UNSUPPORTED = -4,
    BH_ERR_STATE = -5
} bh_status;

/* Per-ray end classes. */
enum { BH_SKY = 0, BH_CAPTURED = 1, BH_DISK = 2, BH_UNRESOLVED = 3, BH_INVALID = 4 };

/* Which part of the path produced a ray's result (bh_ray_out.path). */
enum {
    BH_PATH_NONE = 0,     /* classified at set-up: analytic capture, radial, invalid */
    BH_PATH_FP64 = 1,     /* FP64 integrator (all rays in FP64 mode; the critical band in FP32 mode) */
    BH_PATH_FP32 = 2,     /* FP32 integrator */
    BH_PATH_SURROGATE = 3 /* MLP surrogate */
};

/* Precision policy (bh_options.precision). */
enum { BH_FP64 = 0, BH_FP32 = 1 };

/* Scene: a hole of mass M at the origin, a procedural checkerboard sky
 * sphere of radius r_sky and an optional thin opaque disk in the plane z = 0
 * (visible from both faces, edges inclusive, emissivity (r/r_in)^disk_power,
 * first crossing only).  Lengths are absolute (not in units of M). */
typedef struct {
    double M;            /* >= 0; 0 gives straight lines                       */
    double r_sky;        /* > camera / ray-origin distance                      */
    int    has_disk;
    double disk_rin;     /* 0 < disk_rin < disk_rout                            */
    double disk_rout;
    double disk_power;   /* -3 for the r^-3 emissivity                          */
    double checker_deg;  /* checker cell in degrees of theta and varphi (> 0)  */
    const float* sky_tex;/* optional equirectangular sky image instead of the
                            checker: device, tex_h rows (theta 0 .. pi) of tex_w
                            RGBA float texels (varphi 0 .. 2 pi), texel centres at
                            ((i + 1/2) 2 pi / tex_w, (j + 1/2) pi / tex_h);
                            bilinear filtering, wrapping in varphi and clamped at
                            the poles; caller-owned; NULL: the checker          */
    int    tex_w, tex_h; /* >= 1 each, tex_w * tex_h <= 2^28 when sky_tex is set */
} bh_scene;

/* Pinhole camera looking at the hole: position r (sin i cos a, sin i sin a,
 * cos i), "up" = -e_theta, vertical field of view, one ray through each
 * pixel centre, row 0 at the top. */
typedef struct {
    double r;            /* 3M < r < r_sky                                     */
    double incl_deg;     /* i, polar angle from +z                              */
    double azim_deg;     /* a                                                   */
    double fov_deg;      /* in (0, 180)                                         */
    int    width, height;/* >= 1                                                */
} bh_camera;

typedef struct {
    int    precision;        /* BH_FP64, or BH_FP32 with FP64 kept for the critical band */
    double rtol;             /* FP64 mode: the integrator's relative tolerance          */
    double atol;             /* FP64 mode: absolute tolerance; <= 0 means rtol / r_sky  */
    double rtol_fp32;        /* FP32 integrator tolerance; atol = rtol_fp32 / r_sky     */
    double band_halfwidth;   /* FP32 mode: |b - 3 sqrt(3) M| < band_halfwidth * M -> FP64 */
    double h0;               /* first trial step in phi (FP64 integrator)               */
    double h0_fp32;          /* first trial step in phi of the FP32 integrator          */
    double hmax;             /* largest step in phi                                     */
    double max_phi;          /* sweep cap -> BH_UNRESOLVED                              */
    int    max_steps;        /* cap on step attempts per ray -> BH_UNRESOLVED           */
    int    analytic_capture; /* 1: with no disk, an ingoing ray with b below the band is
                                classified CAPTURED without integration (exact: the
                                effective potential peaks at b = 3 sqrt(3) M)          */
    int    grid_blocks;      /* persistent integrator grid, 256-thread blocks; 0 = auto
                                (single renders and traces: 3/4 of the resident
                                blocks; batches: all resident blocks)               */
    int    chunk;            /* rays taken from the queue per wavefront grab; 0 = auto
                                (512 for FP32 batches; FP32 single renders: at least
                                256, about four grabs per wavefront of the grid, 384
                                for a 4K frame; 256 otherwise)                      */
    int    samples_side;     /* bh_render: n x n rays per pixel at the stratified
                                sub-pixel centres, averaged (box filter); 0 or 1 =
                                one ray through the pixel centre; at most 16        */
    int    batch_groups;     /* batches: consecutive request groups traced one after
                                another (1 = one launch sequence for all); 0 = auto:
                                about 64M rays per group                             */
    double fixed_eps;        /* > 0: the paper's fixed-step mode (FP64 only): points
                                about fixed_eps apart (absolute length) along the ray,
                                one Dormand-Prince step each with no error control,
                                disk / horizon / sky hits on the straight chords
                                between consecutive points.  0: adaptive steps with
                                events located on the curve (the default)            */
    const struct bh_surrogate* surrogate; /* FP32 renders only: route eligible rays to this
                                trained network (NULL = off; see bh_surrogate_*)     */
    int    refill_fp32;      /* persistent integrator: a wavefront starts new FP32 rays
                                once this many of its 64 lanes are idle (or its queue is
                                dry); 1..64, 0 = auto (28).  Any value gives the same
                                results; it only changes the schedule                 */
    int    refill_fp64;      /* the same for the FP64 rays of FP64 mode; 0 = auto (6).
                                (The critical band of FP32 mode always refills at 1.) */
    int    collect_stats;    /* bh_render / bh_trace_rays: 1 = count the statistics that
                                bh_last_stats reports, with an instrumented integrator (the
                                same results, somewhat slower); 0 = off.  Batches: must be 0 */
    double rtol_fp32_growth; /* FP32 rays: their tolerance grows with the distance of the
                                impact parameter from the critical value, where the exit
                                direction is less sensitive to integration error: rtol =
                                rtol_fp32 * clamp(|b - 3 sqrt(3) M| / (0.5 M), 1, growth),
                                atol likewise, first step h0_fp32 * (that factor)^(1/5).
                                1 = the same tolerance for every ray; in [1, 1e4]      */
    double rtol_band;        /* FP32 mode: relative tolerance of the FP64 integrator that
                                serves the critical band (atol = rtol_band / r_sky).  A
                                band ray's exit error is about b rtol_band / |b - b_c|,
                                5.2e-6 rad at |b - b_c| = 1e-3 M for 1e-9               */
} bh_options;

/* Optional per-ray outputs (device arrays of length n, any may be NULL).
 * exit_dir is n*3 doubles: the unit vector of the end point (sky-sphere hit,
 * disk hit, or the last point for other classes). */
typedef struct {
    uint8_t* cls;
    double*  b;          /* impact parameter from the first integral            */
    double*  phi_end;    /* azimuth of the end event in the orbital plane       */
    double*  exit_dir;
    double*  r_hit;      /* disk hit radius (BH_DISK), else 0                    */
    int32_t* steps;      /* Dormand-Prince step evaluations spent on the ray    */
    uint8_t* path;       /* BH_PATH_*                                            */
} bh_ray_out;

/* Fills defaults: FP64, rtol 1e-10, atol 0 (-> rtol/r_sky), rtol_fp32 1e-6,
 * rtol_fp32_growth 50, rtol_band 1e-9, band 0.05, h0 1e-2, h0_fp32 0.2, hmax 1, max_phi 8 pi, max_steps
 * 1e6, analytic capture on, auto launch shape, refill thresholds and batch groups.
 * Returns BH_ERR_ARG for NULL. */
bh_status bh_default_options(bh_options* opt);

/* Traces n rays with world-space origins and directions (device, n*3 doubles
 * each, need not be unit length).  Per ray: origins with |o| <= 3M or
 * |o| >= r_sky, zero or non-finite input give BH_INVALID.  Outputs per
 * `out` (at least out->cls must be non-NULL).  n = 0 is a no-op.
 * Paper: Eq. (1) and its initial conditions (sections named above). */
bh_status bh_trace_rays(const double* origin, const double* dir, int64_t n,
                        const bh_scene* scene, const bh_options* opt,
                        const bh_ray_out* out, void* stream);

/* Renders one frame into rgba (device, height*width*4 floats, row-major,
 * row 0 at the top): checker sky (1,1,1,1)/(0.1,0.1,0.1,1), disk
 * (1, 0.6, 0.2) * I with alpha 1, black (0,0,0,1) for captured, unresolved
 * and invalid rays.  per_pixel (may be NULL) receives per-ray records indexed
 * y*width + x.  With opt->samples_side = n > 1 each pixel is the mean of
 * n*n rays through the centres of an n x n grid of sub-pixels (the rays of a
 * (n*width) x (n*height) image of the same camera), and per_pixel then holds
 * n*n*width*height records indexed (n*y + j)*(n*width) + (n*x + i).
 * Paper: Introduction (one ray per pixel; more samples per pixel are the
 * Results' image-quality axis), Results (renders with an Einstein ring). */
bh_status bh_render(const bh_camera* cam, const bh_scene* scene, const bh_options* opt,
                    float* rgba, const bh_ray_out* per_pixel, void* stream);

/* bh_render for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, checks, kernels and results as bh_render (the image and records
 * are bit-identical); it calls no hipMalloc, hipFree or other allocating
 * routine.  Its per-ray workspace is a fixed array in the library's device
 * memory, sized for BH_NOALLOC_MAX_RAYS rays (about 89 MB; rays = width *
 * height * samples_side^2).  Each GPU holds its own copy from the library's
 * first use on it until the process ends.  Larger frames return BH_ERR_ARG
 * with nothing enqueued.  Every call on one GPU shares that GPU's array and
 * it keeps the last call's contents (each call clears what must start at
 * zero itself): calls that overlap on one GPU (several streams or threads)
 * race, so order them on one stream.  It does not share memory with
 * bh_render's workspace, bh_last_counts does not report it, and
 * collect_stats = 1 is BH_ERR_UNSUPPORTED. */
#define BH_NOALLOC_MAX_RAYS 1048576
bh_status bh_render_noalloc(const bh_camera* cam, const bh_scene* scene, const bh_options* opt,
                            float* rgba, const bh_ray_out* per_pixel, void* stream);

/* Sizes the workspace of the current device for frames of up to n rays
 * (synchronises the device if it grows). */
bh_status bh_reserve(int64_t n);

/* Copies the ray counts of the last trace/render on this device into
 * counts[0..3] = {set-up only, FP64 integrator, FP32 integrator, surrogate}.
 * Synchronises `stream`. */
bh_status bh_last_counts(int64_t counts[4], void* stream);

/* Statistics of the last bh_render / bh_trace_rays on this device that ran
 * with bh_options.collect_stats = 1.  Steps are Dormand-Prince step
 * evaluations (the per-ray count bh_ray_out.steps reports is accepted +
 * rejected + newton of that ray). */
typedef struct {
    int64_t rays;            /* rays of the call (every sample of every pixel)          */
    int64_t cls[5];          /* rays per end class, BH_SKY .. BH_INVALID                */
    int64_t path[4];         /* rays per BH_PATH_*                                      */
    int64_t step_evals;      /* all step evaluations of the call                       */
    int64_t accepted[2];     /* accepted steps: [0] FP64 integrator (FP64 mode, or the
                                critical band of FP32 mode), [1] FP32 integrator        */
    int64_t rejected[2];     /* rejected trial steps                                    */
    int64_t newton[2];       /* re-steps of the sky crossing's Newton refinement        */
    int64_t capped[2];       /* rays ended by the step or sweep cap (BH_UNRESOLVED)     */
    int64_t sur_listed;      /* rays routed to the surrogate at set-up                  */
    int64_t sur_fallback;    /* of those, rays the network handed back to the FP32
                                integrator (capture logit not negative)                 */
    int64_t sur_untrusted;   /* rays eligible for the surrogate whose trust-map bin is
                                not trusted (they stay on the integrator)              */
    /* Queue timeline of a bh_render (0 waves for bh_trace_rays): per wavefront
     * of the main queue (FP32 rays in FP32 mode, all rays in FP64 mode), the
     * times at which it entered the queue, found it dry and left it, in
     * microseconds after the first wavefront entered; min, median and max
     * over the wavefronts.  (The blocks that first drain FP32 mode's critical
     * band enter the main queue late.) */
    int64_t timeline_waves;
    double  wave_enter_us[3];
    double  queue_dry_us[3];
    double  wave_exit_us[3];
} bh_stats;

/* Copies the statistics of the last call on this device into *st and
 * synchronises `stream`.  BH_ERR_STATE if that call did not collect them. */
bh_status bh_last_stats(bh_stats* st, void* stream);

/* ---------------------------------------------------------------------------
 * Batched rendering for serving: many requests (each a camera, a scene and an
 * output image) traced together.  The requests are split into consecutive
 * groups of about equal ray count (bh_options.batch_groups).  Within a group
 * all rays share one index space: one set-up launch, ONE persistent
 * integrator launch whose wavefronts pull rays of every request of the group
 * from the same queue (so small and large requests keep the whole chip busy),
 * and one shading launch that records each request's completion on the
 * device clock.  Groups run one after another, so early requests complete
 * early.  With use_graph the whole sequence is captured once into a hipGraph
 * and each bh_batch_launch replays it.  Output pixels are bit-identical to
 * bh_render of each request with the same options.  With opt->surrogate set
 * (FP32), each group's set-up also lists the rays of eligible requests (as
 * bh_render would: M > 0, sky at 1000 M, a valid trust map) for one
 * inference launch before its integrator; the network must outlive the
 * batch, and a launch after its parameters or trust map changed returns
 * BH_ERR_STATE.
 * ------------------------------------------------------------------------- */
typedef struct {
    bh_camera cam;
    bh_scene  scene;
    float*    rgba;        /* device, height*width*4 floats, written by each launch */
} bh_request;

typedef struct {
    int64_t requests, rays;
    double  makespan_ms;   /* last request's completion after the batch start */
    double  p50_ms, p99_ms, min_ms;  /* per-request completion times */
    double  mrays_per_s;   /* rays / makespan */
} bh_batch_summary;

typedef struct bh_batch bh_batch;

/* Validates the requests (as bh_render), allocates the batch's device tables
 * and per-ray workspace (~60 bytes per ray, ~20 more with the surrogate), and
 * with use_graph != 0 captures the launch sequence into a hipGraph.  The
 * request array is copied; the output pointers are kept.  samples_side > 1,
 * fixed_eps > 0 and collect_stats are BH_ERR_UNSUPPORTED.  Each request group
 * stages its requests' integrator constants in one block's LDS (32 bytes per
 * request in FP32 batches, 64 in FP64 ones; about 5000 and 2500 requests per
 * group with 160 KiB): a larger group is BH_ERR_ARG (use more batch_groups).
 * Synchronous. */
bh_status bh_batch_create(const bh_request* reqs, int n, const bh_options* opt, int use_graph,
                          bh_batch** out);
/* Enqueues one execution of the batch on `stream`. */
bh_status bh_batch_launch(bh_batch* b, void* stream);
/* Waits for the last launch and summarises its per-request completion times. */
bh_status bh_batch_stats(bh_batch* b, bh_batch_summary* st);
/* Per-request completion times (ms after the batch start) of the last launch. */
bh_status bh_batch_latencies(bh_batch* b, double* host_ms, int n);
bh_status bh_batch_destroy(bh_batch* b);

/* ---------------------------------------------------------------------------
 * Learned surrogate of the sweep (an extension of the paper's method): an MLP
 * 2 -> 128 -> 128 -> 128 -> 2 (ReLU) maps (b/M, r0/M) of an ingoing ray to the
 * exit azimuth on the sky sphere at r_sky = 1000 M (as a residual over the
 * first-order weak-field sweep, scaled by 12 (M/b)^2) and a capture logit.
 * BF16 weights and activations on the matrix cores, FP32 accumulation and FP32
 * master weights with Adam.  Labels come from the FP64 integrator.  A trust
 * map over (ln(b - 3 sqrt(3) M), r0) bins, built from the integrator's labels,
 * gates which rays a render may hand to the network; outside the band, with
 * the periapsis beyond the disk, in a trusted bin.  Rays whose capture logit
 * disagrees with b > 3 sqrt(3) M go back to the integrator.
 *
 * Parameters are one float vector of 33666 values in the order
 * W1[2][128] b1[128] W2[128][128] b2 W3[128][128] b3 W4[128][2] b4[2]
 * (row-major, layer input index first).  All array arguments are device
 * pointers unless named host_*; sizes are element counts.
 * ------------------------------------------------------------------------- */
typedef struct bh_surrogate bh_surrogate;
typedef struct { float lr, beta1, beta2, eps; } bh_adam;

/* Creates a network from host params (count must be 33666); training batches
 * are multiples of 32 up to max_batch.  Synchronous. */
bh_status bh_surrogate_create(const float* host_params, int64_t count, int64_t max_batch,
                              bh_surrogate** out);
bh_status bh_surrogate_destroy(bh_surrogate* s);
/* Copies {0 params, 1 last gradient, 2 Adam m, 3 Adam v} to host (33666
 * floats).  Synchronous. */
bh_status bh_surrogate_params(const bh_surrogate* s, int which, float* host_out, int64_t count);
/* Replaces params (and Adam state if m, v are non-NULL; step = Adam step
 * count) from host arrays, e.g. to resume from a checkpoint.  Synchronous.
 * Clears the trust map's validity: renders do not route to the network
 * again until bh_surrogate_build_trust or bh_surrogate_set_trust. */
bh_status bh_surrogate_set_params(bh_surrogate* s, const float* host_params, const float* host_m,
                                  const float* host_v, int step);
/* One training step on n samples (b, r0 in units of M; phi_exit = labelled
 * exit azimuth, NaN unless the ray escaped; captured = 0/1): forward, loss
 * (1/n) sum [escaped (y0 - t)^2 + 0.1 BCE(y1, captured)], backward and, if
 * hp->lr > 0, one Adam step.  loss (device float, may be NULL) receives the
 * loss before the step.  n is a multiple of 32 up to max_batch.  A step with
 * lr > 0 changes the parameters and so clears the trust map's validity, as
 * bh_surrogate_set_params does. */
bh_status bh_surrogate_train_step(bh_surrogate* s, const double* b, const double* r0,
                                  const double* phi_exit, const uint8_t* captured, int64_t n,
                                  const bh_adam* hp, float* loss, void* stream);
/* Network outputs y (n x 2 floats) and/or predicted exit azimuth (n doubles)
 * for samples (b, r0); either output may be NULL. */
bh_status bh_surrogate_infer(const bh_surrogate* s, const double* b, const double* r0, int64_t n,
                             float* y, double* phi_pred, void* stream);
/* Labels by FP64 integration (rtol 1e-10, r_sky = 1000, M = 1) of the ingoing
 * ray from (r0, 0, 0) with impact parameter b: phi_exit (NaN unless it
 * escaped) and captured (0/1).  Pairs no ray from r0 can have give NaN, 0. */
bh_status bh_surrogate_labels(bh_surrogate* s, const double* b, const double* r0, int64_t n,
                              double* phi_exit, uint8_t* captured, void* stream);
/* Builds the trust map from n validation samples with labelled phi_true: a
 * bin is trusted if it holds >= min_count escaping samples whose predicted
 * exit azimuth is within max_err (rad) and whose capture logit is negative.
 * y_scratch (n x 2 floats) and phi_scratch (n doubles) are caller scratch. */
bh_status bh_surrogate_build_trust(bh_surrogate* s, const double* b, const double* r0,
                                   const double* phi_true, int64_t n, float max_err, int min_count,
                                   float* y_scratch, double* phi_scratch, void* stream);
/* Copies the trust map (256 x 64 bytes, 1 = trusted) to / from the host. */
bh_status bh_surrogate_trust(const bh_surrogate* s, uint8_t* host_map, int64_t count);
bh_status bh_surrogate_set_trust(bh_surrogate* s, const uint8_t* host_map, int64_t count);

/* Kernel timing for benchmarks.  While enabled, every kernel launch of the
 * library is bracketed by a pair of hipEvents recorded on its launch stream
 * (batch launches too, each group's set-up, integrator and shading; a batch
 * replayed from its hipGraph records none).
 * bh_timing_read() waits for those events and returns, per kernel class
 * {0 set-up, 1 integrator, 2 shading, 3 surrogate}, the summed milliseconds
 * and the number of launches since the previous read, then clears them.
 * Disabled by default (no events recorded). */
bh_status bh_timing_enable(int on);
bh_status bh_timing_read(double ms[4], int64_t launches[4]);

/* Frees the workspace of every device this thread's process used. */
bh_status bh_shutdown(void);

/* Message for the last non-OK status returned on this thread. */
const char* bh_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
