// C ABI of libbh: argument validation, the per-device workspace and the
// launch sequence of a trace or render.  See include/bh.h for the contract.
#include "bh.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "bh_internal.h"

namespace bh {

thread_local char g_err[512] = "";

bh_status fail(bh_status st, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return st;
}

bh_status hip_fail(hipError_t e, const char* what) {
    return fail(BH_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace bh

namespace {

using bh::fail;
using bh::hip_fail;

constexpr double kPi = 3.14159265358979323846;

// Per-device workspace.  Grows on demand; never shrinks until bh_shutdown.
struct Workspace {
    int64_t cap = 0;
    void* base = nullptr;
    bh::Work w{};
    unsigned long long* counts = nullptr;  // 32 counters: bh_last_counts, bh_last_stats
    int64_t last_n = 0;
    bool last_stats = false;               // the last call collected statistics
    int last_tl_waves = 0;                 // ... and the size of its queue timeline
    double clock_hz = 1e8;                 // device wall clock (queue timeline)
    int cus = 0;
};

std::mutex g_mu;
std::vector<Workspace> g_ws;

// Launch timing (bh_timing_*): event pairs per launch, pooled.
struct Timed {
    int cls;
    hipEvent_t a, b;
};
std::mutex g_tmu;
bool g_timing = false;
std::vector<Timed> g_timed;
std::vector<hipEvent_t> g_event_pool;

hipEvent_t take_event() {
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    // Timing only: no system-scope fence when the event is recorded (with it,
    // per-frame renders of 4K frames took 6-8% longer with timing on than
    // off, without it 4-6%; the 16-frame batch step 1.0% and 0.6%);
    // bh_timing_read waits for each event before reading its time.
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
}

// Records the start event of a timed launch; returns the slot or -1.
int timing_begin(int cls, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_tmu);
    if (!g_timing) return -1;
    Timed t{cls, take_event(), take_event()};
    if (!t.a || !t.b) return -1;
    if (hipEventRecord(t.a, s) != hipSuccess) return -1;
    g_timed.push_back(t);
    return (int)g_timed.size() - 1;
}

void timing_end(int slot, hipStream_t s) {
    if (slot < 0) return;
    std::lock_guard<std::mutex> lk(g_tmu);
    (void)hipEventRecord(g_timed[slot].b, s);
}

constexpr size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Layout of the per-ray workspace for up to `cap` rays: rec, res, q64rec
// (16 B per ray each), the surrogate list (qsurrec 16 B, qsur 4 B per entry,
// kSurSlices * sur_slice_cap(cap) entries), u0 (8 B), clst and q64 (4 B
// each), path (1 B), the queue counters and 4 path counters.  Returns the
// bytes it needs; with base != NULL also points w and counts into it.
constexpr size_t carve_workspace(char* base, int64_t cap, bh::Work* w,
                                 unsigned long long** counts) {
    const int64_t scap = bh::kSurSlices * bh::sur_slice_cap(cap);
    const size_t sz16 = align256((size_t)cap * 16), sz8 = align256((size_t)cap * 8),
                 sz4 = align256((size_t)cap * 4), sz1 = align256((size_t)cap);
    const size_t szs16 = align256((size_t)scap * 16), szs4 = align256((size_t)scap * 4);
    const size_t szc = align256(sizeof(int32_t) * bh::kCtrInts);
    const size_t total = 3 * sz16 + szs16 + sz8 + 2 * sz4 + szs4 + sz1 + szc + 256;
    if (base) {
        char* c = base;
        *w = bh::Work{};
        w->rec = (double2*)c; c += sz16;
        w->res = (double2*)c; c += sz16;
        w->q64rec = (double2*)c; c += sz16;
        w->qsurrec = (double2*)c; c += szs16;
        w->qsur = (int32_t*)c; c += szs4;
        w->u0 = (double*)c; c += sz8;
        w->clst = (int32_t*)c; c += sz4;
        w->q64 = (int32_t*)c; c += sz4;
        w->path = (uint8_t*)c; c += sz1;
        w->ctr = (int32_t*)c; c += szc;
        *counts = (unsigned long long*)c;
    }
    return total;
}

bh_status get_workspace(int64_t n, hipStream_t stream, Workspace** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_mu);
    if ((int)g_ws.size() <= dev) g_ws.resize(dev + 1);
    Workspace& ws = g_ws[dev];
    if (ws.cus == 0) {
        int cus = 0;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
        ws.cus = cus > 0 ? cus : 256;
        int khz = 0;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
            ws.clock_hz = 1e3 * khz;
    }
    if (n > ws.cap || ws.base == nullptr) {
        int64_t cap = n > 4096 ? n : 4096;
        const size_t total = carve_workspace(nullptr, cap, nullptr, nullptr);
        if (ws.base) {
            e = hipStreamSynchronize(stream);
            if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
            e = hipDeviceSynchronize();
            if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
            (void)hipFree(ws.base);
            ws.base = nullptr;
            ws.cap = 0;
        }
        void* p = nullptr;
        e = hipMalloc(&p, total);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(BH_ERR_NOMEM, "workspace of %zu bytes: %s", total, hipGetErrorString(e));
        }
        carve_workspace((char*)p, cap, &ws.w, &ws.counts);
        ws.base = p;
        ws.cap = cap;
    }
    *out = &ws;
    return BH_OK;
}

bool finite_pos(double x) { return isfinite(x) && x > 0.0; }

bh_status check_scene(const bh_scene* sc) {
    if (!sc) return fail(BH_ERR_ARG, "scene is NULL");
    if (!(isfinite(sc->M) && sc->M >= 0.0)) return fail(BH_ERR_ARG, "M must be finite and >= 0");
    if (!finite_pos(sc->r_sky)) return fail(BH_ERR_ARG, "r_sky must be > 0");
    if (!finite_pos(sc->checker_deg)) return fail(BH_ERR_ARG, "checker_deg must be > 0");
    if (sc->has_disk) {
        if (!(finite_pos(sc->disk_rin) && isfinite(sc->disk_rout) && sc->disk_rin < sc->disk_rout))
            return fail(BH_ERR_ARG, "disk needs 0 < r_in < r_out");
        if (!isfinite(sc->disk_power)) return fail(BH_ERR_ARG, "disk_power must be finite");
    }
    if (sc->sky_tex) {
        if (sc->tex_w < 1 || sc->tex_h < 1 || (int64_t)sc->tex_w * sc->tex_h > (1ll << 28))
            return fail(BH_ERR_ARG, "sky texture needs 1 <= tex_w, tex_h and tex_w * tex_h <= 2^28");
        if ((uintptr_t)sc->sky_tex % 16 != 0)
            return fail(BH_ERR_ARG, "sky texture must be 16-byte aligned (RGBA float texels)");
    }
    return BH_OK;
}

bh_status check_opt(const bh_options* o) {
    if (!o) return fail(BH_ERR_ARG, "options is NULL");
    if (o->precision != BH_FP64 && o->precision != BH_FP32)
        return fail(BH_ERR_ARG, "precision must be BH_FP64 or BH_FP32");
    if (!finite_pos(o->rtol) || !finite_pos(o->rtol_fp32))
        return fail(BH_ERR_ARG, "tolerances must be > 0");
    if (!isfinite(o->atol)) return fail(BH_ERR_ARG, "atol must be finite");
    if (!finite_pos(o->rtol_band)) return fail(BH_ERR_ARG, "rtol_band must be > 0");
    if (!(o->rtol_fp32_growth >= 1.0 && o->rtol_fp32_growth <= 1e4))
        return fail(BH_ERR_ARG, "rtol_fp32_growth must lie in [1, 1e4]");
    if (!(isfinite(o->band_halfwidth) && o->band_halfwidth >= 0.0))
        return fail(BH_ERR_ARG, "band_halfwidth must be >= 0");
    if (!finite_pos(o->h0) || !finite_pos(o->h0_fp32) || !finite_pos(o->hmax) ||
        !finite_pos(o->max_phi))
        return fail(BH_ERR_ARG, "h0, h0_fp32, hmax and max_phi must be > 0");
    if (o->max_steps < 1) return fail(BH_ERR_ARG, "max_steps must be >= 1");
    if (!(isfinite(o->fixed_eps) && o->fixed_eps >= 0.0))
        return fail(BH_ERR_ARG, "fixed_eps must be finite and >= 0");
    if (o->fixed_eps > 0.0 && (o->precision != BH_FP64 || o->surrogate))
        return fail(BH_ERR_UNSUPPORTED, "the fixed-step mode runs in FP64 without the surrogate");
    if (o->samples_side < 0 || o->samples_side > 16)
        return fail(BH_ERR_ARG, "samples_side must be in [0, 16]");
    if (o->grid_blocks < 0 || o->chunk < 0 || o->batch_groups < 0)
        return fail(BH_ERR_ARG, "launch shape and batch groups must be >= 0");
    if (o->chunk % 64 != 0) return fail(BH_ERR_ARG, "chunk must be a multiple of 64");
    if (o->refill_fp32 < 0 || o->refill_fp32 > 64 || o->refill_fp64 < 0 || o->refill_fp64 > 64)
        return fail(BH_ERR_ARG, "refill thresholds must be in [0, 64]");
    if (o->collect_stats != 0 && o->collect_stats != 1)
        return fail(BH_ERR_ARG, "collect_stats must be 0 or 1");
    return BH_OK;
}

bh::DevScene dev_scene(const bh_scene* sc) {
    bh::DevScene d;
    d.M = sc->M;
    d.r_sky = sc->r_sky;
    d.u_sky = 1.0 / sc->r_sky;
    d.has_disk = sc->has_disk ? 1 : 0;
    d.rin = sc->has_disk ? sc->disk_rin : 0.0;
    d.rout = sc->has_disk ? sc->disk_rout : 0.0;
    d.power = sc->has_disk ? sc->disk_power : 0.0;
    d.urin = sc->has_disk ? 1.0 / sc->disk_rin : 0.0;
    d.urout = sc->has_disk ? 1.0 / sc->disk_rout : 0.0;
    d.cell_rad = sc->checker_deg * kPi / 180.0;
    d.inv_cell = 1.0 / d.cell_rad;
    d.tex = reinterpret_cast<const float4*>(sc->sky_tex);
    d.tex_w = sc->sky_tex ? sc->tex_w : 0;
    d.tex_h = sc->sky_tex ? sc->tex_h : 0;
    d.tex_su = sc->sky_tex ? sc->tex_w / (2.0 * kPi) : 0.0;
    d.tex_sv = sc->sky_tex ? sc->tex_h / kPi : 0.0;
    return d;
}

bh::DevTol dev_tol(const bh_options* o, const bh_scene* sc) {
    bh::DevTol t;
    // FP32 mode integrates only its critical band in FP64, at rtol_band
    if (o->precision == BH_FP32) {
        t.rtol64 = o->rtol_band;
        t.atol64 = o->rtol_band / sc->r_sky;
    } else {
        t.rtol64 = o->rtol;
        t.atol64 = o->atol > 0.0 ? o->atol : o->rtol / sc->r_sky;
    }
    t.rtol32 = (float)o->rtol_fp32;
    t.atol32 = (float)(o->rtol_fp32 / sc->r_sky);
    t.grow32 = (float)o->rtol_fp32_growth;
    t.h0 = o->h0;
    t.h0_32 = o->h0_fp32;
    t.hmax = o->hmax;
    t.max_phi = o->max_phi;
    // Newton stop of the sky-crossing refinement, on the last correction
    // |dh|.  Convergence is quadratic: the error left after applying dh is
    // about |u''/(2w)| dh^2 = (b / (2 r_sky)) dh^2 < dh^2 / 2 at the sky
    // sphere.  FP64 rays refine to 1e-15 as the oracle; FP32 rays stop at
    // 1e-3 rad (residual < 5e-7 rad, far below their integration error),
    // which saves a refinement step on about a quarter of the sky rays.
    t.newton64 = 1e-15;
    t.newton32 = 1e-3f;
    t.max_steps = o->max_steps;
    // Lazy refill: a wavefront starts new rays once this many lanes are idle
    // (or its queue is dry).  Several steps' worth of finished rays: FP32
    // rays took ~11 step evaluations (6.8 with the per-ray tolerance), FP64
    // rays ~60.  Measured on the 4K orbit: 20 and 6 took ~5% less integrator
    // time than 1, and 28 with the FP32 batches' 512-ray chunks 2% less again
    // (single renders measured the same at 20 to 28; at 7.5 steps per ray,
    // 20 to 36 within 1%).
    t.refill32 = o->refill_fp32 > 0 ? o->refill_fp32 : 28;
    t.refill64 = o->refill_fp64 > 0 ? o->refill_fp64 : 6;
    return t;
}

bh::DevRoute dev_route(const bh_options* o, const bh_scene* sc) {
    bh::DevRoute r;
    r.precision = o->precision;
    r.analytic_capture = o->analytic_capture ? 1 : 0;
    r.band = o->band_halfwidth * sc->M;
    r.trust = nullptr;
    r.r0m = 0.0f;
    r.stats = nullptr;
    return r;
}

bh::Out dev_out(const bh_ray_out* o) {
    bh::Out d{};
    if (o) {
        d.cls = o->cls;
        d.b = o->b;
        d.phi_end = o->phi_end;
        d.exit_dir = o->exit_dir;
        d.r_hit = o->r_hit;
        d.steps = o->steps;
        d.path = o->path;
    }
    return d;
}

// Queue chunk: 512 rays per grab for FP32 batches (their one drain at the end
// of many requests gains less from small chunks than the grabs cost: the
// 16-frame 4K orbit integrates 2% faster at 512, with refill 28), 256 for FP64
// renders and batches.  FP32 single renders of n rays take at most about four
// grabs per wavefront of their grid (3/4 of 8 resident blocks per CU, or
// grid_blocks): the smallest multiple of 64 rays, at least 256, that does.
// At 6.8 step evaluations per ray the grabs of 256-ray chunks cost a 4K frame
// (5.3 grabs per wavefront) 11% of its integration against 384 rays (3.5),
// while frames of 2560x1440 and smaller (2.4 grabs or fewer) integrate
// fastest at 256 and 4-14% slower at 320-512.
int auto_chunk(const bh_options* o, bool batch = false, int64_t n = 0, int cus = 0) {
    if (o->chunk > 0) return o->chunk;
    if (batch) return o->precision == BH_FP32 ? 512 : 256;
    if (o->precision != BH_FP32 || cus <= 0 || n <= 0) return 256;
    const int64_t waves = (o->grid_blocks > 0 ? (int64_t)o->grid_blocks : (int64_t)cus * 6) * 4;
    int64_t c = (n + 4 * waves - 1) / (4 * waves);
    c = (c + 63) / 64 * 64;
    return (int)std::min<int64_t>(std::max<int64_t>(c, 256), 1024);
}

bh_status check_camera(const bh_camera* cam, const bh_scene* scene) {
    if (!cam) return fail(BH_ERR_ARG, "camera is NULL");
    if (cam->width < 1 || cam->height < 1) return fail(BH_ERR_ARG, "width and height must be >= 1");
    if ((int64_t)cam->width * cam->height > INT32_MAX)
        return fail(BH_ERR_ARG, "image must have < 2^31 pixels");
    if (!(isfinite(cam->r) && cam->r > 3.0 * scene->M))
        return fail(BH_ERR_ARG, "camera must be outside the photon sphere (r > 3M)");
    if (!(cam->r < scene->r_sky)) return fail(BH_ERR_ARG, "camera must be inside the sky sphere");
    if (!(isfinite(cam->fov_deg) && cam->fov_deg > 0.0 && cam->fov_deg < 180.0))
        return fail(BH_ERR_ARG, "fov_deg must be in (0, 180)");
    if (!isfinite(cam->incl_deg) || !isfinite(cam->azim_deg))
        return fail(BH_ERR_ARG, "camera angles must be finite");
    return BH_OK;
}

// Camera basis (per frame): position r (sin i cos a, sin i sin a, cos i),
// forward = -position/r, up = -e_theta, right = forward x up; and the FP32
// routing thresholds of its rays in the scene.
bh::DevCam make_cam(const bh_camera* cam, const bh_scene* scene, const bh_options* opt) {
    const double inc = cam->incl_deg * kPi / 180.0, az = cam->azim_deg * kPi / 180.0;
    const double ph[3] = {sin(inc) * cos(az), sin(inc) * sin(az), cos(inc)};
    bh::DevCam c{};
    for (int k = 0; k < 3; ++k) {
        c.pos[k] = cam->r * ph[k];
        c.fwd[k] = -ph[k];
    }
    c.up[0] = -cos(inc) * cos(az);
    c.up[1] = -cos(inc) * sin(az);
    c.up[2] = sin(inc);
    c.right[0] = c.fwd[1] * c.up[2] - c.fwd[2] * c.up[1];
    c.right[1] = c.fwd[2] * c.up[0] - c.fwd[0] * c.up[2];
    c.right[2] = c.fwd[0] * c.up[1] - c.fwd[1] * c.up[0];
    c.tan_half = tan(0.5 * cam->fov_deg * kPi / 180.0);
    c.W = cam->width;
    c.H = cam->height;
    // Pixel-centre coordinates on the image plane at unit distance (vertical
    // field of view, square pixels): x = (2 (px + 1/2) / W - 1) t W / H and
    // y = (1 - 2 (py + 1/2) / H) t, written as (px + 1/2) ax + bx and
    // t - (py + 1/2) ax with ax = 2 t / H, bx = -t W / H.
    c.ax = 2.0 * c.tan_half / cam->height;
    c.bx = -c.tan_half * cam->width / cam->height;
    c.r0 = sqrt(c.pos[0] * c.pos[0] + c.pos[1] * c.pos[1] + c.pos[2] * c.pos[2]);
    for (int k = 0; k < 3; ++k) c.e1[k] = c.pos[k] / c.r0;
    c.u0 = 1.0 / c.r0;
    c.inv_w = 1.0 / cam->width;
    c.hinv_w = 0.5 * c.inv_w;
    c.wd = cam->width;
    for (int k = 0; k < 3; ++k) {
        c.f_right[k] = (float)c.right[k];
        c.f_up[k] = (float)c.up[k];
        c.f_e1[k] = (float)c.e1[k];
    }
    c.f_ax = (float)c.ax;
    c.f_bx = (float)c.bx;
    c.f_tan_half = (float)c.tan_half;
    // E = 1/b^2 is decreasing in b: b above the band is E < 1/(b_c + band)^2,
    // b below it E > 1/(b_c - band)^2.  E in FP32 is good to about 1e-6
    // relative (a few roundings of positive terms); the thresholds move by
    // 1e-5, so a ray the FP32 test calls clear is clear in FP64 too.
    constexpr double kMargin = 1e-5;
    const double M = scene->M, bc = 3.0 * sqrt(3.0) * M, band = opt->band_halfwidth * M;
    c.f_u0 = (float)c.u0;
    c.f_c0 = (float)(c.u0 * c.u0 * (1.0 - 2.0 * M * c.u0));
    const double b_hi = bc + band, b_lo = bc - band;
    c.f_e_in = b_hi > 0.0 ? (float)((1.0 - kMargin) / (b_hi * b_hi)) : __builtin_inff();
    c.f_e_out = b_lo > 0.0 ? (float)((1.0 + kMargin) / (b_lo * b_lo)) : __builtin_inff();
    return c;
}

// The shared sequence on a given workspace w (capacity >= src.n rays):
// reset counters, set-up, integrate, shade.  timed: bracket the launches with
// the bh_timing events (when enabled).
bh_status run_on(const bh::Work& ws_w, int cus, const bh::Source& src, bool explicit_u0,
                 double u0_uniform, const bh_scene* scene, const bh_options* opt, float* rgba,
                 const bh_ray_out* out, hipStream_t stream, int samples_side, bool timed) {
    const bh::DevScene sc = dev_scene(scene);
    const bh::DevTol tol = dev_tol(opt, scene);
    bh::DevRoute rt = dev_route(opt, scene);
    // The surrogate serves FP32 renders of scenes with the sky at 1000 M (the
    // radius it was trained for).
    const void* sur_pack = nullptr;
    if (opt->surrogate && !explicit_u0 && opt->precision == BH_FP32 && scene->M > 0.0 &&
        fabs(scene->r_sky / scene->M - 1000.0) < 1e-9) {
        rt.trust = bh::surrogate_trust(opt->surrogate);
        rt.r0m = (float)(1.0 / (u0_uniform * scene->M));
        sur_pack = rt.trust ? bh::surrogate_pack(opt->surrogate) : nullptr;
    }
    bh::Work w = ws_w;
    if (!explicit_u0) w.u0 = nullptr;
    // An FP32 camera render that returns only the image keeps its start and
    // result records in FP32, in the FP64 records' memory, as FP32 batches
    // do: set-up writes, the integrator reads and writes, and shading reads
    // 16 bytes per ray fewer, for the same pixels (FP32 shading rounds its
    // inputs to float either way).  Per-ray outputs, the surrogate,
    // samples per pixel and the fixed-step mode keep the FP64 records.
    const bh::Out dout = dev_out(out);
    const bool any_out = dout.cls || dout.b || dout.phi_end || dout.exit_dir || dout.r_hit ||
                         dout.steps || dout.path;
    if (opt->precision == BH_FP32 && !explicit_u0 && !any_out && !sur_pack &&
        !(opt->fixed_eps > 0.0) && samples_side == 1) {
        w.rec32 = reinterpret_cast<float2*>(w.rec);
        w.res32 = reinterpret_cast<float2*>(w.res);
    }
    const bool stats = opt->collect_stats != 0;
    if (stats) rt.stats = reinterpret_cast<unsigned long long*>(w.ctr + bh::kCtrStats);
    hipError_t e = bh::launch_reset(w.ctr, stream);
    if (e != hipSuccess) return hip_fail(e, "reset");
    int t = timed ? timing_begin(0, stream) : -1;
    e = bh::launch_setup(src, sc, rt, w, out ? out->b : nullptr, stream);
    timing_end(t, stream);
    if (e != hipSuccess) return hip_fail(e, "setup");
    if (sur_pack) {
        t = timed ? timing_begin(3, stream) : -1;
        e = bh::launch_surrogate_render(src.n, w, sur_pack, scene->M, 1.0 / u0_uniform, cus, stream);
        timing_end(t, stream);
        if (e != hipSuccess) return hip_fail(e, "surrogate");
    }
    t = timed ? timing_begin(1, stream) : -1;
    e = opt->fixed_eps > 0.0
            ? bh::launch_integrate_paper(src.n, explicit_u0, u0_uniform, sc, tol, opt->fixed_eps, w,
                                         cus, stream)
            : bh::launch_integrate(src.n, explicit_u0, u0_uniform, sc, tol, opt->precision, w,
                                   cus, opt->grid_blocks, auto_chunk(opt, false, src.n, cus), stats,
                                   stream);
    timing_end(t, stream);
    if (e != hipSuccess) return hip_fail(e, "integrate");
    t = timed ? timing_begin(2, stream) : -1;
    e = samples_side > 1
            ? bh::launch_shade_samples(src, sc, w, rgba, dev_out(out), opt->precision, samples_side,
                                       stream)
            : bh::launch_shade(src, sc, w, rgba, dev_out(out), opt->precision, stream);
    timing_end(t, stream);
    if (e != hipSuccess) return hip_fail(e, "shade");
    return BH_OK;
}

// The same sequence on the library's per-device workspace (grown on demand).
bh_status run(const bh::Source& src, bool explicit_u0, double u0_uniform, const bh_scene* scene,
              const bh_options* opt, float* rgba, const bh_ray_out* out, hipStream_t stream,
              int samples_side = 1) {
    Workspace* ws = nullptr;
    bh_status st = get_workspace(src.n, stream, &ws);
    if (st != BH_OK) return st;
    bh::Work w = ws->w;
    if (opt->collect_stats && !explicit_u0) {
        // the queue timeline goes to the explicit-ray u0 array, unused here
        w.tl = reinterpret_cast<unsigned long long*>(ws->w.u0);
        w.tl_waves = (int)std::min<int64_t>(bh::kTimelineWaves, ws->cap / 3);
        hipError_t e = bh::launch_zero(w.tl, 3 * (int64_t)w.tl_waves, stream);
        if (e != hipSuccess) return hip_fail(e, "timeline");
    }
    st = run_on(w, ws->cus, src, explicit_u0, u0_uniform, scene, opt, rgba, out, stream,
                samples_side, true);
    if (st == BH_OK) {
        ws->last_n = src.n;
        ws->last_stats = opt->collect_stats != 0;
        ws->last_tl_waves = w.tl ? w.tl_waves : 0;
    }
    return st;
}

}  // namespace

// ---------------------------------------------------------------------------
// Allocation-free rendering (bh_render_noalloc).  The per-ray workspace of a
// call is this fixed device array, laid out exactly as the per-device
// workspace for BH_NOALLOC_MAX_RAYS rays.  Each GPU the library runs on holds
// its own copy at its own address from the code object's load until the
// process ends.  Host code must not pass the array's name to a kernel (on the
// host it is only a stand-in for the symbol): it uses the device address that
// hipGetSymbolAddress returned on that device.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kNoAllocBytes = carve_workspace(nullptr, BH_NOALLOC_MAX_RAYS, nullptr, nullptr);
}  // namespace

static __device__ __align__(256) char scratch[kNoAllocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_nmu;
char* g_scratch_dev[kMaxDevices] = {};  // device address of `scratch`, per device
int g_scratch_cus[kMaxDevices] = {};

// Device address of this device's `scratch` array (looked up once per device,
// with that device current) and the device's CU count.  No allocation.
bh_status noalloc_scratch(char** base, int* cus) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return fail(BH_ERR_UNSUPPORTED, "bh_render_noalloc supports devices 0..%d", kMaxDevices - 1);
    std::lock_guard<std::mutex> lk(g_nmu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(BH_ERR_DEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        int c = 0;
        e = hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
        g_scratch_cus[dev] = c > 0 ? c : 256;
        g_scratch_dev[dev] = (char*)p;
    }
    *base = g_scratch_dev[dev];
    *cus = g_scratch_cus[dev];
    return BH_OK;
}

// Checks of bh_render's arguments; fills the ray source (the sample camera
// for samples_side > 1) and the sample count per side.
bh_status render_source(const bh_camera* cam, const bh_scene* scene, const bh_options* opt,
                        const float* rgba, bh::Source* src, int* nside) {
    bh_status st = check_scene(scene);
    if (st != BH_OK) return st;
    if ((st = check_opt(opt)) != BH_OK) return st;
    if ((st = check_camera(cam, scene)) != BH_OK) return st;
    if (!rgba) return fail(BH_ERR_ARG, "rgba is NULL");
    const int n = opt->samples_side > 1 ? opt->samples_side : 1;
    // n x n samples per pixel: the rays of the same camera at n times the
    // resolution (their pixel centres are the stratified sub-pixel centres)
    bh_camera sub = *cam;
    if ((int64_t)cam->width * n * cam->height * n > INT32_MAX)
        return fail(BH_ERR_ARG, "image * samples must have < 2^31 rays");
    sub.width = cam->width * n;
    sub.height = cam->height * n;
    *src = bh::Source{};
    src->n = (int64_t)sub.width * sub.height;
    src->cam = make_cam(&sub, scene, opt);
    *nside = n;
    return BH_OK;
}

}  // namespace

extern "C" {

bh_status bh_default_options(bh_options* o) {
    if (!o) return fail(BH_ERR_ARG, "options is NULL");
    memset(o, 0, sizeof *o);
    o->precision = BH_FP64;
    o->rtol = 1e-10;
    o->atol = 0.0;
    o->rtol_fp32 = 1e-6;
    // FP32 rays far from the critical curve take up to 50x the tolerance.  On
    // the 16 4K orbit frames that leaves the largest exit and disk-radius
    // errors where they were (rays next to the critical band, which keep the
    // base tolerance; the far rays reach about 0.6 of them) and takes 6.8
    // instead of 11.2 step evaluations per ray.
    o->rtol_fp32_growth = 50.0;
    // The critical band of FP32 mode needs the FP32 path's 1e-4 rad, not the
    // FP64 mode's accuracy: at 1e-9 a band ray's exit error, b rtol / |b - b_c|,
    // stays below 5.2e-6 rad wherever band rays are compared (|b - b_c| >=
    // 1e-3 M), and one-frame renders end sooner (their longest band rays set
    // the end of the launch).
    o->rtol_band = 1e-9;
    o->band_halfwidth = 0.05;
    o->h0 = 1e-2;
    // The FP32 path starts near the step its base tolerance allows in the far
    // field (rtol 1e-6: ~0.2 rad) instead of ramping up from 1e-2; a ray whose
    // tolerance grows by f starts at 0.2 f^(1/5).
    o->h0_fp32 = 0.2;
    o->hmax = 1.0;
    o->max_phi = 8.0 * kPi;
    o->max_steps = 1000000;
    o->analytic_capture = 1;
    o->grid_blocks = 0;
    o->chunk = 0;
    return BH_OK;
}

bh_status bh_trace_rays(const double* origin, const double* dir, int64_t n, const bh_scene* scene,
                        const bh_options* opt, const bh_ray_out* out, void* stream) {
    if (n < 0) return fail(BH_ERR_ARG, "n must be >= 0");
    if (n > INT32_MAX) return fail(BH_ERR_ARG, "n must be < 2^31");
    bh_status st = check_scene(scene);
    if (st != BH_OK) return st;
    if ((st = check_opt(opt)) != BH_OK) return st;
    if (n == 0) return BH_OK;
    if (!out || !out->cls) return fail(BH_ERR_ARG, "out->cls is required");
    if (!origin || !dir) return fail(BH_ERR_ARG, "origin and dir are required");
    bh::Source src{};
    src.n = n;
    src.origin = origin;
    src.dir = dir;
    return run(src, true, 0.0, scene, opt, nullptr, out, (hipStream_t)stream);
}

bh_status bh_render(const bh_camera* cam, const bh_scene* scene, const bh_options* opt,
                    float* rgba, const bh_ray_out* per_pixel, void* stream) {
    bh::Source src;
    int n = 1;
    bh_status st = render_source(cam, scene, opt, rgba, &src, &n);
    if (st != BH_OK) return st;
    return run(src, false, 1.0 / cam->r, scene, opt, rgba, per_pixel, (hipStream_t)stream, n);
}

bh_status bh_render_noalloc(const bh_camera* cam, const bh_scene* scene, const bh_options* opt,
                            float* rgba, const bh_ray_out* per_pixel, void* stream) {
    bh::Source src;
    int n = 1;
    bh_status st = render_source(cam, scene, opt, rgba, &src, &n);
    if (st != BH_OK) return st;
    if (opt->collect_stats)
        return fail(BH_ERR_UNSUPPORTED, "bh_render_noalloc does not collect statistics");
    if (src.n > BH_NOALLOC_MAX_RAYS)
        return fail(BH_ERR_ARG,
                    "bh_render_noalloc: %lld rays (width * height * samples_side^2) exceed its "
                    "fixed workspace of %d rays",
                    (long long)src.n, BH_NOALLOC_MAX_RAYS);
    char* base = nullptr;
    int cus = 0;
    if ((st = noalloc_scratch(&base, &cus)) != BH_OK) return st;
    bh::Work w{};
    unsigned long long* counts = nullptr;
    carve_workspace(base, BH_NOALLOC_MAX_RAYS, &w, &counts);
    // Same launch sequence and kernels as bh_render; no timing events (their
    // creation could allocate).  The sequence starts by clearing the queue
    // counters with a kernel, so nothing left by an earlier call is read.
    return run_on(w, cus, src, false, 1.0 / cam->r, scene, opt, rgba, per_pixel,
                  (hipStream_t)stream, n, false);
}

bh_status bh_reserve(int64_t n) {
    if (n < 0 || n > INT32_MAX) return fail(BH_ERR_ARG, "n out of range");
    Workspace* ws = nullptr;
    return get_workspace(n, nullptr, &ws);
}

bh_status bh_last_counts(int64_t counts[4], void* stream) {
    if (!counts) return fail(BH_ERR_ARG, "counts is NULL");
    Workspace* ws = nullptr;
    bh_status st = get_workspace(0, (hipStream_t)stream, &ws);
    if (st != BH_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemsetAsync(ws->counts, 0, 4 * sizeof(unsigned long long), s);
    if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync");
    if (ws->last_n > 0) {
        e = bh::launch_count_paths(ws->last_n, ws->w, ws->counts, s);
        if (e != hipSuccess) return hip_fail(e, "count");
    }
    unsigned long long h[4] = {0, 0, 0, 0};
    e = hipMemcpyAsync(h, ws->counts, sizeof h, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    for (int k = 0; k < 4; ++k) counts[k] = (int64_t)h[k];
    return BH_OK;
}

bh_status bh_last_stats(bh_stats* st, void* stream) {
    if (!st) return fail(BH_ERR_ARG, "st is NULL");
    Workspace* ws = nullptr;
    bh_status rc = get_workspace(0, (hipStream_t)stream, &ws);
    if (rc != BH_OK) return rc;
    if (!ws->last_stats || ws->last_n == 0)
        return fail(BH_ERR_STATE, "the last call on this device did not collect statistics");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemsetAsync(ws->counts, 0, 10 * sizeof(unsigned long long), s);
    if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync");
    e = bh::launch_stats(ws->last_n, ws->w, ws->counts, s);
    if (e != hipSuccess) return hip_fail(e, "stats");
    unsigned long long h[10];
    std::vector<int32_t> ctr(bh::kCtrInts);
    e = hipMemcpyAsync(h, ws->counts, sizeof h, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ctr.data(), ws->w.ctr, sizeof(int32_t) * bh::kCtrInts,
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "reading the statistics");
    unsigned long long c[bh::kStatSlots];
    memcpy(c, ctr.data() + bh::kCtrStats, sizeof c);
    *st = bh_stats{};
    st->rays = ws->last_n;
    for (int k = 0; k < 5; ++k) st->cls[k] = (int64_t)h[k];
    for (int k = 0; k < 4; ++k) st->path[k] = (int64_t)h[5 + k];
    st->step_evals = (int64_t)h[9];
    for (int k = 0; k < 2; ++k) {
        st->accepted[k] = (int64_t)c[4 * k];
        st->rejected[k] = (int64_t)c[4 * k + 1];
        st->newton[k] = (int64_t)c[4 * k + 2];
        st->capped[k] = (int64_t)c[4 * k + 3];
    }
    int64_t listed = 0;
    for (int q = 0; q < bh::kSurSlices; ++q) listed += ctr[bh::kCtrSur + q * bh::kCtrStride];
    st->sur_listed = listed;
    st->sur_fallback = listed - st->path[BH_PATH_SURROGATE];
    st->sur_untrusted = (int64_t)c[8];
    if (ws->last_tl_waves > 0) {
        std::vector<unsigned long long> tl(3 * (size_t)ws->last_tl_waves);
        e = hipMemcpy(tl.data(), ws->w.u0, sizeof(unsigned long long) * tl.size(),
                      hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "reading the queue timeline");
        std::vector<double> t[3];
        unsigned long long t0 = ~0ull;
        for (int k = 0; k < ws->last_tl_waves; ++k)
            if (tl[3 * k]) t0 = std::min(t0, tl[3 * k]);
        for (int k = 0; k < ws->last_tl_waves; ++k) {
            if (!tl[3 * k]) continue;  // a wavefront of the band only, or not launched
            for (int q = 0; q < 3; ++q)
                t[q].push_back(tl[3 * k + q] >= t0 ? 1e6 * (double)(tl[3 * k + q] - t0) / ws->clock_hz : 0.0);
        }
        st->timeline_waves = (int64_t)t[0].size();
        double* dst[3] = {st->wave_enter_us, st->queue_dry_us, st->wave_exit_us};
        for (int q = 0; q < 3 && !t[q].empty(); ++q) {
            std::sort(t[q].begin(), t[q].end());
            dst[q][0] = t[q].front();
            dst[q][1] = t[q][t[q].size() / 2];
            dst[q][2] = t[q].back();
        }
    }
    return BH_OK;
}

}  // extern "C"

struct bh_batch {
    int device = 0;
    int nreq = 0;
    int64_t total = 0;
    int use_graph = 0;
    void* base = nullptr;
    bh::BatchDev dev{};
    bh::Work w{};
    bh::DevTol tol{};
    int precision = 0, grid_blocks = 0, chunk = 256, cus = 256;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t last = nullptr;
    double clock_hz = 1e8;
    // consecutive request groups: tables (offsets relative to the group's
    // first ray) and the group's slice of the per-ray workspace
    std::vector<bh::BatchDev> gdev;
    std::vector<bh::Work> gw;
    std::vector<int> gfirst;  // first request of each group (the tables' rq are group-local)
    // surrogate routing (FP32 batches with a trusted network): the network,
    // its parameter/trust version at creation, its inference pack and the
    // per-request constants of its inference
    const bh_surrogate* sur = nullptr;
    unsigned sur_version = 0;
    const void* sur_pack = nullptr;
    const bh::SurReq* sur_req = nullptr;
};

namespace {
// Enqueues a whole batch: start stamp, then each group's sequence.
// timed: bracket each launch with the bh_timing events (not while capturing).
hipError_t launch_groups(const bh_batch* b, hipStream_t s, bool timed) {
    hipError_t e = bh::launch_batch_begin(b->dev, s);
    for (size_t g = 0; g < b->gdev.size() && e == hipSuccess; ++g) {
        int t = timed ? timing_begin(0, s) : -1;
        e = bh::launch_batch_setup(b->gdev[g], b->gw[g], s);
        timing_end(t, s);
        if (e != hipSuccess) break;
        if (b->sur_pack && b->gdev[g].any_sur) {
            t = timed ? timing_begin(3, s) : -1;
            e = bh::launch_surrogate_render_batch(b->gdev[g].total, b->gw[g], b->sur_pack,
                                                  b->sur_req + b->gfirst[g], b->cus, s);
            timing_end(t, s);
            if (e != hipSuccess) break;
        }
        t = timed ? timing_begin(1, s) : -1;
        e = bh::launch_batch_integrate(b->gdev[g], b->gw[g], b->tol, b->precision, b->cus,
                                       b->grid_blocks, b->chunk, s);
        timing_end(t, s);
        if (e != hipSuccess) break;
        t = timed ? timing_begin(2, s) : -1;
        e = bh::launch_batch_shade(b->gdev[g], b->gw[g], b->precision, b->cus, s);
        timing_end(t, s);
    }
    return e;
}

// Group boundaries (request indices, G+1 of them): consecutive requests with
// about total/G rays each; G from the option, or about 64M rays per group.
std::vector<int> make_groups(const std::vector<int64_t>& off, int option) {
    const int n = (int)off.size() - 1;
    const int64_t N = off[n];
    int G = option > 0 ? option : (int)((N + (64ll << 20) - 1) / (64ll << 20));
    if (G < 1) G = 1;
    if (G > n) G = n;
    std::vector<int> gr{0};
    for (int r = 1; r < n && (int)gr.size() < G; ++r)
        if (off[r] * G >= N * (int64_t)gr.size()) gr.push_back(r);
    gr.push_back(n);
    return gr;
}
}  // namespace

extern "C" {

bh_status bh_batch_create(const bh_request* reqs, int n, const bh_options* opt, int use_graph,
                          bh_batch** out) {
    if (!out) return fail(BH_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!reqs || n < 1) return fail(BH_ERR_ARG, "need at least one request");
    bh_status st = check_opt(opt);
    if (st != BH_OK) return st;
    if (opt->collect_stats) return fail(BH_ERR_UNSUPPORTED, "batches do not collect statistics");
    if (opt->samples_side > 1) return fail(BH_ERR_UNSUPPORTED, "batches trace one ray per pixel");
    if (opt->fixed_eps > 0.0) return fail(BH_ERR_UNSUPPORTED, "batches use adaptive steps");
    std::vector<bh::ReqDev> req(n);
    std::vector<bh::BatchConst> bc(n);
    std::vector<bh::SurReq> sreq(n);
    std::vector<int> routes(n, 0);
    std::vector<int64_t> off(n + 1, 0);
    int any_flat = 0, any_sur = 0;
    // The surrogate serves FP32 requests whose sky is at 1000 M (the radius it
    // was trained for), while its trust map is valid.
    const uint8_t* trust = opt->surrogate && opt->precision == BH_FP32
                               ? bh::surrogate_trust(opt->surrogate) : nullptr;
    for (int r = 0; r < n; ++r) {
        const bh_request& q = reqs[r];
        if ((st = check_scene(&q.scene)) != BH_OK) return fail(st, "request %d: %s", r, bh_last_error());
        if ((st = check_camera(&q.cam, &q.scene)) != BH_OK)
            return fail(st, "request %d: %s", r, bh_last_error());
        if (!q.rgba) return fail(BH_ERR_ARG, "request %d: rgba is NULL", r);
        req[r].cam = make_cam(&q.cam, &q.scene, opt);
        req[r].sc = dev_scene(&q.scene);
        req[r].rt = dev_route(opt, &q.scene);
        req[r].rgba = q.rgba;
        const bh::DevTol t = dev_tol(opt, &q.scene);
        bc[r] = bh::integ_consts(req[r].sc, t, 1.0 / q.cam.r);
        any_flat = any_flat || !(q.scene.M > 0.0);
        sreq[r] = bh::SurReq{0.0, 0.0f, 0.0f};
        if (trust && q.scene.M > 0.0 && fabs(q.scene.r_sky / q.scene.M - 1000.0) < 1e-9) {
            req[r].rt.trust = trust;
            req[r].rt.r0m = (float)(q.cam.r / q.scene.M);
            sreq[r] = bh::SurReq{1.0 / q.scene.M, (float)(q.cam.r / q.scene.M),
                                 (float)(q.scene.M / q.cam.r)};
            routes[r] = 1;
            any_sur = 1;
        }
        off[r + 1] = off[r] + (int64_t)q.cam.width * q.cam.height;
    }
    if (off[n] > INT32_MAX) return fail(BH_ERR_ARG, "a batch must have < 2^31 rays");
    bh_batch* b = new bh_batch();
    b->nreq = n;
    b->total = off[n];
    b->use_graph = use_graph ? 1 : 0;
    b->tol = dev_tol(opt, &reqs[0].scene);
    b->precision = opt->precision;
    b->grid_blocks = opt->grid_blocks;
    b->chunk = auto_chunk(opt, true);
    auto cleanup = [b](bh_status s) {
        bh_batch_destroy(b);
        return s;
    };
    hipError_t e = hipGetDevice(&b->device);
    if (e != hipSuccess) return cleanup(hip_fail(e, "hipGetDevice"));
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, b->device) == hipSuccess && v > 0)
        b->cus = v;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeWallClockRate, b->device) == hipSuccess && v > 0)
        b->clock_hz = 1e3 * v;
    const int64_t N = b->total;
    const size_t sz16 = align256((size_t)N * 16), sz4 = align256((size_t)N * 4),
                 sz1 = align256((size_t)N), szc = align256(sizeof(int32_t) * bh::kCtrInts);
    const std::vector<int> gr = make_groups(off, opt->batch_groups);
    const int G = (int)gr.size() - 1;
    // A group's integrator stages its requests' constants in LDS (32 bytes
    // per request in FP32 batches, 64 in FP64 ones), its set-up and shading
    // the request offsets (8 bytes each): a group's tables must fit one
    // block's LDS.
    int lds_max = 0;
    if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, b->device) !=
            hipSuccess || lds_max <= 0)
        lds_max = 65536;
    const size_t per_req =
        opt->precision == BH_FP32 ? sizeof(bh::Consts32) : sizeof(bh::Consts64);
    for (int g = 0; g < G; ++g) {
        const size_t ng = (size_t)(gr[g + 1] - gr[g]);
        if (per_req * ng > (size_t)lds_max || 8 * (ng + 1) > (size_t)lds_max)
            return cleanup(fail(BH_ERR_ARG,
                                "request group %d holds %zu requests, more than one block's LDS "
                                "(%d bytes) has room for; use more batch_groups",
                                g, ng, lds_max));
    }
    // per group: its requests' offsets relative to the group's first ray
    std::vector<int64_t> goff;
    for (int g = 0; g < G; ++g)
        for (int r = gr[g]; r <= gr[g + 1]; ++r) goff.push_back(off[r] - off[gr[g]]);
    const size_t tables = align256(sizeof(int64_t) * (n + 1)) + align256(sizeof(bh::ReqDev) * n) +
                          align256(sizeof(bh::BatchConst) * n) + align256(8 * (size_t)n) +
                          align256(8 * (size_t)(n + 1)) + align256(sizeof(int64_t) * goff.size()) +
                          align256(sizeof(bh::SurReq) * n);
    // the surrogate list (rays of one group at a time), sized for the largest group
    int64_t gmax = 0;
    for (int g = 0; g < G; ++g) gmax = std::max(gmax, off[gr[g + 1]] - off[gr[g]]);
    const int64_t scap = any_sur ? bh::kSurSlices * bh::sur_slice_cap(gmax) : 0;
    const size_t szs = align256((size_t)scap * 16) + align256((size_t)scap * 4);
    const size_t total = 3 * sz16 + 3 * sz4 + sz1 + szc + tables + szs;
    e = hipMalloc(&b->base, total);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        b->base = nullptr;
        return cleanup(fail(BH_ERR_NOMEM, "batch buffers of %zu bytes", total));
    }
    char* c = (char*)b->base;
    b->w.rec = (double2*)c; c += sz16;
    b->w.res = (double2*)c; c += sz16;
    b->w.q64rec = (double2*)c; c += sz16;
    b->w.clst = (int32_t*)c; c += sz4;
    b->w.q64 = (int32_t*)c; c += sz4;
    b->w.rq = (int32_t*)c; c += sz4;
    b->w.path = (uint8_t*)c; c += sz1;
    b->w.ctr = (int32_t*)c; c += szc;
    b->w.res32 = opt->precision == BH_FP32 ? (float2*)b->w.res : nullptr;
    b->w.rec32 = opt->precision == BH_FP32 ? (float2*)b->w.rec : nullptr;
    b->w.u0 = nullptr;
    b->w.qsur = nullptr;
    b->w.qsurrec = nullptr;
    if (any_sur) {
        b->w.qsurrec = (double2*)c; c += align256((size_t)scap * 16);
        b->w.qsur = (int32_t*)c; c += align256((size_t)scap * 4);
    }
    int64_t* d_off = (int64_t*)c; c += align256(sizeof(int64_t) * (n + 1));
    bh::ReqDev* d_req = (bh::ReqDev*)c; c += align256(sizeof(bh::ReqDev) * n);
    bh::BatchConst* d_bc = (bh::BatchConst*)c; c += align256(sizeof(bh::BatchConst) * n);
    unsigned long long* d_done = (unsigned long long*)c; c += align256(8 * (size_t)n);
    unsigned long long* d_stamp = (unsigned long long*)c; c += align256(8 * (size_t)(n + 1));
    bh::SurReq* d_sreq = (bh::SurReq*)c; c += align256(sizeof(bh::SurReq) * n);
    int64_t* d_goff = (int64_t*)c;
    if ((e = hipMemcpy(d_off, off.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(d_goff, goff.data(), sizeof(int64_t) * goff.size(), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(d_req, req.data(), sizeof(bh::ReqDev) * n, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(d_bc, bc.data(), sizeof(bh::BatchConst) * n, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(d_sreq, sreq.data(), sizeof(bh::SurReq) * n, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemset(d_stamp, 0, 8 * (size_t)(n + 1))) != hipSuccess)
        return cleanup(hip_fail(e, "batch tables"));
    bh::BatchDev& d = b->dev;
    d.nreq = n;
    d.total = N;
    d.off = d_off;
    d.req = d_req;
    d.bconst = d_bc;
    d.done = d_done;
    d.stamp = d_stamp;
    d.any_flat = any_flat;
    d.any_sur = any_sur;
    if (any_sur) {
        b->sur = opt->surrogate;
        b->sur_version = bh::surrogate_version(opt->surrogate);
        b->sur_pack = bh::surrogate_pack(opt->surrogate);
        b->sur_req = d_sreq;
    }
    for (int g = 0, k = 0; g < G; ++g) {
        const int r0 = gr[g], ng = gr[g + 1] - gr[g];
        const int64_t base = off[r0];
        bh::BatchDev dg = d;
        dg.nreq = ng;
        dg.total = off[gr[g + 1]] - base;
        dg.off = d_goff + k;
        dg.req = d_req + r0;
        dg.bconst = d_bc + r0;
        dg.done = d_done + r0;
        dg.stamp = d_stamp + r0;
        dg.any_sur = 0;
        for (int r = r0; r < r0 + ng; ++r) dg.any_sur |= routes[r];
        k += ng + 1;
        bh::Work wg = b->w;
        wg.rec += base;
        wg.res += base;
        if (wg.res32) wg.res32 += base;
        if (wg.rec32) wg.rec32 += base;
        wg.clst += base;
        wg.rq += base;
        wg.path += base;
        b->gdev.push_back(dg);
        b->gw.push_back(wg);
        b->gfirst.push_back(r0);
    }
    if (b->use_graph) {
        // Capture the whole sequence (counter resets are kernels, not memsets)
        // once; each launch replays it.
        if ((e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking)) != hipSuccess)
            return cleanup(hip_fail(e, "capture stream"));
        if ((e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed)) != hipSuccess)
            return cleanup(hip_fail(e, "hipStreamBeginCapture"));
        e = launch_groups(b, b->cap, false);
        hipGraph_t g = nullptr;
        const hipError_t e2 = hipStreamEndCapture(b->cap, &g);
        b->graph = g;
        if (e != hipSuccess) return cleanup(hip_fail(e, "batch capture"));
        if (e2 != hipSuccess) return cleanup(hip_fail(e2, "hipStreamEndCapture"));
        if ((e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0)) != hipSuccess)
            return cleanup(hip_fail(e, "hipGraphInstantiate"));
    }
    if ((e = hipDeviceSynchronize()) != hipSuccess) return cleanup(hip_fail(e, "sync"));
    *out = b;
    return BH_OK;
}

bh_status bh_batch_launch(bh_batch* b, void* stream) {
    if (!b) return fail(BH_ERR_ARG, "batch is NULL");
    if (b->sur && bh::surrogate_version(b->sur) != b->sur_version)
        return fail(BH_ERR_STATE, "the surrogate's parameters or trust map changed since the batch "
                                  "was created; create the batch again");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if (b->use_graph)
        e = hipGraphLaunch(b->exec, s);
    else
        e = launch_groups(b, s, true);
    if (e != hipSuccess) return hip_fail(e, "batch launch");
    b->last = s;
    return BH_OK;
}

bh_status bh_batch_stats(bh_batch* b, bh_batch_summary* st) {
    if (!b || !st) return fail(BH_ERR_ARG, "batch and stats are required");
    hipError_t e = hipStreamSynchronize(b->last);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    std::vector<unsigned long long> stamp(b->nreq + 1);
    e = hipMemcpy(stamp.data(), b->dev.stamp, 8 * stamp.size(), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "stamps");
    std::vector<double> lat(b->nreq);
    const unsigned long long t0 = stamp[b->nreq];
    for (int r = 0; r < b->nreq; ++r)
        lat[r] = stamp[r] >= t0 ? 1e3 * (double)(stamp[r] - t0) / b->clock_hz : -1.0;
    std::vector<double> sorted = lat;
    std::sort(sorted.begin(), sorted.end());
    auto pct = [&sorted](double p) {
        size_t k = (size_t)ceil(p * sorted.size()) ;
        k = k == 0 ? 0 : k - 1;
        if (k >= sorted.size()) k = sorted.size() - 1;
        return sorted[k];
    };
    st->requests = b->nreq;
    st->rays = b->total;
    st->makespan_ms = sorted.back();
    st->p50_ms = pct(0.50);
    st->p99_ms = pct(0.99);
    st->min_ms = sorted.front();
    st->mrays_per_s = st->makespan_ms > 0 ? (double)b->total / (st->makespan_ms * 1e-3) / 1e6 : 0.0;
    return BH_OK;
}

bh_status bh_batch_latencies(bh_batch* b, double* host_ms, int n) {
    if (!b || !host_ms || n != b->nreq) return fail(BH_ERR_ARG, "need nreq doubles");
    hipError_t e = hipStreamSynchronize(b->last);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    std::vector<unsigned long long> stamp(b->nreq + 1);
    e = hipMemcpy(stamp.data(), b->dev.stamp, 8 * stamp.size(), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "stamps");
    for (int r = 0; r < n; ++r)
        host_ms[r] = 1e3 * ((double)stamp[r] - (double)stamp[n]) / b->clock_hz;
    return BH_OK;
}

bh_status bh_batch_destroy(bh_batch* b) {
    if (!b) return BH_OK;
    (void)hipDeviceSynchronize();
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->base) (void)hipFree(b->base);
    delete b;
    return BH_OK;
}

bh_status bh_timing_enable(int on) {
    std::lock_guard<std::mutex> lk(g_tmu);
    g_timing = on != 0;
    return BH_OK;
}

bh_status bh_timing_read(double ms[4], int64_t launches[4]) {
    if (!ms || !launches) return fail(BH_ERR_ARG, "ms and launches are required");
    std::lock_guard<std::mutex> lk(g_tmu);
    for (int k = 0; k < 4; ++k) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    bh_status st = BH_OK;
    for (Timed& t : g_timed) {
        float v = 0.f;
        hipError_t e = hipEventSynchronize(t.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&v, t.a, t.b);
        if (e != hipSuccess && st == BH_OK) st = hip_fail(e, "hipEventElapsedTime");
        if (t.cls >= 0 && t.cls < 4) {
            ms[t.cls] += v;
            launches[t.cls] += 1;
        }
        g_event_pool.push_back(t.a);
        g_event_pool.push_back(t.b);
    }
    g_timed.clear();
    return st;
}

bh_status bh_shutdown(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (size_t d = 0; d < g_ws.size(); ++d) {
        if (!g_ws[d].base) continue;
        (void)hipSetDevice((int)d);
        (void)hipDeviceSynchronize();
        (void)hipFree(g_ws[d].base);
        g_ws[d] = Workspace{};
    }
    (void)hipSetDevice(cur);
    return BH_OK;
}

const char* bh_last_error(void) { return bh::g_err; }

}  // extern "C"
