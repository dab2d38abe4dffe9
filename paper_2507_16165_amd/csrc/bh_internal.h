// Internal definitions shared by the host runtime and the kernels of libbh.
// Not part of the public ABI (include/bh.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bh.h"

namespace bh {

// Error reporting shared by the ABI entry points (bh_abi.cpp).
bh_status fail(bh_status st, const char* fmt, ...);
bh_status hip_fail(hipError_t e, const char* what);

constexpr int kBlock = 256;   // threads per block for every kernel
constexpr int kWave = 64;     // CDNA wavefront

// Per-ray path tags (bh_ray_out.path) and end classes.
enum : uint8_t { SKY = 0, CAPTURED = 1, DISK = 2, UNRESOLVED = 3, INVALID = 4 };
enum : uint8_t { PATH_NONE = 0, PATH_FP64 = 1, PATH_FP32 = 2, PATH_SUR = 3 };

// FP32 result records (Work::res32) hold the end class in their r_hit field:
// a disk hit's radius (> 0), or minus the class for every other end (SKY 0,
// CAPTURED -1, UNRESOLVED -3, INVALID -4; small integers, exact in float).
__device__ __forceinline__ float rec32_radius(uint8_t cls, float r_hit) {
    return cls == DISK ? r_hit : (float)(-(int)cls);
}
__device__ __forceinline__ uint8_t rec32_class(float r) {
    return r > 0.0f ? (uint8_t)DISK : (uint8_t)(int)(-r);
}

// Surrogate trust map: 256 bins of ln(b - b_c) x 64 bins of r0 (see trust_bin).
constexpr int kTrustB = 256, kTrustR = 64;

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// Number of set bits of `mask` below this lane.
__device__ __forceinline__ int rank_in(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Trust-map bin of (b/M, r0/M) on the escape side of the band: 256 bins of
// ln(b - b_c) over [ln 0.05, ln 995] times 64 bins of r0 over [10, 200]; -1
// outside.  Evaluated in FP32 on the device both when the map is built and
// when rays are routed, so both see the same bins.
__device__ __forceinline__ int trust_bin(float bm, float r0m) {
    const float d = bm - 5.19615242270663188f;
    if (!(d > 0.05f)) return -1;
    const float lo = -2.99573227f, hi = 6.90274738f;  // ln 0.05, ln 995
    const float x = (__logf(d) - lo) * (256.0f / (hi - lo));
    const float y = (r0m - 10.0f) * (64.0f / 190.0f);
    if (!(x >= 0.0f && x < 256.0f && y >= 0.0f && y < 64.0f)) return -1;
    return (int)x * kTrustR + (int)y;
}

// Scene constants in the form the kernels use.
struct DevScene {
    double M;
    double r_sky, u_sky;
    double rin, rout, power;
    double urin, urout;       // 1/rin, 1/rout: the disk test runs on u = 1/r
    double cell_rad;          // checker cell in radians
    double inv_cell;          // 1 / cell_rad
    const float4* tex;        // sky image (NULL: checker), tex_h rows of tex_w texels
    double tex_su, tex_sv;    // texels per radian: tex_w / (2 pi), tex_h / pi
    int tex_w, tex_h;
    int has_disk;
};

// Integrator tolerances and caps.
struct DevTol {
    double rtol64, atol64;
    float rtol32, atol32;
    float grow32;             // largest factor on an FP32 ray's rtol32 and atol32 (>= 1)
    double h0, h0_32, hmax, max_phi;  // h0_32: first step of the FP32 integrator
    double newton64;          // Newton stop on |dh| for the sky crossing
    float newton32;
    int max_steps;
    int refill32, refill64;   // idle lanes a wavefront waits for before starting rays (1..64)
};

// Camera basis for one frame, computed once per frame by the host runtime.
struct DevCam {
    double pos[3];            // camera position C
    double fwd[3], right[3], up[3];
    double tan_half;          // tan(vfov/2)
    double e1[3], r0, u0;     // C / |C|, |C| (first basis vector of every ray's plane), 1/|C|
    double ax, bx;            // image-plane x of pixel column px: (px + 1/2) ax + bx
    double inv_w, hinv_w, wd; // 1/W rounded to double, exactly half of it, and W
    // FP32 copies (rounded once on the host) for the FP32 shading path.
    float f_right[3], f_up[3], f_e1[3];
    float f_ax, f_bx, f_tan_half;
    // FP32 set-up of FP32-mode renders: u0 and u0^2 - 2 M u0^3 in float, and
    // the critical band's edges as thresholds on E = w0^2 + u0^2 - 2 M u0^3
    // = 1/b^2, each moved away from the band by a relative margin far above
    // the error of E computed in FP32: E < f_e_in is clearly above the band,
    // E > f_e_out clearly below it (+inf: nothing is).
    float f_u0, f_c0, f_e_in, f_e_out;
    int W, H;
};

// Routing policy applied at set-up.
struct DevRoute {
    int precision;            // BH_FP64 / BH_FP32
    int analytic_capture;
    double band;              // half-width of the critical band, absolute units
    const uint8_t* trust;     // surrogate trust map, or NULL: no surrogate routing
    float r0m;                // camera distance / M (surrogate routing only)
    unsigned long long* stats;// per-call statistics (kCtrStats), or NULL: not collected
};

// Per-ray workspace (structure of arrays, capacity >= rays of the call).
struct Work {
    double* u0;               // 1/|origin| per ray (explicit-ray mode only)
    double2* rec;             // start record {w0, phi1}; w0 = NaN: not in the main queue
    // FP32-mode batches, and FP32 camera renders that return only the image:
    // the start record as {w0, phi1} in FP32, the FP32 integrator's inputs,
    // in rec's memory; NULL otherwise
    float2* rec32;
    double2* res;             // result record {phi_end, r_hit}
    // set together with rec32: the result record as {phi_end, r_hit} in FP32,
    // the FP32 shading's inputs, in res's memory; NULL otherwise.  Its r_hit
    // also carries the end class (rec32_radius), so that shading reads
    // nothing else: clst is then written only by statistics runs and by the
    // rays that end at set-up or in the surrogate.
    float2* res32;
    int32_t* qsur;            // surrogate list (kSurSlices slices): ray indices ...
    double2* qsurrec;         // ... and {b, w0}
    int32_t* rq;              // batch: request index of each ray
    int32_t* clst;            // class | (step evaluations << 3) (see res32)
    uint8_t* path;
    int32_t* q64;             // FP64 band queue (FP32 mode): ray indices ...
    double2* q64rec;          // ... and their start records
    int32_t* ctr;             // queue counters, kCtrInts ints (layout below)
    // statistics runs of single renders: per main-queue wavefront (index
    // block * 4 + wave) the device-clock times at which it entered the queue,
    // found it dry and left it (3 values, zeroed before the launch; tl_waves
    // entries); NULL otherwise
    unsigned long long* tl;
    int tl_waves;
};
constexpr int kTimelineWaves = 1 << 16;   // timeline capacity in wavefronts

// Queue counters (int32 indices into Work::ctr); each head sits on its own
// 256-byte line.
constexpr int kCtrStride = 64;
constexpr int kSlices = 8;                              // main-queue slices
constexpr int kCtrBandSize = 0;                         // FP64 band queue length
constexpr int kCtrBand = kCtrStride;                    // band queue head
constexpr int kCtrMain = 2 * kCtrStride;                // kSlices main-queue heads
constexpr int kSurSlices = 64;                          // surrogate-list slices
constexpr int kCtrSur = kCtrMain + kSlices * kCtrStride; // kSurSlices surrogate-list lengths
// Per-call statistics (bh_last_stats), 64-bit counters: for the FP64 rays
// [0..3] and the FP32 rays [4..7] accepted steps, rejected trial steps,
// Newton re-steps and rays ended by a cap; [8] rays eligible for the
// surrogate whose trust bin was not trusted.
constexpr int kCtrStats = kCtrSur + kSurSlices * kCtrStride;
constexpr int kStatSlots = 16;
constexpr int kCtrInts = kCtrStats + 2 * kStatSlots;

// The surrogate list is filled at set-up in kSurSlices slices, one per
// residue of the set-up block index mod kSurSlices (one atomic per block on
// its slice's counter); a slice holds at most the rays of its blocks.
// Capacity of one slice for n rays (the list needs kSurSlices times this, at
// most n + kSurSlices * kBlock entries).
__host__ __device__ constexpr int64_t sur_slice_cap(int64_t n) {
    const int64_t blocks = (n + kBlock - 1) / kBlock;
    return (blocks + kSurSlices - 1) / kSurSlices * kBlock;
}

// Optional caller-owned outputs (mirrors bh_ray_out).
struct Out {
    uint8_t* cls;
    double* b;
    double* phi_end;
    double* exit_dir;
    double* r_hit;
    int32_t* steps;
    uint8_t* path;
};

// Ray source for set-up and shading: a camera, or explicit origin/direction arrays.
struct Source {
    int64_t n;
    const double* origin;     // n*3, or NULL for camera mode
    const double* dir;        // n*3
    DevCam cam;
};

// Integrator constants of one frame (a single render) or one request (a
// batch, staged in LDS).  The integrator follows the scaled variable v = s u
// (s = 3M, or 1 for M = 0) and w = dv/dphi, with which Eq. (1) reads
// v'' + v = k v^2 (k = 1, or 0 for M = 0): each evaluation of the right-hand
// side is then one fma.  Thresholds are in v: the horizon u = 1/(2M) is
// v = 3/2 exactly.  integ_consts computes them on the host for single renders
// and batches alike, so both round every constant the same way.
struct BatchConst {
    double s, v0, vsky, vrin, vrout, vh, atol64, k;   // FP64 rays
    float s32, v032, vsky32, vrin32, vrout32, vh32, atol32, k32;  // FP32 rays
};

// A request's constants in one precision: the per-request tables that batch
// integrators stage in LDS (32 bytes per request for FP32 batches, 64 for
// FP64 ones, instead of the 96 of BatchConst: a table of hundreds of
// requests then leaves room for all resident blocks).
struct Consts32 { float s, k, vh, vsky, vrin, vrout, atol, v0; };
struct Consts64 { double s, k, vh, vsky, vrin, vrout, atol, v0; };

inline BatchConst integ_consts(const DevScene& sc, const DevTol& t, double u0) {
    BatchConst c;
    const bool flat = !(sc.M > 0.0);
    c.s = flat ? 1.0 : 3.0 * sc.M;
    c.k = flat ? 0.0 : 1.0;
    c.v0 = c.s * u0;
    c.vsky = c.s * sc.u_sky;
    c.vrin = c.s * sc.urin;
    c.vrout = c.s * sc.urout;
    c.vh = flat ? __builtin_inf() : 1.5;
    c.atol64 = c.s * t.atol64;
    c.s32 = (float)c.s;
    c.k32 = (float)c.k;
    c.v032 = (float)c.v0;
    c.vsky32 = (float)c.vsky;
    c.vrin32 = (float)c.vrin;
    c.vrout32 = (float)c.vrout;
    c.vh32 = (float)c.vh;
    c.atol32 = (float)(c.s * (double)t.atol32);
    return c;
}

struct ReqDev {
    DevCam cam;
    DevScene sc;
    DevRoute rt;
    float* rgba;
};

// Per-request constants of the surrogate's batch inference (surrogate-routed
// requests: M > 0 and the sky at 1000 M).
struct SurReq {
    double inv_M;             // 1/M
    float r0m, inv_r0m;       // camera distance / M and its reciprocal
};

struct BatchDev {
    int nreq;
    int64_t total;                 // rays of all requests
    const int64_t* off;            // nreq + 1 ray offsets
    const ReqDev* req;
    const BatchConst* bconst;
    unsigned long long* done;      // pixels shaded per request
    unsigned long long* stamp;     // finish clock per request; stamp[nreq] = start
    int any_flat;                  // some request has M = 0 (integrator variant with k)
    int any_sur;                   // some request routes rays to the surrogate
};

// Launch helpers (defined in bh_kernels.hip).
hipError_t launch_batch_begin(const BatchDev& b, hipStream_t s);
hipError_t launch_integrate_paper(int64_t n, bool explicit_u0, double u0_uniform,
                                  const DevScene& sc, const DevTol& tol, double eps,
                                  const Work& w, int cus, hipStream_t s);
hipError_t launch_batch_setup(const BatchDev& b, const Work& w, hipStream_t s);
hipError_t launch_batch_integrate(const BatchDev& b, const Work& w, const DevTol& tol,
                                  int precision, int cus, int grid_blocks, int chunk,
                                  hipStream_t s);
hipError_t launch_batch_shade(const BatchDev& b, const Work& w, int precision, int cus,
                              hipStream_t s);
hipError_t launch_reset(int32_t* ctr, hipStream_t s);
hipError_t launch_setup(const Source& src, const DevScene& sc, const DevRoute& rt, const Work& w,
                        double* out_b, hipStream_t s);
hipError_t launch_integrate(int64_t n, bool explicit_u0, double u0_uniform, const DevScene& sc,
                            const DevTol& tol, int precision, const Work& w, int cus,
                            int grid_blocks, int chunk, bool stats, hipStream_t s);
hipError_t launch_stats(int64_t n, const Work& w, unsigned long long* out, hipStream_t s);
hipError_t launch_zero(unsigned long long* p, int64_t n, hipStream_t s);
hipError_t launch_shade(const Source& src, const DevScene& sc, const Work& w, float* rgba,
                        const Out& out, int precision, hipStream_t s);
hipError_t launch_shade_samples(const Source& src, const DevScene& sc, const Work& w, float* rgba,
                                const Out& out, int precision, int n, hipStream_t s);
// Surrogate (bh_surrogate.hip): the device trust map (NULL until built) and
// inference pack of a handle, and the render-path kernel over PATH_SUR rays.
const uint8_t* surrogate_trust(const bh_surrogate* s);
const void* surrogate_pack(const bh_surrogate* s);
hipError_t launch_surrogate_render(int64_t n, const Work& w, const void* pack, double M,
                                   double r_cam, int cus, hipStream_t s);
// The same over a batch group's list (FP32 batch records; w.rq gives each
// ray's request within the group, whose constants are req[request]: the
// group's slice of the table).
hipError_t launch_surrogate_render_batch(int64_t n, const Work& w, const void* pack,
                                         const SurReq* req, int cus, hipStream_t s);
// A counter that changes whenever the network's parameters or trust map do.
unsigned surrogate_version(const bh_surrogate* s);
hipError_t launch_count_paths(int64_t n, const Work& w, unsigned long long* counts, hipStream_t s);

}  // namespace bh
