// Kernels of the Schwarzschild ray tracer for gfx950 (CDNA4, wave64).
//
// Three stages per frame, each a plain HIP kernel:
//   setup     one thread per ray: camera ray, orbital-plane reduction, initial
//             slope w0 and impact parameter b (FP64), first disk-plane
//             crossing angle, routing (analytic capture / FP64 band / main).
//   integrate persistent: wavefronts pull rays from a queue; each lane runs
//             Dormand-Prince 5(4) on the photon-orbit system until its ray
//             ends, then takes the next ray, so lanes do not idle while the
//             rest of the wavefront finishes longer rays.
//   shade     one thread per ray: end vector, checker / disk colour, one
//             coalesced float4 store per pixel.
// Paper: Eq. (1) (read as u'' + u = 3 M u^2) and the text after it;
// Implementation, "Using GSL for ODE approximation" and Fig. 1 (initial point
// and straight-line successor; step size against accuracy).
#include "bh_internal.h"

#include <math.h>

namespace bh {


constexpr double kPi = 3.14159265358979323846;
constexpr double kBcrit = 5.19615242270663188058;  // 3 sqrt(3)

// ---------------------------------------------------------------------------
// Geometry shared by set-up and shading (identical code, so both stages see
// the same plane basis bit for bit).
// ---------------------------------------------------------------------------
struct Basis {
    double e1[3], e2[3];
    // p = dv . e1 has the sign of the cosine of the angle between the ray and
    // e1; p * iv = cos / sin (iv = 1 / |dv - p e1|, 0 for a radial ray).
    double p, iv, r0, u0;  // u0 = 1/r0
    bool radial, ok;
};

// 1/sqrt(x): for 1e-250 < x < 1e250 the hardware estimate refined by two
// Newton steps r <- r + r (1 - x r^2) / 2 (each squares the relative error;
// the result is within a few ulp); elsewhere IEEE sqrt and division.
__device__ __forceinline__ double rsqrt_d(double x) {
    if (!(x > 1e-250 && x < 1e250)) return 1.0 / sqrt(x);
    double r = __builtin_amdgcn_rsq(x);
    r = fma(0.5 * r, fma(-x * r, r, 1.0), r);
    r = fma(0.5 * r, fma(-x * r, r, 1.0), r);
    return r;
}

// Column px and row py of pixel i < 2^31 (row-major), as exact doubles.
// py = trunc((i + 1/2) / W) from one fma with the rounded 1/W: the quotient
// is within 2^-52 of its true value relative, so within 2^-21 / W, while
// (i + 1/2) / W lies at least 1/(2W) from every integer; truncation therefore
// gives floor(i / W) for every W.  px = i - py W is exact (integers < 2^31).
__device__ __forceinline__ void pixel_of(const DevCam& cam, int64_t i, double& px, double& py) {
    const double id = (double)(uint32_t)i;
    py = trunc(fma(id, cam.inv_w, cam.hinv_w));
    px = fma(-py, cam.wd, id);
}

// Plane of a ray from r0 e1 with direction dv (any length): v = dv - (dv.e1) e1
// is the part of dv orthogonal to e1, e2 = v / |v| (zero for a radial ray).
// Nothing needs dv normalised: the set-up uses the sign of dv.e1 and the
// ratio cos/sin = (dv.e1) / |v|.
__device__ __forceinline__ Basis basis_from(const double e1[3], double r0, double u0, bool ok,
                                            const double dv[3], double M, double r_sky) {
    Basis B;
    B.u0 = u0;
    const double dn2 = dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2];
    B.ok = ok && isfinite(dn2) && (r0 > 3.0 * M) && (r0 < r_sky) && (dn2 > 0.0);
    B.r0 = r0;
    double v[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) B.e1[k] = e1[k];
    B.p = dv[0] * e1[0] + dv[1] * e1[1] + dv[2] * e1[2];
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = dv[k] - B.p * e1[k];
    const double s2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    B.radial = !(s2 > 1e-30 * dn2);  // sin < 1e-15
    const double iv = (B.ok && !B.radial) ? rsqrt_d(s2) : 0.0;
    B.iv = iv;
#pragma unroll
    for (int k = 0; k < 3; ++k) B.e2[k] = v[k] * iv;
    return B;
}

// Plane of a ray with explicit origin o and direction dv.
__device__ __forceinline__ Basis plane_basis(const double o[3], const double dv[3], double M,
                                             double r_sky) {
    const double ro2 = o[0] * o[0] + o[1] * o[1] + o[2] * o[2];
    const bool ok = isfinite(ro2) && ro2 > 0.0;
    const double ir = ok ? rsqrt_d(ro2) : 0.0;
    const double e1[3] = {o[0] * ir, o[1] * ir, o[2] * ir};
    return basis_from(e1, ro2 * ir, ir, ok, dv, M, r_sky);
}

// Plane of camera pixel i (row 0 at the top, through the pixel centre).  The
// camera looks at the hole: e1 = C / |C| = -fwd, and right and up are unit
// vectors orthogonal to fwd and to each other.  The pixel's direction
// fwd + x right + y up therefore has component -1 along e1 (every camera ray
// starts inward) and orthogonal part x right + y up, of length
// sqrt(x^2 + y^2): the plane needs no projection, and has no cancellation
// near the image centre.
__device__ __forceinline__ Basis camera_basis(const DevCam& cam, int64_t i, double M,
                                              double r_sky) {
    double px, py;
    pixel_of(cam, i, px, py);
    const double x = fma(px + 0.5, cam.ax, cam.bx);
    const double y = fma(-(py + 0.5), cam.ax, cam.tan_half);
    Basis B;
    B.u0 = cam.u0;
    B.r0 = cam.r0;
    B.ok = (cam.r0 > 3.0 * M) && (cam.r0 < r_sky);
    B.p = -1.0;
    const double s2 = fma(x, x, y * y);
    B.radial = !(s2 > 1e-30);  // sin < 1e-15
    const double iv = (B.ok && !B.radial) ? rsqrt_d(s2) : 0.0;
    B.iv = iv;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        B.e1[k] = cam.e1[k];
        B.e2[k] = fma(x, cam.right[k], y * cam.up[k]) * iv;
    }
    return B;
}

// Plane of ray i of a source (camera pixel, or explicit origin/direction);
// set-up and shading both call this, so they see the same basis bit for bit.
__device__ __forceinline__ Basis source_basis(const Source& src, int64_t i, double M,
                                              double r_sky) {
    double dv[3];
    if (src.origin) {
        double o[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            o[k] = src.origin[3 * i + k];
            dv[k] = src.dir[3 * i + k];
        }
        return plane_basis(o, dv, M, r_sky);
    }
    return camera_basis(src.cam, i, M, r_sky);
}

// First root in (0, pi] of e1z cos(phi) + e2z sin(phi) = 0; +inf if the
// orbital plane is the disk plane (no crossings).
__device__ __forceinline__ double first_crossing(double a, double bz) {
    if (!(hypot(a, bz) > 1e-15)) return __builtin_inf();
    if (a == 0.0) return kPi;
    if (bz == 0.0) return 0.5 * kPi;
    double p = atan(-a / bz);
    if (p <= 0.0) p += kPi;
    return p;
}

// The same root to FP32 accuracy (the FP32 integrator's): the quotient from
// the hardware reciprocal (1 ulp), then atanf (a few ulp).
__device__ __forceinline__ double first_crossing32(double a, double bz) {
    if (!(a * a + bz * bz > 1e-30)) return __builtin_inf();
    if (a == 0.0) return kPi;
    if (bz == 0.0) return 0.5 * kPi;
    double p = (double)atanf(-(float)a * __builtin_amdgcn_rcpf((float)bz));
    if (p <= 0.0) p += kPi;
    return p;
}

// ---------------------------------------------------------------------------
// Counter reset (a kernel rather than a memset so the sequence can be
// captured in a graph).
// ---------------------------------------------------------------------------
__global__ void k_reset(int32_t* ctr) {
    for (int i = threadIdx.x; i < kCtrInts; i += blockDim.x) ctr[i] = 0;
}

// ---------------------------------------------------------------------------
// Set-up and routing.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double nan_d() { return __builtin_nan(""); }

// Set-up of ray i (index into the per-ray workspace) with origin o and
// direction dv: plane reduction, impact parameter, first disk-plane crossing,
// routing.  Returns the queue the ray joins besides the main one: kToBand
// (FP64 band queue), kToSur (surrogate list) or kToNone.
constexpr int kToNone = 0, kToBand = 1, kToSur = 2;

// BATCH: no path byte (only single renders report it).  R32 (FP32 batches):
// the start record goes to w.rec32, and the result record of a ray that ends
// at set-up to w.res32.
template <bool BATCH = false, bool R32 = false>
__device__ __forceinline__ int setup_ray(const Basis& B, const DevScene& sc, const DevRoute& rt,
                                         int64_t i, const Work& w, double* out_b, double& b,
                                         double& w0, double& phi1) {
    int to = kToNone;
    uint8_t path = PATH_NONE, cls = INVALID;
    double phi_end = 0.0;
    b = 0.0;
    w0 = 0.0;
    phi1 = 0.0;
    if (B.ok && B.radial) {
        // Radial ray: inward is captured (flat space: straight through the
        // centre to the antipode); outward escapes along e1.
        if (B.p < 0.0) {
            cls = sc.M > 0.0 ? CAPTURED : SKY;
            phi_end = sc.M > 0.0 ? 0.0 : kPi;
        } else {
            cls = SKY;
        }
    } else if (B.ok) {
        const double u0 = B.u0;
        w0 = -u0 * B.p * B.iv;
        // First integral of Eq. (1): w^2 + u^2 - 2 M u^3 = 1/b^2.
        const double E0 = w0 * w0 + u0 * u0 - 2.0 * sc.M * u0 * u0 * u0;
        b = rsqrt_d(E0);
        const double bc = kBcrit * sc.M;
        if (w.u0) w.u0[i] = u0;
        // Surrogate: ingoing rays above the band whose periapsis lies outside
        // the disk (u_out^2 - 2 M u_out^3 > 1/b^2: the ray turns before
        // reaching r_out), in a bin the trust map accepts.
        bool sur = false;
        if (rt.trust && B.p < 0.0 && b > bc + rt.band &&
            (!sc.has_disk || sc.urout * sc.urout * (1.0 - 2.0 * sc.M * sc.urout) > E0)) {
            const int bin = trust_bin((float)(b / sc.M), rt.r0m);
            sur = bin >= 0 && rt.trust[bin] != 0;
            if (rt.stats && !sur) atomicAdd(&rt.stats[8], 1ull);
        }
        if (rt.analytic_capture && !sc.has_disk && B.p < 0.0 && b < bc - rt.band) {
            cls = CAPTURED;  // below the potential peak: falls in, no disk to hit
        } else if (sur) {
            path = PATH_SUR;
            to = kToSur;
        } else if (rt.precision == 1 && fabs(b - bc) < rt.band) {
            path = PATH_FP64;
            to = kToBand;
        } else {
            path = rt.precision == 1 ? PATH_FP32 : PATH_FP64;
        }
        // First disk-plane crossing: FP32 accuracy for the FP32 integrator,
        // FP64 for the FP64 paths (FP64 mode and the band).
        if (sc.has_disk) {
            phi1 = (rt.precision == 1 && to != kToBand) ? first_crossing32(B.e1[2], B.e2[2])
                                                        : first_crossing(B.e1[2], B.e2[2]);
        } else {
            phi1 = __builtin_inf();
        }
    }
    if (!BATCH) w.path[i] = path;
    // The main queue is the index range itself; its record marks rays that
    // belong to another path (band, surrogate, set-up only) with w0 = NaN.
    const bool main = path != PATH_NONE && to == kToNone;
    if (R32) w.rec32[i] = make_float2(main ? (float)w0 : __builtin_nanf(""), (float)phi1);
    else w.rec[i] = make_double2(main ? w0 : nan_d(), phi1);
    if (path == PATH_NONE) {
        if (R32) w.res32[i] = make_float2((float)phi_end, rec32_radius(cls, 0.0f));
        else w.res[i] = make_double2(phi_end, 0.0);
        w.clst[i] = cls;
    }
    if (out_b) out_b[i] = b;
    return to;
}

// Set-up of camera pixel i (workspace index g) in FP32 mode without surrogate
// routing.  The routing needs the impact parameter to FP64 accuracy only
// near a band edge: E = w0^2 + u0^2 - 2 M u0^3 = 1/b^2 is first formed in
// FP32 from the start slope, and a ray whose E is clearly outside the band
// (thresholds moved 1e-5 relative away from it, DevCam) is routed on that
// value -- to the FP32 integrator, or, below the band in a scene without a
// disk, to analytic capture: the decisions the FP64 values would take.  Every
// other ray (in or near the band, or the radial ray through the image
// centre) takes the FP64 set-up.
//
// The start slope w0 = u0 / sqrt(x^2 + y^2) is the FP32 integrator's input
// rounded once to float, as the FP64 set-up rounds it: x, y and x^2 + y^2 in
// FP64 (in FP32 the image-plane coordinates cancel near the image centre,
// and a start-direction error is amplified like 1/|b - b_c| by the sweep),
// the reciprocal square root from the hardware estimate and one Newton step
// (relative error ~1e-14, far below float rounding).  out_b (single renders
// only) is the FP64 b.
template <bool BATCH, bool R32>
__device__ __forceinline__ int setup_camera32(const DevCam& cam, const DevScene& sc,
                                              const DevRoute& rt, int64_t i, int64_t g,
                                              const Work& w, double* out_b, double& b,
                                              double& w0, double& phi1) {
    double pxd, pyd;
    pixel_of(cam, i, pxd, pyd);
    const double x = fma(pxd + 0.5, cam.ax, cam.bx);
    const double y = fma(-(pyd + 0.5), cam.ax, cam.tan_half);
    const double s2 = fma(x, x, y * y);
    double iv = __builtin_amdgcn_rsq(s2);
    iv = fma(0.5 * iv, fma(-s2 * iv, iv, 1.0), iv);
    const double w0d = cam.u0 * iv;
    const float w0f = (float)w0d;
    const float E = fmaf(w0f, w0f, cam.f_c0);
    const bool above = E < cam.f_e_in, below = E > cam.f_e_out;
    if (!(s2 > 1e-30 && s2 < 1e30) || !(above | below))
        return setup_ray<BATCH, R32>(camera_basis(cam, i, sc.M, sc.r_sky), sc, rt, g, w, out_b, b,
                                     w0, phi1);
    b = 0.0;
    if (out_b) out_b[g] = rsqrt_d(fma(w0d, w0d, cam.u0 * cam.u0 * (1.0 - 2.0 * sc.M * cam.u0)));
    if (below & (rt.analytic_capture != 0) & !sc.has_disk) {
        // below the potential peak: falls in, no disk to hit
        if (!BATCH) w.path[g] = PATH_NONE;
        if (R32) {
            w.rec32[g] = make_float2(__builtin_nanf(""), 0.0f);
            w.res32[g] = make_float2(0.0f, rec32_radius(CAPTURED, 0.0f));
        } else {
            w.rec[g] = make_double2(nan_d(), 0.0);
            w.res[g] = make_double2(0.0, 0.0);
        }
        w.clst[g] = CAPTURED;
        w0 = 0.0;
        phi1 = 0.0;
        return kToNone;
    }
    // first disk-plane crossing (e2 = (x right + y up) / sqrt(x^2 + y^2))
    phi1 = sc.has_disk ? first_crossing32(cam.e1[2], fma(x, cam.right[2], y * cam.up[2]) * iv)
                       : __builtin_inf();
    if (!BATCH) w.path[g] = PATH_FP32;
    if (R32) w.rec32[g] = make_float2(w0f, (float)phi1);
    else w.rec[g] = make_double2((double)w0f, phi1);
    w0 = (double)w0f;
    return kToNone;
}

// Wave-aggregated append to the FP64 band queue: one atomic per wavefront
// that holds band rays (a fraction of a percent of all wavefronts).
__device__ __forceinline__ void append_band(bool to_q64, int64_t i, double w0, double phi1,
                                            const Work& w) {
    const uint64_t m = __ballot(to_q64);
    if (m) {
        const int leader = __ffsll((unsigned long long)m) - 1;
        int base = 0;
        if (lane_id() == leader) base = atomicAdd(&w.ctr[kCtrBandSize], __popcll(m));
        base = __shfl(base, leader);
        if (to_q64) {
            const int slot = base + rank_in(m);
            w.q64[slot] = (int32_t)i;
            w.q64rec[slot] = make_double2(w0, phi1);
        }
    }
}

// Block-aggregated append to slice (block index mod kSurSlices) of the
// surrogate list: one atomic per block that holds surrogate rays.  Every
// thread of the block calls it (two barriers).
__device__ __forceinline__ void append_sur(bool to_sur, int64_t i, double b, double w0,
                                           int64_t n, const Work& w) {
    __shared__ int s_cnt[kBlock / 64];
    __shared__ int s_base;
    const int wv = threadIdx.x >> 6;
    const uint64_t m = __ballot(to_sur);
    if (lane_id() == 0) s_cnt[wv] = __popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int k = 0; k < kBlock / 64; ++k) {
            const int c = s_cnt[k];
            s_cnt[k] = tot;  // exclusive prefix over the block's wavefronts
            tot += c;
        }
        const int slice = (int)(blockIdx.x % (unsigned)kSurSlices);
        s_base = tot > 0 ? atomicAdd(&w.ctr[kCtrSur + slice * kCtrStride], tot) : 0;
    }
    __syncthreads();
    if (to_sur) {
        const int slice = (int)(blockIdx.x % (unsigned)kSurSlices);
        const int64_t slot = slice * sur_slice_cap(n) + s_base + s_cnt[wv] + rank_in(m);
        w.qsur[slot] = (int32_t)i;
        w.qsurrec[slot] = make_double2(b, w0);
    }
}

// R32: FP32 records (w.rec32 / w.res32), for FP32 camera renders that return
// only the image; the FP32 integrator and shading then read them as batches
// do.
template <bool R32>
__global__ __launch_bounds__(kBlock) void k_setup(Source src, DevScene sc, DevRoute rt, Work w,
                                                  double* out_b) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int to = kToNone;
    double b = 0.0, w0 = 0.0, phi1 = 0.0;
    if (i < src.n) {
        if (!src.origin && rt.precision == 1 && !rt.trust)
            to = setup_camera32<false, R32>(src.cam, sc, rt, i, i, w, out_b, b, w0, phi1);
        else
            to = setup_ray<false, R32>(source_basis(src, i, sc.M, sc.r_sky), sc, rt, i, w, out_b,
                                       b, w0, phi1);
    }
    append_band(to == kToBand, i, w0, phi1, w);
    if (rt.trust) append_sur(to == kToSur, i, b, w0, src.n, w);
}

// Request of batch ray g: the last r with off[r] <= g (binary search over the
// request offsets staged in LDS).
__device__ __forceinline__ int find_req(const int64_t* off, int nreq, int64_t g) {
    int lo = 0, hi = nreq - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ void stage_offsets(const BatchDev& b, int64_t* s_off) {
    for (int k = threadIdx.x; k <= b.nreq; k += blockDim.x) s_off[k] = b.off[k];
    __syncthreads();
}

// *p, read by every lane from the same address, as wave-uniform values
// (scalar registers): a request's constants then cost no per-ray loads.
template <typename S>
__device__ __forceinline__ S uniform_load(const S* __restrict__ p) {
    static_assert(sizeof(S) % 4 == 0, "whole dwords");
    constexpr int n = (int)(sizeof(S) / 4);
    int v[n];
    __builtin_memcpy(v, p, sizeof(S));
#pragma unroll
    for (int k = 0; k < n; ++k) v[k] = __builtin_amdgcn_readfirstlane(v[k]);
    S out;
    __builtin_memcpy(&out, v, sizeof(S));
    return out;
}

// Set-up of pixel i of request q (workspace index g) in a batch: FP32-mode
// requests without surrogate routing take the FP32 camera set-up, the others
// the FP64 set-up (which routes to the surrogate).
template <bool R32>
__device__ __forceinline__ int batch_ray(const ReqDev& q, int64_t i, int64_t g, const Work& w,
                                         double& b, double& w0, double& phi1) {
    if (q.rt.precision == 1 && !q.rt.trust)
        return setup_camera32<true, R32>(q.cam, q.sc, q.rt, i, g, w, nullptr, b, w0, phi1);
    return setup_ray<true, R32>(camera_basis(q.cam, i, q.sc.M, q.sc.r_sky), q.sc, q.rt, g, w,
                                nullptr, b, w0, phi1);
}

// Batch set-up: all requests' rays in one index space; each ray also records
// its request for the integrator.  A block whose rays lie in one request (all
// but a few) takes that request's constants as uniform values; a block that
// straddles requests looks each ray's request up.
template <bool R32>
__global__ __launch_bounds__(kBlock) void k_setup_batch(BatchDev b, Work w) {
    extern __shared__ int64_t s_off[];
    stage_offsets(b, s_off);
    const int64_t g0 = (int64_t)blockIdx.x * kBlock;
    const int64_t g = g0 + threadIdx.x;
    const int64_t glast = min(g0 + (int64_t)kBlock, b.total) - 1;
    const int r0 = __builtin_amdgcn_readfirstlane(find_req(s_off, b.nreq, g0));
    int to = kToNone;
    double bi = 0.0, w0 = 0.0, phi1 = 0.0;
    if (s_off[r0 + 1] > glast) {
        const ReqDev q = uniform_load(b.req + r0);
        if (g < b.total) {
            w.rq[g] = r0;
            to = batch_ray<R32>(q, g - s_off[r0], g, w, bi, w0, phi1);
        }
    } else if (g < b.total) {
        const int r = find_req(s_off, b.nreq, g);
        const ReqDev& q = b.req[r];
        w.rq[g] = r;
        to = batch_ray<R32>(q, g - s_off[r], g, w, bi, w0, phi1);
    }
    append_band(to == kToBand, g, w0, phi1, w);
    if (b.any_sur) append_sur(to == kToSur, g, bi, w0, b.total, w);  // block-uniform
}

// ---------------------------------------------------------------------------
// Dormand-Prince 5(4) step for y = (u, w), y' = (w, g(u)): g(u) = u (3 M u - 1)
// in the variable u = 1/r (the fixed-step mode), g(v) = v (k v - 1) in the
// integrator's scaled variable v = s u (s = 3M, k = 1; s = 1, k = 0 for
// M = 0).  First-same-as-last: g1 = g(u) comes in, g7 = g(u_new) goes out.
// The u component of every stage derivative is the stage's w value, so only
// g is evaluated (6 evaluations per step).
// Tableau: Dormand & Prince (1980); Hairer, Norsett & Wanner, Solving ODEs I,
// Sec. II.5.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T g_of(T M3, T u) {
    return u * fma(M3, u, T(-1));
}

// g of the scaled variable: v^2 - v, one fma; with KAPPA, v (k v) - v, whose
// k = 1 gives the same bits and k = 0 (flat space) gives -v exactly.
template <bool KAPPA, typename T>
__device__ __forceinline__ T g_scaled(T k, T v) {
    if constexpr (KAPPA) return fma(v, v * k, -v);
    else return fma(v, v, -v);
}

template <typename T, typename G>
__device__ __forceinline__ void dp45(const G& g_of, T u, T w, T g1, T h, T& un, T& wn, T& g7,
                                     T& eu, T& ew) {
    // The published tableau.
    constexpr double a21 = 1.0 / 5.0;
    constexpr double a31 = 3.0 / 40.0, a32 = 9.0 / 40.0;
    constexpr double a41 = 44.0 / 45.0, a42 = -56.0 / 15.0, a43 = 32.0 / 9.0;
    constexpr double a51 = 19372.0 / 6561.0, a52 = -25360.0 / 2187.0, a53 = 64448.0 / 6561.0,
                     a54 = -212.0 / 729.0;
    constexpr double a61 = 9017.0 / 3168.0, a62 = -355.0 / 33.0, a63 = 46732.0 / 5247.0,
                     a64 = 49.0 / 176.0, a65 = -5103.0 / 18656.0;
    constexpr double b1 = 35.0 / 384.0, b3 = 500.0 / 1113.0, b4 = 125.0 / 192.0,
                     b5 = -2187.0 / 6784.0, b6 = 11.0 / 84.0;
    constexpr double e1 = 71.0 / 57600.0, e3 = -71.0 / 16695.0, e4 = 71.0 / 1920.0,
                     e5 = -17253.0 / 339200.0, e6 = 22.0 / 525.0, e7 = -1.0 / 40.0;

    // Nystrom form.  The u component's derivative is w itself, so the w value
    // of stage j is w + h sum_m a_jm g_m, and the u value of stage k is
    //   u_k = u + c_k h w + h^2 sum_m abar_km g_m,  c_k = sum_j a_kj,
    //   abar_km = sum_j a_kj a_jm,
    // and likewise u_new = u + h w + h^2 sum_m bbar_m g_m with bbar = b A
    // (sum_j b_j = 1) and the u error h^2 sum_m ebar_m g_m with ebar = e A
    // (the seventh row of A is b; sum_j e_j = 0).  The same step, without the
    // five stage sums for w: the products below are evaluated at compile
    // time from the tableau (bbar_2 = ebar_2 = 0).
    constexpr double c3 = a31 + a32, c4 = a41 + a42 + a43, c5 = a51 + a52 + a53 + a54;
    constexpr double A31 = a32 * a21;
    constexpr double A41 = a42 * a21 + a43 * a31, A42 = a43 * a32;
    constexpr double A51 = a52 * a21 + a53 * a31 + a54 * a41, A52 = a53 * a32 + a54 * a42,
                     A53 = a54 * a43;
    constexpr double A61 = a62 * a21 + a63 * a31 + a64 * a41 + a65 * a51,
                     A62 = a63 * a32 + a64 * a42 + a65 * a52, A63 = a64 * a43 + a65 * a53,
                     A64 = a65 * a54;
    constexpr double B1 = b3 * a31 + b4 * a41 + b5 * a51 + b6 * a61,
                     B3 = b4 * a43 + b5 * a53 + b6 * a63, B4 = b5 * a54 + b6 * a64,
                     B5 = b6 * a65;
    constexpr double E1 = e3 * a31 + e4 * a41 + e5 * a51 + e6 * a61 + e7 * b1,
                     E3 = e4 * a43 + e5 * a53 + e6 * a63 + e7 * b3,
                     E4 = e5 * a54 + e6 * a64 + e7 * b4, E5 = e6 * a65 + e7 * b5, E6 = e7 * b6;

    const T hw = h * w, h2 = h * h;
    const T uhw = u + hw;  // c6 = c7 = 1
    const T g2 = g_of(fma(T(a21), hw, u));
    const T g3 = g_of(fma(h2, T(A31) * g1, fma(T(c3), hw, u)));
    const T g4 = g_of(fma(h2, fma(T(A42), g2, T(A41) * g1), fma(T(c4), hw, u)));
    const T g5 = g_of(fma(h2, fma(T(A53), g3, fma(T(A52), g2, T(A51) * g1)), fma(T(c5), hw, u)));
    const T g6 =
        g_of(fma(h2, fma(T(A64), g4, fma(T(A63), g3, fma(T(A62), g2, T(A61) * g1))), uhw));

    un = fma(h2, fma(T(B5), g5, fma(T(B4), g4, fma(T(B3), g3, T(B1) * g1))), uhw);
    wn = fma(h, fma(T(b6), g6, fma(T(b5), g5, fma(T(b4), g4, fma(T(b3), g3, T(b1) * g1)))), w);
    g7 = g_of(un);

    eu = h2 * fma(T(E6), g6, fma(T(E5), g5, fma(T(E4), g4, fma(T(E3), g3, T(E1) * g1))));
    ew = h * fma(T(e7), g7, fma(T(e6), g6, fma(T(e5), g5, fma(T(e4), g4, fma(T(e3), g3, T(e1) * g1)))));
}

// Step-size factor s err^(-1/5) = s 2^(-log2(err) / 5) from the hardware
// log2 and exp2 (a few ulp; the factor is a heuristic, only the accept test
// needs full precision).  Their limits give the callers' clamps what they
// need: err = NaN or inf gives NaN or 0 (clamped to 0.2), err = 0 gives inf
// (clamped to 5).
//
// Safety s: 0.9 for FP64 rays, as the oracle; 0.8 for FP32 rays.  At the
// FP32 path's tolerances (rtol 1e-6 .. 2e-5) the elementary controller at 0.9
// keeps proposing steps just too long while the error constant grows towards
// periapsis (rejected steps had err 1.0-1.5), and about a fifth of all step
// evaluations were rejections; at 0.8 a ray takes ~15% fewer evaluations with
// a smaller error.  At FP64 tolerances 0.9 is the cheaper setting.
template <typename T>
__device__ __forceinline__ float step_factor(float err) {
    // s err^(-1/5) = exp2(log2(s) - log2(err) / 5), s = 0.8 (FP32 rays) or 0.9
    constexpr float log2s = sizeof(T) == 4 ? -0.321928095f : -0.152003093f;
    return __builtin_amdgcn_exp2f(fmaf(-0.2f, __builtin_amdgcn_logf(err), log2s));
}

// max(|a|, |b|), and min(a, b) of two non-negative values, as one
// instruction each.  fmax and fmin in the default IEEE mode also quiet each
// input not known to be canonical, one more instruction per operand every
// step.  In FP32 a v_med3 (against FLT_MAX, respectively 0) avoids that (a
// med3 against +-inf is folded back into fmax/fmin); FP64 has no med3, so
// v_max_f64 / v_min_f64 are written out.  (Inputs here are finite, or NaN in
// a step the error test rejects anyway.)
__device__ __forceinline__ float max_abs(float a, float b) {
    return __builtin_amdgcn_fmed3f(fabsf(a), fabsf(b), 3.40282347e38f);
}
__device__ __forceinline__ double max_abs(double a, double b) {
    double r;
    asm("v_max_f64 %0, |%1|, |%2|" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ float min2(float a, float b) { return __builtin_amdgcn_fmed3f(a, b, 0.0f); }
__device__ __forceinline__ double min2(double a, double b) {
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// ---------------------------------------------------------------------------
// Persistent integrator.
// ---------------------------------------------------------------------------
struct IntegArgs {
    int64_t n;
    const double* u0;         // per-ray u0, or NULL (use u0_uniform)
    double u0_uniform;
    DevScene sc;
    DevTol tol;
    Work w;
    int chunk;
    const BatchConst* bconst; // batch: per-request constants (global), nreq entries
    int nreq;
    BatchConst fc;            // single render: the frame's integrator constants
};

// 1/x in FP64 from the hardware reciprocal estimate and one Newton step
// (relative error ~1e-16; used for the Newton update of the sky crossing).
__device__ __forceinline__ double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }

// Idle lanes a wavefront waits for before it starts new rays come from the
// options (DevTol::refill32 / refill64; defaults 28 and 6).  The FP64
// critical band of FP32 mode, whose rays are long, refills at once.

// Drains one queue.  VIRTUAL: the queue is the index range [0, total) and
// the start records come from rec[id] (w0 = NaN: the ray is not for this
// queue); otherwise queue[] holds ray indices and qrec[] their records.
//
// Each lane keeps the start record of its NEXT ray in registers: the loads
// are issued at a refill (step C, before the step arithmetic) and consumed
// when the lane starts that ray (step A, at a later refill, after its current
// ray has ended).  Positions are handed out per wavefront from a chunk taken
// with one atomic.
//
// The step (B) is a predicated state machine: every lane evaluates one
// Dormand-Prince step per iteration -- a normal trial step, or a Newton
// re-step of the sky crossing -- and all outcomes (accept / reject, disk
// landing, horizon, sky crossing, caps) are applied with selects, so the
// wavefront stays converged except for the store of a finished ray.
//
// A frame's or request's integrator constants in the ray's precision.
template <typename T>
__device__ __forceinline__ void ray_consts(const BatchConst& c, T& s, T& k, T& vh, T& vsky,
                                           T& vrin, T& vrout, T& atol, T& v0) {
    if constexpr (sizeof(T) == 4) {
        s = c.s32, k = c.k32, vh = c.vh32, vsky = c.vsky32;
        vrin = c.vrin32, vrout = c.vrout32, atol = c.atol32, v0 = c.v032;
    } else {
        s = c.s, k = c.k, vh = c.vh, vsky = c.vsky;
        vrin = c.vrin, vrout = c.vrout, atol = c.atol64, v0 = c.v0;
    }
}

__device__ __forceinline__ void ray_consts(const Consts32& c, float& s, float& k, float& vh,
                                           float& vsky, float& vrin, float& vrout, float& atol,
                                           float& v0) {
    s = c.s, k = c.k, vh = c.vh, vsky = c.vsky, vrin = c.vrin, vrout = c.vrout, atol = c.atol;
    v0 = c.v0;
}
__device__ __forceinline__ void ray_consts(const Consts64& c, double& s, double& k, double& vh,
                                           double& vsky, double& vrin, double& vrout,
                                           double& atol, double& v0) {
    s = c.s, k = c.k, vh = c.vh, vsky = c.vsky, vrin = c.vrin, vrout = c.vrout, atol = c.atol;
    v0 = c.v0;
}

// Tolerance factor of an FP32 ray, in [1, grow]: |b - 3 sqrt(3) M| / (0.5 M),
// clamped.  Near the critical impact parameter the sweep's sensitivity to
// integration error grows like 1/|b - b_c|, so a tolerance proportional to
// that distance keeps the exit error about even across rays; the rays next to
// the critical band keep the base tolerance.  b/M from the ray's start: with
// v = 3M u and w = dv/dphi, 9 M^2 / b^2 = w^2 + v^2 - (2/3) v^3 (the first
// integral of Eq. (1)); k = 0 drops the cubic for flat space, where any
// factor in [1, grow] is as good.  The start has v < 1 (outside the photon
// sphere), so the sum is positive.
__device__ __forceinline__ float tol_growth(float v, float w, float k, float grow) {
    const float e = fmaf(w, w, v * v * fmaf(-0.666666667f * k, v, 1.0f));
    const float bm = 3.0f * __builtin_amdgcn_rsqf(e);
    return __builtin_amdgcn_fmed3f(fabsf(bm - 5.19615242f) * 2.0f, 1.0f, grow);
}

template <bool C, typename A, typename B> struct Pick { using type = A; };
template <typename A, typename B> struct Pick<false, A, B> { using type = B; };

// Constants come from a table (`bct`, of type C): one entry in LDS for a
// single frame; with BATCH, rays of several requests share the queue and each
// ray's request index selects its entry (a per-request table in LDS in the
// queue's precision, or the global BatchConst table for the band rays of an
// FP32 batch).
// R32 (FP32 batches and image-only FP32 renders): main-queue start records
// come from a.w.rec32 and result records go to a.w.res32.
// STATS: count accepted, rejected and Newton steps and capped rays into
// the per-call statistics (an instrumented variant; the default one counts
// nothing).
template <typename T, bool VIRTUAL, bool BATCH, bool R32, bool KAPPA, bool STATS = false,
          typename C = BatchConst>
__device__ void run_queue(const IntegArgs& a, const int32_t* __restrict__ queue,
                          const double2* __restrict__ qrec, int64_t total, int32_t* heads,
                          int nslices, T rtol, T ntol, const C* __restrict__ bct,
                          int refill_min, int qblocks) {
    const int lane = lane_id();
    // constants in the scaled variable v = s u (s = 3M; s = 1, k = 0 for
    // M = 0): wave-uniform for one frame, per lane for a batch
    T s, k, vh, vsky, vrin, vrout, atol, pf_v0;
    ray_consts(bct[0], s, k, vh, vsky, vrin, vrout, atol, pf_v0);
    const T h0 = T(sizeof(T) == 4 ? a.tol.h0_32 : a.tol.h0), hmax = T(a.tol.hmax);
    const T max_phi = T(a.tol.max_phi);
    const int max_steps = a.tol.max_steps;
    int pf_rq = 0;
    // the ray's relative tolerance (FP32 rays: rtol times tol_growth, set at
    // the ray's start, atol scaled alike)
    T rt = rtol;

    // ray state
    T v = T(0), w = T(0), g = T(0), h = T(0), hh = T(0);
    // azimuth and the next disk-plane crossing in the ray's precision: FP32
    // rays are shaded from a float azimuth, so a double one would be rounded
    // away at the end (about ten float additions per ray, ~1e-6 rad at most)
    T phi = T(0), phik = T(0);
    int id = 0, attempts = 0, it = 0;
    bool rej = false, refine = false, active = false;
    // prefetched next ray
    int pf_id = 0;
    // (the main queue of an FP32 batch has FP32 start records)
    typename Pick<R32 && VIRTUAL, float2, double2>::type pf{};
    bool pf_valid = false;
    // queue cursor: positions < 2^31 (a render or batch has fewer rays), so
    // 32-bit wave-uniform values that the scalar unit compares
    int cnext = 0, cend = 0;
    bool drained = false;
    int slice = (int)(blockIdx.x % (unsigned)nslices), dry = 0;
    // Single renders: a wavefront's first chunk in its block's slice is
    // assigned without an atomic.  The slice's first chunks go to the
    // wavefronts of its blocks in block order (W of them, qblocks blocks take
    // part in the queue); the head counter hands out chunks W, W + 1, ...
    // (one-frame launches spend a larger share of their time starting up:
    // 3% less per-frame integration; batches measured 1% slower with it)
    constexpr int kWavesPerBlock = kBlock / kWave;
    int first_k = -1;
    if constexpr (!BATCH)
        first_k = __builtin_amdgcn_readfirstlane((int)(blockIdx.x / (unsigned)nslices) * kWavesPerBlock +
                                                 (int)(threadIdx.x >> 6));
    // per-lane statistics over all its rays (STATS only), and the
    // wavefront's queue timeline (main queues of single renders)
    int n_acc = 0, n_rej = 0, n_newt = 0, n_cap = 0;
    unsigned long long t_enter = 0, t_dry = 0;
    if constexpr (STATS && VIRTUAL) t_enter = wall_clock64();

    for (;;) {
        // ---- (A) idle lanes start their prefetched rays, once at least
        // refill_min lanes (1..64) are idle or the queue has run dry: the
        // start and fetch code then runs once for several finished rays
        // instead of on almost every step --------------------------------------
        const bool refill = __popcll(__ballot(!active)) >= refill_min || (drained && cnext >= cend);
        if (refill & !active & pf_valid) {
            pf_valid = false;
            if (!VIRTUAL || pf.x == pf.x) {
                id = pf_id;
                if (BATCH) ray_consts(bct[pf_rq], s, k, vh, vsky, vrin, vrout, atol, pf_v0);
                v = pf_v0;
                w = s * T(pf.x);
                g = g_scaled<KAPPA>(k, v);
                h = h0;
                if constexpr (sizeof(T) == 4) {
                    // the first step grows with the tolerance as the
                    // controller's steps do (local error ~ h^5)
                    const float f = tol_growth(v, w, k, a.tol.grow32);
                    if constexpr (!BATCH) atol = bct[0].atol32;
                    rt = rtol * f;
                    atol *= f;
                    if (f > 1.0f) h = h0 * __builtin_amdgcn_exp2f(0.2f * __builtin_amdgcn_logf(f));
                }
                phi = T(0);
                phik = T(pf.y);
                attempts = 0;
                it = 0;
                rej = false;
                refine = false;
                active = true;
            }
        }
        // ---- (C) lanes without a next ray fetch one (loads not awaited) ----
        const uint64_t need = __ballot(!pf_valid);
        if (need != 0 && !(drained && cnext >= cend)) {
            // Chunk k of slice s covers positions [(k*nslices + s)*chunk, +chunk):
            // the slices interleave over the queue, each with its own head
            // counter (one atomic per chunk; separate counters spread the
            // atomics of the whole chip over several addresses).  A wavefront
            // starts on its block's slice and moves on when a slice is dry.
            while (cnext >= cend && !drained) {
                int k = 0;
                if (first_k >= 0) {
                    k = first_k;
                    first_k = -1;
                } else {
                    if (lane == 0) k = atomicAdd(&heads[slice * kCtrStride], 1);
                    // lane 0's value, read into a scalar register: the chunk
                    // bounds derived from it stay wave-uniform (scalar ALU)
                    k = __builtin_amdgcn_readlane(k, 0);
                    if constexpr (!BATCH) {
                        const int wslice =
                            slice < qblocks ? (qblocks - slice + nslices - 1) / nslices : 0;
                        k += wslice * kWavesPerBlock;
                    }
                }
                const int64_t base = ((int64_t)k * nslices + slice) * a.chunk;
                if (k >= 0 && base < total) {
                    cnext = (int)base;
                    cend = (int)min(base + a.chunk, total);
                } else {
                    slice = slice + 1 == nslices ? 0 : slice + 1;
                    drained = ++dry >= nslices;
                }
            }
            if (cnext < cend) {
                const int rank = rank_in(need);
                const int avail = cend - cnext;
                if (!pf_valid && rank < avail) {
                    const int pos = cnext + rank;
                    pf_id = VIRTUAL ? (int)pos : queue[pos];
                    if constexpr (!VIRTUAL) pf = qrec[pos];
                    else if constexpr (R32) pf = a.w.rec32[pos];
                    else pf = a.w.rec[pos];
                    if (BATCH) pf_rq = a.w.rq[pf_id];
                    else if (a.u0) pf_v0 = T(bct[0].s * a.u0[pf_id]);
                    pf_valid = true;
                }
                cnext += min((int)__popcll(need), avail);
            }
        }
        // Done when no lane has a ray or a prefetched one and the queue is
        // dry.  (A wavefront with no active lane otherwise runs one step with
        // every lane masked off, at its start and while the queue drains;
        // the loop keeps a single back edge.)
        if constexpr (STATS && VIRTUAL) {
            if (drained && t_dry == 0) t_dry = wall_clock64();
        }
        if (drained && cnext >= cend && __ballot(active || pf_valid) == 0) {
            if constexpr (STATS && VIRTUAL) {
                const int wid = (int)(blockIdx.x * (kBlock / kWave) + (threadIdx.x >> 6));
                if (a.w.tl && wid < a.w.tl_waves && lane == 0) {
                    a.w.tl[3 * wid] = t_enter;
                    a.w.tl[3 * wid + 1] = t_dry;
                    a.w.tl[3 * wid + 2] = wall_clock64();
                }
            }
            if constexpr (STATS) {
                // one atomic per counter and wavefront
                unsigned long long* st =
                    reinterpret_cast<unsigned long long*>(a.w.ctr + kCtrStats) + (sizeof(T) == 4 ? 4 : 0);
                const int c4[4] = {n_acc, n_rej, n_newt, n_cap};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    int x = c4[q];
#pragma unroll
                    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
                    if (lane == 0 && x) atomicAdd(&st[q], (unsigned long long)x);
                }
            }
            break;
        }

        // ---- (B) one step evaluation per lane ------------------------------
        const bool nrm = active & !refine;            // normal trial step
        const bool capped = nrm & (attempts >= max_steps);
        const T hx = refine ? hh : h;
        // A trial step that would pass the next disk-plane crossing is
        // shortened to land on it exactly.
        const T phx = phi + hx;
        const bool land = nrm & (phx >= phik);
        const T ht = land ? phik - phi : hx;
        T vn, wn, gn, eu, ew;
        dp45<T>([k](T x) { return g_scaled<KAPPA>(k, x); }, v, w, g, ht, vn, wn, gn, eu, ew);

        // Error test: accept iff |e_i| <= atol + rtol max(|y_i|, |y_new_i|)
        // for both components (exact comparison); the ratio for the step-size
        // proposal needs one reciprocal.
        const T su = fma(rt, max_abs(v, vn), atol);
        const T sw = fma(rt, max_abs(w, wn), atol);
        const bool fits = (fabs(eu) <= su) & (fabs(ew) <= sw);
        const float fsu = (float)su, fsw = (float)sw;
        // |e| fs = |e fs| (fs > 0, rounding is sign-symmetric): the absolute
        // values ride on the max as operand modifiers.
        const float err = fmaxf(fabsf((float)eu * fsw), fabsf((float)ew * fsu)) *
                          __builtin_amdgcn_rcpf(fsu * fsw);
        const float fac = step_factor<T>(err);
        const bool go = nrm & !capped;               // a trial step was taken
        const bool acc = go & fits;
        // Factor of the next trial step: fac clamped to [0.2, 5] after an
        // accepted step ([0.2, 1] right after a rejection) and to [0.2, inf)
        // after a rejected one, as one med3 with its upper bound selected (a
        // NaN fac, from a step the error test rejected, gives 0.2).
        const float fcap = acc ? (rej ? 1.0f : 5.0f) : __builtin_inff();
        const float f = __builtin_amdgcn_fmed3f(fac, 0.2f, fcap);

        // Events of an accepted step, in order: disk, horizon, sky sphere.
        const T phin = land ? phik : phx;
        const bool disk_hit = acc & land & (vn >= vrout) & (vn <= vrin);
        // Horizon: u >= 1/(2M) is v >= 3/2, exact in either precision (+inf
        // for M = 0).
        const bool capture = acc & !disk_hit & (vn >= vh);
        const bool skyx = acc & !disk_hit & !capture & (vn <= vsky) & (wn < T(0));
        const bool advance = acc & !disk_hit & !capture & !skyx;
        // Newton on the step length for v(h) = v_sky (u = u_sky), redoing the
        // step from the last accepted state: h <- h - (v(h) - v_sky) / v'(h).
        // The accepted crossing step gives the first update; each refinement
        // step gives one more (at most four updates).
        const bool newton = (active & refine) | skyx;
        if constexpr (STATS) {
            n_acc += acc ? 1 : 0;
            n_rej += (go & !fits) ? 1 : 0;
            n_newt += (active & refine) ? 1 : 0;
        }
        const T dh = (vn - vsky) * recip(wn);
        const T hh_new = ht - dh;
        // (it is 0 until a ray's first sky crossing: set at the ray's start,
        // changed only by Newton updates, and a ray in refinement ends there)
        const int it_new = it + 1;
        const bool sky_done = newton & ((fabs(dh) < ntol) | (it_new >= 4));
        const bool over = advance & (phin > max_phi);

        // State updates.
        if (go) {
            ++attempts;
            h = min2((acc & land) ? h : ht * T(f), hmax);
            rej = !acc;
        }
        if (acc & land & !disk_hit) phik += T(kPi);
        if (advance) {
            v = vn;
            w = wn;
            g = gn;
            phi = phin;
        }
        if (newton) {
            hh = hh_new;
            it = it_new;
            refine = !sky_done;
        }

        // A finished ray stores its result record.
        if (capped | disk_hit | capture | sky_done | over) {
            if constexpr (STATS) n_cap += (capped | over) ? 1 : 0;
            const uint8_t cls = (capped | over) ? UNRESOLVED
                                : disk_hit       ? DISK
                                : capture        ? CAPTURED
                                                 : SKY;
            const double pe = (double)(sky_done ? phi + hh_new : (capped ? phi : phin));
            // r = 1/u = s/v from the reciprocal: the hardware estimate for FP32
            // rays (1 ulp), refined by one Newton step for FP64 rays (the
            // step squares the estimate's relative error, which leaves it far
            // below their integration error; an IEEE division here cost
            // about ten instructions in the block every finishing ray runs)
            const double rh = !disk_hit ? 0.0 : (double)(s * recip(vn));
            if (R32) a.w.res32[id] = make_float2((float)pe, rec32_radius(cls, (float)rh));
            else a.w.res[id] = make_double2(pe, rh);
            // Step evaluations: the trial steps, plus the Newton re-steps of a
            // sky crossing (a ray in refinement ends only there; its last
            // update is the it_new-th, the first came from the trial step).
            // FP32 records carry the class, and only statistics runs read the
            // counts then.
            if (!R32 || STATS) {
                const int nsteps = attempts + (sky_done ? it_new - 1 : 0);
                a.w.clst[id] = (int32_t)cls | (nsteps << 3);
            }
            active = false;
        }
    }
}

// Stages the integrator constants in LDS: a single frame's constants, or a
// batch's per-request table in one precision (C = Consts32 or Consts64; the
// launch gives the kernel sizeof(C) bytes of LDS per request).  A single
// frame's constants are read back from LDS, so the loop holds them in vector
// registers; taken from the kernel arguments they would sit in scalar
// registers, which the FP32 loop would then spill.
__device__ __forceinline__ const BatchConst* stage_frame_consts(const IntegArgs& a) {
    __shared__ BatchConst s_fc;
    if (threadIdx.x == 0) s_fc = a.fc;
    __syncthreads();
    return &s_fc;
}

template <typename C>
__device__ __forceinline__ const C* stage_batch_consts(const IntegArgs& a) {
    extern __shared__ __align__(8) char s_tab[];
    C* t = reinterpret_cast<C*>(s_tab);
    for (int r = threadIdx.x; r < a.nreq; r += blockDim.x) {
        const BatchConst& c = a.bconst[r];
        if constexpr (sizeof(C) == sizeof(Consts32))
            t[r] = C{c.s32, c.k32, c.vh32, c.vsky32, c.vrin32, c.vrout32, c.atol32, c.v032};
        else
            t[r] = C{c.s, c.k, c.vh, c.vsky, c.vrin, c.vrout, c.atol64, c.v0};
    }
    __syncthreads();
    return t;
}

// FP64 mode: one pass over all rays tagged FP64.  KAPPA: some ray's scene
// is flat (M = 0), so g keeps its factor k.
template <bool BATCH, bool KAPPA, bool STATS = false>
__device__ __forceinline__ void integrate_fp64(const IntegArgs& a) {
    if constexpr (BATCH) {
        const Consts64* bct = stage_batch_consts<Consts64>(a);
        run_queue<double, true, BATCH, false, KAPPA, STATS>(a, nullptr, nullptr, a.n,
                                                     &a.w.ctr[kCtrMain], kSlices, a.tol.rtol64,
                                                     a.tol.newton64, bct, a.tol.refill64,
                                                     (int)gridDim.x);
    } else {
        const BatchConst* bct = stage_frame_consts(a);
        run_queue<double, true, BATCH, false, KAPPA, STATS>(a, nullptr, nullptr, a.n,
                                                     &a.w.ctr[kCtrMain], kSlices, a.tol.rtol64,
                                                     a.tol.newton64, bct, a.tol.refill64,
                                                     (int)gridDim.x);
    }
}

// FP32 mode (batches keep FP32 records).  The first `band_blocks` blocks
// first drain the FP64 queue of the critical band, then join the FP32 rays.
// Band rays are few but long (up to a few hundred FP64 steps) and
// latency-bound; their waves start with the launch and run at raised issue
// priority, so the FP32 waves sharing their SIMDs fill the gaps and the band
// ends inside the FP32 work instead of trailing it.
template <bool BATCH, bool R32, bool KAPPA, bool STATS = false>
__device__ __forceinline__ void integrate_fp32(const IntegArgs& a, int band_blocks) {
    // A batch stages its FP32 constants in LDS; its band rays, a fraction of
    // a percent, read their FP64 constants from the global table at each
    // start.  A single frame's constants sit in LDS for both.
    const BatchConst* fc = nullptr;
    const Consts32* t32 = nullptr;
    if constexpr (BATCH) t32 = stage_batch_consts<Consts32>(a);
    else fc = stage_frame_consts(a);
    if ((int)blockIdx.x < band_blocks) {
        __builtin_amdgcn_s_setprio(3);
        IntegArgs ab = a;
        ab.chunk = 64;
        run_queue<double, false, BATCH, R32, KAPPA, STATS>(ab, a.w.q64, a.w.q64rec,
                                                      a.w.ctr[kCtrBandSize], &a.w.ctr[kCtrBand], 1,
                                                      a.tol.rtol64, a.tol.newton64,
                                                      BATCH ? a.bconst : fc, 1, band_blocks);
        __builtin_amdgcn_s_setprio(0);
    }
    if constexpr (BATCH)
        run_queue<float, true, BATCH, R32, KAPPA, STATS, Consts32>(
            a, nullptr, nullptr, a.n, &a.w.ctr[kCtrMain], kSlices, a.tol.rtol32, a.tol.newton32,
            t32, a.tol.refill32, (int)gridDim.x);
    else
        run_queue<float, true, BATCH, R32, KAPPA, STATS>(
            a, nullptr, nullptr, a.n, &a.w.ctr[kCtrMain], kSlices, a.tol.rtol32, a.tol.newton32,
            fc, a.tol.refill32, (int)gridDim.x);
}

template <bool KAPPA, bool STATS>
__global__ __launch_bounds__(kBlock) void k_integrate_fp64(IntegArgs a) {
    integrate_fp64<false, KAPPA, STATS>(a);
}

// Held to 64 VGPRs (8 waves per SIMD for the FP32 rays); the FP64 band code
// spills a few registers, which only band waves pay.
template <bool KAPPA, bool STATS, bool R32>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8))) void
k_integrate_fp32(IntegArgs a, int band_blocks) {
    integrate_fp32<false, R32, KAPPA, STATS>(a, band_blocks);
}

// Batch kernels: per-request constants come from LDS.
template <bool KAPPA>
__global__ __launch_bounds__(kBlock) void k_integrate_fp64_batch(IntegArgs a) {
    integrate_fp64<true, KAPPA>(a);
}

template <bool KAPPA>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8))) void
k_integrate_fp32_batch(IntegArgs a, int band_blocks) {
    integrate_fp32<true, true, KAPPA>(a, band_blocks);
}

// ---------------------------------------------------------------------------
// The paper's fixed-step mode (FP64).  The ray is followed as a sequence of
// points about eps apart: from (u, w, phi) the azimuth advances by the angle
// a straight segment of length eps along the ray's current direction
// (radial and tangential components proportional to (-w, u)) subtends at the
// hole, dphi = atan2(eps u^2, sqrt(u^2 + w^2) - eps u w), with one
// Dormand-Prince step and no error control.  Scene hits are found on the
// straight chord between consecutive points (in-plane coordinates
// x = r cos phi, y = r sin phi): the disk plane where the height, which is
// proportional to r sin(phi_1 - phi), changes sign (a hit if the chord point
// lies within [r_in, r_out]); the horizon when the new point is inside
// r = 2M; the sky sphere where the chord reaches r_sky.  One thread per ray
// (rays take hundreds to thousands of steps; neighbouring pixels take about
// as many).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_integrate_paper(IntegArgs a, double eps) {
    const double M = a.sc.M, M3 = 3.0 * a.sc.M, u_sky = a.sc.u_sky;
    const double R = a.sc.r_sky;
    const auto gu = [M3](double x) { return g_of(M3, x); };
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < a.n;
         i += (int64_t)gridDim.x * kBlock) {
        const double2 rec = a.w.rec[i];
        if (!(rec.x == rec.x)) continue;  // finished at set-up
        const double phi1 = rec.y;
        const bool disk_on = a.sc.has_disk && phi1 < 1e300;
        double u = a.u0 ? a.u0[i] : a.u0_uniform, w = rec.x, g = g_of(M3, u), phi = 0.0;
        double x = 1.0 / u, y = 0.0, z = disk_on ? x * sin(phi1) : 0.0;
        int steps = 0;
        uint8_t cls = UNRESOLVED;
        double pe = 0.0, rh = 0.0;
        for (;;) {
            if (steps >= a.tol.max_steps || phi > a.tol.max_phi) {
                pe = phi;
                break;
            }
            const double h = atan2(eps * u * u, sqrt(fma(u, u, w * w)) - eps * u * w);
            double un, wn, gn, eu, ew;
            dp45<double>(gu, u, w, g, h, un, wn, gn, eu, ew);
            ++steps;
            const double phin = phi + h;
            const double rn = un > 0.0 ? 1.0 / un : 1e300;
            double sn, cn;
            sincos(phin, &sn, &cn);
            const double xn = rn * cn, yn = rn * sn;
            const double zn = disk_on ? rn * sin(phi1 - phin) : 0.0;
            if (disk_on && ((z < 0.0 && zn >= 0.0) || (z > 0.0 && zn <= 0.0))) {
                const double t = z / (z - zn);
                const double qx = fma(t, xn - x, x), qy = fma(t, yn - y, y);
                const double rq = sqrt(fma(qx, qx, qy * qy));
                if (rq >= a.sc.rin && rq <= a.sc.rout) {
                    cls = DISK;
                    rh = rq;
                    pe = phi + atan2(x * qy - y * qx, fma(x, qx, y * qy));
                    break;
                }
            }
            if (M > 0.0 && 2.0 * M * un >= 1.0) {
                cls = CAPTURED;
                pe = phin;
                break;
            }
            if (un <= u_sky) {
                const double dx = xn - x, dy = yn - y;
                const double qa = fma(dx, dx, dy * dy), qb = 2.0 * fma(x, dx, y * dy);
                const double qc = fma(x, x, y * y) - R * R;
                const double t = (-qb + sqrt(fma(qb, qb, -4.0 * qa * qc))) / (2.0 * qa);
                const double qx = fma(t, dx, x), qy = fma(t, dy, y);
                cls = SKY;
                pe = phi + atan2(x * qy - y * qx, fma(x, qx, y * qy));
                break;
            }
            u = un;
            w = wn;
            g = gn;
            phi = phin;
            x = xn;
            y = yn;
            z = zn;
        }
        a.w.res[i] = make_double2(pe, rh);
        a.w.clst[i] = (int32_t)cls | (steps << 3);
    }
}

// ---------------------------------------------------------------------------
// Shading and output.
// ---------------------------------------------------------------------------
// Mapping back to 3-D and shading of workspace ray i; px (may be NULL)
// receives the RGBA value, out[oi] the per-ray record.  The FP32 path's rays
// are mapped and shaded in FP32 (their error budget is 1e-4 rad), the FP64
// path's in FP64.
//
// The FP32 path's mapping back to 3-D, all in FP32: the plane basis, then the
// exit vector and the shading.  (For an explicit direction the basis is a
// projection: a ray whose sin(angle to e1) is s has e2 good to ~1e-7/s; rays
// with s below ~1e-3 fall in near the axis, where sin(phi_end) is as small.)
struct Basis32 {
    float e1[3], e2[3];
};

__device__ __forceinline__ Basis32 basis32(const float e1[3], const float dv[3]) {
    Basis32 B;
    const float dn2 = dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2];
    const float id = dn2 > 0.0f ? __builtin_amdgcn_rsqf(dn2) : 0.0f;
    float v[3];
    float c = 0.0f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        B.e1[k] = e1[k];
        c = fmaf(dv[k] * id, e1[k], c);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = fmaf(-c, e1[k], dv[k] * id);
    const float s2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    const float is = s2 > 1e-30f ? __builtin_amdgcn_rsqf(s2) : 0.0f;
#pragma unroll
    for (int k = 0; k < 3; ++k) B.e2[k] = v[k] * is;
    return B;
}

// Camera pixel i: the closed form of camera_basis in FP32 (e2 good to a few
// ulp for every pixel).
__device__ __forceinline__ Basis32 camera_basis32(const DevCam& cam, int64_t i) {
    double px, py;
    pixel_of(cam, i, px, py);
    const float x = fmaf((float)px + 0.5f, cam.f_ax, cam.f_bx);
    const float y = fmaf(-((float)py + 0.5f), cam.f_ax, cam.f_tan_half);
    const float s2 = fmaf(x, x, y * y);
    const float iv = s2 > 1e-30f ? __builtin_amdgcn_rsqf(s2) : 0.0f;
    Basis32 B;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        B.e1[k] = cam.f_e1[k];
        B.e2[k] = fmaf(x, cam.f_right[k], y * cam.f_up[k]) * iv;
    }
    return B;
}

__device__ __forceinline__ Basis32 source_basis32(const Source& src, int64_t i) {
    float e1[3], dv[3];
    if (src.origin) {
        float o[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            o[k] = (float)src.origin[3 * i + k];
            dv[k] = (float)src.dir[3 * i + k];
        }
        const float ro2 = o[0] * o[0] + o[1] * o[1] + o[2] * o[2];
        const float ir = ro2 > 0.0f ? __builtin_amdgcn_rsqf(ro2) : 0.0f;
#pragma unroll
        for (int k = 0; k < 3; ++k) e1[k] = o[k] * ir;
        return basis32(e1, dv);
    }
    return camera_basis32(src.cam, i);
}

// Bilinear sample of the sky image at (theta, varphi): texel centres at
// integer continuous coordinates u = varphi tex_w / (2 pi) - 1/2,
// v = theta tex_h / pi - 1/2; columns wrap, rows clamp.  FP32 and FP64 forms.
__device__ __forceinline__ float4 sky_texel32(const DevScene& sc, float theta, float varphi) {
    const int W = sc.tex_w, H = sc.tex_h;
    const float u = fmaf(varphi, (float)sc.tex_su, -0.5f);
    const float v = fmaf(theta, (float)sc.tex_sv, -0.5f);
    const float uf = floorf(u), vf = floorf(v);
    const float fu = u - uf, fv = v - vf;
    int i0 = (int)uf % W;
    if (i0 < 0) i0 += W;
    const int i1 = i0 + 1 == W ? 0 : i0 + 1;
    const int j0 = min(max((int)vf, 0), H - 1), j1 = min(max((int)vf + 1, 0), H - 1);
    const float4 a = sc.tex[(int64_t)j0 * W + i0], b = sc.tex[(int64_t)j0 * W + i1];
    const float4 c = sc.tex[(int64_t)j1 * W + i0], d = sc.tex[(int64_t)j1 * W + i1];
    auto lerp2 = [fu, fv](float p, float q, float r, float t) {
        return fmaf(fv, fmaf(fu, t - r, r) - fmaf(fu, q - p, p), fmaf(fu, q - p, p));
    };
    return make_float4(lerp2(a.x, b.x, c.x, d.x), lerp2(a.y, b.y, c.y, d.y),
                       lerp2(a.z, b.z, c.z, d.z), lerp2(a.w, b.w, c.w, d.w));
}

__device__ __forceinline__ float4 sky_texel64(const DevScene& sc, double theta, double varphi) {
    const int W = sc.tex_w, H = sc.tex_h;
    const double u = fma(varphi, sc.tex_su, -0.5);
    const double v = fma(theta, sc.tex_sv, -0.5);
    const double uf = floor(u), vf = floor(v);
    const double fu = u - uf, fv = v - vf;
    int64_t i0 = (int64_t)uf % W;
    if (i0 < 0) i0 += W;
    const int64_t i1 = i0 + 1 == W ? 0 : i0 + 1;
    const int64_t j0 = min(max((int64_t)vf, (int64_t)0), (int64_t)H - 1);
    const int64_t j1 = min(max((int64_t)vf + 1, (int64_t)0), (int64_t)H - 1);
    const float4 a = sc.tex[j0 * W + i0], b = sc.tex[j0 * W + i1];
    const float4 c = sc.tex[j1 * W + i0], d = sc.tex[j1 * W + i1];
    auto lerp2 = [fu, fv](double p, double q, double r, double t) {
        const double top = fma(fu, q - p, p), bot = fma(fu, t - r, r);
        return (float)fma(fv, bot - top, top);
    };
    return make_float4(lerp2(a.x, b.x, c.x, d.x), lerp2(a.y, b.y, c.y, d.y),
                       lerp2(a.z, b.z, c.z, d.z), lerp2(a.w, b.w, c.w, d.w));
}

// phi and r_hit come in as floats: the same values whether the record was
// kept in FP64 (single renders) or FP32 (batches), so both shade alike.
__device__ __forceinline__ float4 shade_px32(const Basis32& B, const DevScene& sc, uint8_t cls,
                                             float phi, float r_hit, float sv[3]) {
    float sf, cf;
    sincosf(phi, &sf, &cf);
#pragma unroll
    for (int k = 0; k < 3; ++k) sv[k] = fmaf(cf, B.e1[k], sf * B.e2[k]);
    if (cls == INVALID) sv[0] = sv[1] = sv[2] = 0.0f;
    float4 px = make_float4(0.f, 0.f, 0.f, 1.f);
    if (cls == SKY) {
        const float theta = atan2f(sqrtf(fmaf(sv[0], sv[0], sv[1] * sv[1])), sv[2]);
        float varphi = atan2f(sv[1], sv[0]);
        if (varphi < 0.0f) varphi += 6.28318531f;
        if (sc.tex) {
            px = sky_texel32(sc, theta, varphi);
        } else {
            const float icell = (float)sc.inv_cell;
            const int parity = ((int)floorf(theta * icell) + (int)floorf(varphi * icell)) & 1;
            const float g = parity ? 0.1f : 1.0f;
            px = make_float4(g, g, g, 1.f);
        }
    } else if (cls == DISK) {
        const float I = powf(r_hit * (float)sc.urin, (float)sc.power);
        px = make_float4(I, 0.6f * I, 0.2f * I, 1.f);
    }
    return px;
}

// R32: the record, class included, is read from w.res32 (FP32 batches and
// image-only FP32 renders, which return no per-ray outputs).
template <bool R32 = false>
__device__ __forceinline__ void shade_ray32(const Basis32& B, const DevScene& sc, const Work& w,
                                            int64_t i, float4* px_out, const Out& out,
                                            int64_t oi) {
    const int32_t cs = R32 ? 0 : w.clst[i];
    const double2 rr = R32 ? make_double2(0.0, 0.0) : w.res[i];
    const float2 rf = R32 ? w.res32[i] : make_float2((float)rr.x, (float)rr.y);
    const uint8_t cls = R32 ? rec32_class(rf.y) : (uint8_t)(cs & 7);
    float sv[3];
    const float4 px = shade_px32(B, sc, cls, rf.x, rf.y, sv);
    if (px_out) *px_out = px;
    if (out.cls) out.cls[oi] = cls;
    if (out.phi_end) out.phi_end[oi] = rr.x;
    if (out.r_hit) out.r_hit[oi] = rr.y;
    if (out.steps) out.steps[oi] = cs >> 3;
    if (out.path) out.path[oi] = w.path[i];
    if (out.exit_dir) {
#pragma unroll
        for (int k = 0; k < 3; ++k) out.exit_dir[3 * oi + k] = sv[k];
    }
}

__device__ __forceinline__ void shade_ray(const Basis& B, const DevScene& sc, const Work& w,
                                          int64_t i, float4* px_out, const Out& out, int64_t oi) {
    const int32_t cs = w.clst[i];
    const uint8_t cls = (uint8_t)(cs & 7);
    const double2 rr = w.res[i];
    const double phi = rr.x;
    const double r_hit = rr.y;
    double s[3];
    float4 px = make_float4(0.f, 0.f, 0.f, 1.f);
    double sphi, cphi;
    sincos(phi, &sphi, &cphi);
#pragma unroll
    for (int k = 0; k < 3; ++k) s[k] = cphi * B.e1[k] + sphi * B.e2[k];
    if (cls == INVALID) s[0] = s[1] = s[2] = 0.0;
    if (cls == SKY) {
        const double theta = atan2(hypot(s[0], s[1]), s[2]);
        double varphi = atan2(s[1], s[0]);
        if (varphi < 0.0) varphi += 2.0 * kPi;
        if (sc.tex) {
            px = sky_texel64(sc, theta, varphi);
        } else {
            const long parity =
                ((long)floor(theta * sc.inv_cell) + (long)floor(varphi * sc.inv_cell)) & 1L;
            const float g = parity ? 0.1f : 1.0f;
            px = make_float4(g, g, g, 1.f);
        }
    } else if (cls == DISK) {
        const double I = pow(r_hit / sc.rin, sc.power);
        px = make_float4((float)I, (float)(0.6 * I), (float)(0.2 * I), 1.f);
    }
    if (px_out) *px_out = px;
    if (out.cls) out.cls[oi] = cls;
    if (out.phi_end) out.phi_end[oi] = phi;
    if (out.r_hit) out.r_hit[oi] = r_hit;
    if (out.steps) out.steps[oi] = cs >> 3;
    if (out.path) out.path[oi] = w.path[i];
    if (out.exit_dir) {
#pragma unroll
        for (int k = 0; k < 3; ++k) out.exit_dir[3 * oi + k] = s[k];
    }
}

// R32 (with F32): the result records are FP32 (w.res32).
template <bool F32, bool R32 = false>
__global__ __launch_bounds__(kBlock) void k_shade(Source src, DevScene sc, Work w, float* rgba,
                                                  Out out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= src.n) return;
    float4* px = rgba ? reinterpret_cast<float4*>(rgba) + i : nullptr;
    if (F32) shade_ray32<R32>(source_basis32(src, i), sc, w, i, px, out, i);
    else shade_ray(source_basis(src, i, sc.M, sc.r_sky), sc, w, i, px, out, i);
}

// Batch shading: each pixel goes to its request's image.  A block shades
// chunks of kShadeChunk consecutive rays; after each chunk one thread adds the
// chunk's pixels to the completion counter of every request it overlaps, and
// the addition that completes a request records the device clock as its
// finish time (one atomic per chunk and request, so the counters of large
// requests are not contended).
constexpr int kShadeChunk = 32 * kBlock;
// Blocks per CU of batch shading.  On the 16 4K orbit frames (FP32: 8 B of
// records read and 16 B of image written per ray) 6 shaded in 0.69-0.71 ms,
// 4 in 0.83, 5 in 0.76 and 7 (the occupancy limit at 71 VGPRs) in 0.82.
constexpr int kShadeBlocksPerCu = 6;

template <bool F32>
__global__ __launch_bounds__(kBlock) void k_shade_batch(BatchDev b, Work w) {
    extern __shared__ int64_t s_off[];
    stage_offsets(b, s_off);
    const int64_t nchunks = (b.total + kShadeChunk - 1) / kShadeChunk;
    for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const int64_t c0 = c * kShadeChunk, c1 = min(c0 + kShadeChunk, b.total);
        const int rc = __builtin_amdgcn_readfirstlane(find_req(s_off, b.nreq, c0));
        if (s_off[rc + 1] >= c1) {
            // the chunk lies in one request: its constants as uniform values
            const ReqDev q = uniform_load(b.req + rc);
            const int64_t base = s_off[rc];
            float4* img = reinterpret_cast<float4*>(q.rgba);
            for (int64_t g = c0 + threadIdx.x; g < c1; g += kBlock) {
                const int64_t i = g - base;
                if (F32) shade_ray32<true>(camera_basis32(q.cam, i), q.sc, w, g, img + i, Out{}, 0);
                else shade_ray(camera_basis(q.cam, i, q.sc.M, q.sc.r_sky), q.sc, w, g, img + i, Out{}, 0);
            }
        } else {
            for (int64_t g = c0 + threadIdx.x; g < c1; g += kBlock) {
                const int r = find_req(s_off, b.nreq, g);
                const ReqDev& q = b.req[r];
                const int64_t i = g - s_off[r];
                float4* px = reinterpret_cast<float4*>(q.rgba) + i;
                if (F32) shade_ray32<true>(camera_basis32(q.cam, i), q.sc, w, g, px, Out{}, 0);
                else shade_ray(camera_basis(q.cam, i, q.sc.M, q.sc.r_sky), q.sc, w, g, px, Out{}, 0);
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int r = rc; r < b.nreq && s_off[r] < c1; ++r) {
                const int64_t lo = max(c0, s_off[r]), hi = min(c1, s_off[r + 1]);
                if (hi <= lo) continue;
                const unsigned long long cnt = (unsigned long long)(hi - lo);
                const unsigned long long total = (unsigned long long)(s_off[r + 1] - s_off[r]);
                if (atomicAdd(&b.done[r], cnt) + cnt == total) b.stamp[r] = wall_clock64();
            }
        }
    }
}

// n x n samples per pixel: src is the (n W) x (n H) sample camera; thread
// (x, y) shades its pixel's n*n samples in a fixed order and writes their mean
// to the W x H image (per-ray records go to the sample index).
template <bool F32>
__global__ __launch_bounds__(kBlock) void k_shade_samples(Source src, DevScene sc, Work w,
                                                          float* rgba, Out out, int n) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int Wn = src.cam.W, W = Wn / n;
    const int64_t npx = src.n / ((int64_t)n * n);
    if (p >= npx) return;
    const int64_t y = p / W, x = p - y * W;
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int j = 0; j < n; ++j) {
        for (int i = 0; i < n; ++i) {
            const int64_t q = (y * n + j) * Wn + (x * n + i);
            float4 c;
            if (F32) shade_ray32(source_basis32(src, q), sc, w, q, &c, out, q);
            else shade_ray(source_basis(src, q, sc.M, sc.r_sky), sc, w, q, &c, out, q);
            acc.x += c.x;
            acc.y += c.y;
            acc.z += c.z;
            acc.w += c.w;
        }
    }
    const float inv = 1.0f / (float)(n * n);
    reinterpret_cast<float4*>(rgba)[p] = make_float4(acc.x * inv, acc.y * inv, acc.z * inv,
                                                     acc.w * inv);
}

// Per-call statistics of the last single render or trace: out[0..4] rays per
// class, out[5..8] rays per path, out[9] summed step evaluations.
__global__ __launch_bounds__(kBlock) void k_stats(int64_t n, const int32_t* __restrict__ clst,
                                                  const uint8_t* __restrict__ path,
                                                  unsigned long long* out) {
    __shared__ unsigned long long c[10];
    if (threadIdx.x < 10) c[threadIdx.x] = 0;
    __syncthreads();
    unsigned long long steps = 0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const int32_t cs = clst[i];
        const uint8_t p = path[i];
        const int cl = cs & 7;
        atomicAdd(&c[cl < 5 ? cl : 4], 1ull);
        if (p < 4) atomicAdd(&c[5 + p], 1ull);
        steps += (unsigned long long)(uint32_t)cs >> 3;
    }
    atomicAdd(&c[9], steps);
    __syncthreads();
    if (threadIdx.x < 10) atomicAdd(&out[threadIdx.x], c[threadIdx.x]);
}

// Batch start time and completion counters.
__global__ void k_batch_begin(BatchDev b) {
    for (int r = threadIdx.x; r < b.nreq; r += blockDim.x) b.done[r] = 0;
    if (threadIdx.x == 0) b.stamp[b.nreq] = wall_clock64();
}

__global__ __launch_bounds__(kBlock) void k_count_paths(int64_t n, const uint8_t* path,
                                                        unsigned long long* counts) {
    __shared__ unsigned int c[4];
    if (threadIdx.x < 4) c[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const uint8_t p = path[i];
        if (p < 4) atomicAdd(&c[p], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 4) atomicAdd(&counts[threadIdx.x], (unsigned long long)c[threadIdx.x]);
}

// ---------------------------------------------------------------------------
// Launch helpers
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

hipError_t launch_reset(int32_t* ctr, hipStream_t s) {
    k_reset<<<1, 256, 0, s>>>(ctr);
    return hipGetLastError();
}

hipError_t launch_setup(const Source& src, const DevScene& sc, const DevRoute& rt, const Work& w,
                        double* out_b, hipStream_t s) {
    if (src.n == 0) return hipSuccess;
    if (w.rec32) k_setup<true><<<blocks_for(src.n), kBlock, 0, s>>>(src, sc, rt, w, out_b);
    else k_setup<false><<<blocks_for(src.n), kBlock, 0, s>>>(src, sc, rt, w, out_b);
    return hipGetLastError();
}

// Resident blocks per CU of a kernel (queried once).
template <typename K>
static int blocks_per_cu(K kernel, int* cache) {
    if (*cache == 0) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, kBlock, 0) != hipSuccess ||
            nb < 1)
            nb = 1;
        *cache = nb;
    }
    return *cache;
}

// Resident blocks per CU of a kernel with `lds` bytes of dynamic LDS (the
// batch kernels' LDS grows with the number of requests).
template <typename K>
static int blocks_per_cu_lds(K kernel, size_t lds) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, kBlock, lds) != hipSuccess ||
        nb < 1)
        nb = 1;
    return nb;
}

static unsigned persistent_grid(int64_t n, int cus, int per_cu, int grid_blocks) {
    int64_t g = grid_blocks > 0 ? grid_blocks : (int64_t)cus * per_cu;
    const int64_t need = (n + kBlock - 1) / kBlock;
    if (g > need) g = need;
    return (unsigned)(g > 0 ? g : 1);
}

// One-frame launches run on three quarters of the resident blocks by default:
// on 4K orbit frames 6 resident blocks per CU integrated about 3% (FP32, of 8
// resident) and 1.6% (FP64, of 7) faster than all of them, while the batch
// kernels, one drain for all their requests, measured fastest fully resident
// and keep that.
static int single_render_blocks(int per_cu) { return per_cu > 1 ? per_cu - per_cu / 4 : 1; }

template <bool KAPPA, bool STATS, bool R32>
static void launch_integrate32_k(const IntegArgs& a, int cus, int grid_blocks, hipStream_t s) {
    static int occ = 0;  // per variant
    const int per_cu = blocks_per_cu(k_integrate_fp32<KAPPA, STATS, R32>, &occ);
    const unsigned g = persistent_grid(a.n, cus, single_render_blocks(per_cu), grid_blocks);
    // The first cus/2 blocks serve the frame's FP64 band first: one-frame
    // launches integrated 2.5% faster than with cus/4 (cus and 2 cus measured
    // the same as cus/2, cus/8 9% slower); a batch's band, under the FP32 work
    // of all its requests, measured the same from cus/8 to cus/2 and keeps
    // cus/4.
    const int band_blocks = (int)min((unsigned)(cus >= 2 ? cus / 2 : 1), g);
    k_integrate_fp32<KAPPA, STATS, R32><<<g, kBlock, 0, s>>>(a, band_blocks);
}

// FP32 records (a.w.rec32 set by the caller) or FP64 ones.
template <bool KAPPA, bool STATS>
static void launch_integrate_k(const IntegArgs& a, int precision, int cus, int grid_blocks,
                               hipStream_t s) {
    static int occ64 = 0;  // per variant
    if (precision != 1) {
        const int per_cu = blocks_per_cu(k_integrate_fp64<KAPPA, STATS>, &occ64);
        const unsigned g = persistent_grid(a.n, cus, single_render_blocks(per_cu), grid_blocks);
        k_integrate_fp64<KAPPA, STATS><<<g, kBlock, 0, s>>>(a);
    } else if (a.w.rec32) {
        launch_integrate32_k<KAPPA, STATS, true>(a, cus, grid_blocks, s);
    } else {
        launch_integrate32_k<KAPPA, STATS, false>(a, cus, grid_blocks, s);
    }
}

hipError_t launch_integrate(int64_t n, bool explicit_u0, double u0_uniform, const DevScene& sc,
                            const DevTol& tol, int precision, const Work& w, int cus,
                            int grid_blocks, int chunk, bool stats, hipStream_t s) {
    if (n == 0) return hipSuccess;
    IntegArgs a;
    a.n = n;
    a.u0 = explicit_u0 ? w.u0 : nullptr;
    a.u0_uniform = u0_uniform;
    a.sc = sc;
    a.tol = tol;
    a.w = w;
    a.chunk = chunk;
    a.bconst = nullptr;
    a.nreq = 0;
    a.fc = integ_consts(sc, tol, u0_uniform);
    if (stats) {
        if (sc.M > 0.0) launch_integrate_k<false, true>(a, precision, cus, grid_blocks, s);
        else launch_integrate_k<true, true>(a, precision, cus, grid_blocks, s);
    } else {
        if (sc.M > 0.0) launch_integrate_k<false, false>(a, precision, cus, grid_blocks, s);
        else launch_integrate_k<true, false>(a, precision, cus, grid_blocks, s);
    }
    return hipGetLastError();
}

// Batch start: clears every request's completion counter and stamps the start
// time (b covers all requests).
hipError_t launch_batch_begin(const BatchDev& b, hipStream_t s) {
    k_batch_begin<<<1, 256, 0, s>>>(b);
    return hipGetLastError();
}

// One group of a batch, in three launches: b covers the group's requests
// (offsets relative to the group's first ray) and w its rays.
hipError_t launch_batch_setup(const BatchDev& b, const Work& w, hipStream_t s) {
    k_reset<<<1, 256, 0, s>>>(w.ctr);
    const size_t lds_off = sizeof(int64_t) * (b.nreq + 1);
    if ((w.res32 != nullptr) != (w.rec32 != nullptr)) return hipErrorInvalidValue;
    if (b.total > 0) {
        if (w.res32) k_setup_batch<true><<<blocks_for(b.total), kBlock, lds_off, s>>>(b, w);
        else k_setup_batch<false><<<blocks_for(b.total), kBlock, lds_off, s>>>(b, w);
    }
    return hipGetLastError();
}

template <bool KAPPA>
static void launch_batch_integrate_k(const IntegArgs& a, int64_t total, size_t lds_c,
                                     int precision, int cus, int grid_blocks, hipStream_t s) {
    if (precision != 1) {
        const unsigned g = persistent_grid(
            total, cus, blocks_per_cu_lds(k_integrate_fp64_batch<KAPPA>, lds_c), grid_blocks);
        k_integrate_fp64_batch<KAPPA><<<g, kBlock, lds_c, s>>>(a);
    } else {
        const unsigned g = persistent_grid(
            total, cus, blocks_per_cu_lds(k_integrate_fp32_batch<KAPPA>, lds_c), grid_blocks);
        const int band_blocks = (int)min((unsigned)(cus >= 4 ? cus / 4 : 1), g);
        k_integrate_fp32_batch<KAPPA><<<g, kBlock, lds_c, s>>>(a, band_blocks);
    }
}

hipError_t launch_batch_integrate(const BatchDev& b, const Work& w, const DevTol& tol,
                                  int precision, int cus, int grid_blocks, int chunk,
                                  hipStream_t s) {
    if (b.total == 0) return hipSuccess;
    if (precision == 1 && (!w.res32 || !w.rec32)) return hipErrorInvalidValue;  // FP32 records
    IntegArgs a;
    a.n = b.total;
    a.u0 = nullptr;
    a.u0_uniform = 0.0;
    a.sc = DevScene{};  // read by the fixed-step kernel only; batch rays use their request's
    a.tol = tol;
    a.w = w;
    a.chunk = chunk;
    a.bconst = b.bconst;
    a.nreq = b.nreq;
    a.fc = BatchConst{};  // unused: batch rays take their request's entry
    // per-request constants staged in LDS: the FP32 ones for FP32 batches,
    // the FP64 ones for FP64 batches
    const size_t lds_c = (precision == 1 ? sizeof(Consts32) : sizeof(Consts64)) * b.nreq;
    if (b.any_flat) launch_batch_integrate_k<true>(a, b.total, lds_c, precision, cus, grid_blocks, s);
    else launch_batch_integrate_k<false>(a, b.total, lds_c, precision, cus, grid_blocks, s);
    return hipGetLastError();
}

hipError_t launch_batch_shade(const BatchDev& b, const Work& w, int precision, int cus,
                              hipStream_t s) {
    if (b.total == 0) return hipSuccess;
    if (precision == 1 && !w.res32) return hipErrorInvalidValue;  // FP32 batches: FP32 records
    const size_t lds_off = sizeof(int64_t) * (b.nreq + 1);
    // One round of resident blocks, at most kShadeBlocksPerCu per CU: a grid
    // beyond them would leave a second, partly filled round of blocks at the
    // end.
    const int per_cu = precision == 1 ? blocks_per_cu_lds(k_shade_batch<true>, lds_off)
                                      : blocks_per_cu_lds(k_shade_batch<false>, lds_off);
    const int64_t slots = (int64_t)cus * min(per_cu, kShadeBlocksPerCu);
    int64_t gs = (b.total + kShadeChunk - 1) / kShadeChunk;
    if (gs > slots) gs = slots;
    if (precision == 1) k_shade_batch<true><<<(unsigned)gs, kBlock, lds_off, s>>>(b, w);
    else k_shade_batch<false><<<(unsigned)gs, kBlock, lds_off, s>>>(b, w);
    return hipGetLastError();
}

hipError_t launch_shade(const Source& src, const DevScene& sc, const Work& w, float* rgba,
                        const Out& out, int precision, hipStream_t s) {
    if (src.n == 0) return hipSuccess;
    if (precision == 1 && w.res32)
        k_shade<true, true><<<blocks_for(src.n), kBlock, 0, s>>>(src, sc, w, rgba, out);
    else if (precision == 1)
        k_shade<true><<<blocks_for(src.n), kBlock, 0, s>>>(src, sc, w, rgba, out);
    else k_shade<false><<<blocks_for(src.n), kBlock, 0, s>>>(src, sc, w, rgba, out);
    return hipGetLastError();
}

hipError_t launch_shade_samples(const Source& src, const DevScene& sc, const Work& w, float* rgba,
                                const Out& out, int precision, int n, hipStream_t s) {
    const int64_t npx = src.n / ((int64_t)n * n);
    if (npx == 0) return hipSuccess;
    if (precision == 1) k_shade_samples<true><<<blocks_for(npx), kBlock, 0, s>>>(src, sc, w, rgba, out, n);
    else k_shade_samples<false><<<blocks_for(npx), kBlock, 0, s>>>(src, sc, w, rgba, out, n);
    return hipGetLastError();
}

hipError_t launch_integrate_paper(int64_t n, bool explicit_u0, double u0_uniform,
                                  const DevScene& sc, const DevTol& tol, double eps,
                                  const Work& w, int cus, hipStream_t s) {
    if (n == 0) return hipSuccess;
    IntegArgs a{};
    a.n = n;
    a.u0 = explicit_u0 ? w.u0 : nullptr;
    a.u0_uniform = u0_uniform;
    a.sc = sc;
    a.tol = tol;
    a.w = w;
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g > (int64_t)cus * 16) g = (int64_t)cus * 16;
    k_integrate_paper<<<(unsigned)g, kBlock, 0, s>>>(a, eps);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_zero(unsigned long long* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        p[i] = 0;
}

// Zeroes n 64-bit words with a kernel (not a memset, so a caller may capture it).
hipError_t launch_zero(unsigned long long* p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    unsigned g = blocks_for(n);
    if (g > 1024) g = 1024;
    k_zero<<<g, kBlock, 0, s>>>(p, n);
    return hipGetLastError();
}

hipError_t launch_stats(int64_t n, const Work& w, unsigned long long* out, hipStream_t s) {
    unsigned g = blocks_for(n);
    if (g > 4096) g = 4096;
    if (g == 0) g = 1;
    k_stats<<<g, kBlock, 0, s>>>(n, w.clst, w.path, out);
    return hipGetLastError();
}

hipError_t launch_count_paths(int64_t n, const Work& w, unsigned long long* counts,
                              hipStream_t s) {
    unsigned g = blocks_for(n);
    if (g > 4096) g = 4096;
    if (g == 0) g = 1;
    k_count_paths<<<g, kBlock, 0, s>>>(n, w.path, counts);
    return hipGetLastError();
}

}  // namespace bh
