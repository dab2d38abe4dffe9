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

enum : uint8_t { SKY = 0, CAPTURED = 1, DISK = 2, UNRESOLVED = 3, INVALID = 4 };
enum : uint8_t { PATH_NONE = 0, PATH_FP64 = 1, PATH_FP32 = 2, PATH_SUR = 3 };

constexpr double kPi = 3.14159265358979323846;
constexpr double kBcrit = 5.19615242270663188058;  // 3 sqrt(3)

// ---------------------------------------------------------------------------
// Wave helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ int rank_in(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// ---------------------------------------------------------------------------
// Geometry shared by set-up and shading (identical code, so both stages see
// the same plane basis bit for bit).
// ---------------------------------------------------------------------------
struct Basis {
    double e1[3], e2[3];
    double c, s, r0;
    bool radial, ok;
};

__device__ __forceinline__ void camera_dir(const DevCam& cam, int64_t i, double d[3]) {
    const int px = (int)(i % cam.W), py = (int)(i / cam.W);
    const double W = cam.W, H = cam.H;
    const double x = (2.0 * (px + 0.5) / W - 1.0) * cam.tan_half * W / H;
    const double y = (1.0 - 2.0 * (py + 0.5) / H) * cam.tan_half;
#pragma unroll
    for (int k = 0; k < 3; ++k) d[k] = cam.fwd[k] + x * cam.right[k] + y * cam.up[k];
}

__device__ __forceinline__ Basis plane_basis(const double o[3], const double dv[3], double M,
                                             double r_sky) {
    Basis B;
    B.ok = isfinite(o[0]) && isfinite(o[1]) && isfinite(o[2]) && isfinite(dv[0]) &&
           isfinite(dv[1]) && isfinite(dv[2]);
    const double r0 = sqrt(o[0] * o[0] + o[1] * o[1] + o[2] * o[2]);
    const double dn = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
    B.ok = B.ok && (r0 > 3.0 * M) && (r0 < r_sky) && (dn > 0.0);
    B.r0 = r0;
    const double ir = 1.0 / r0, id = 1.0 / dn;
    double d[3], v[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        B.e1[k] = o[k] * ir;
        d[k] = dv[k] * id;
    }
    B.c = d[0] * B.e1[0] + d[1] * B.e1[1] + d[2] * B.e1[2];
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = d[k] - B.c * B.e1[k];
    B.s = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    B.radial = !(B.s > 1e-15);
    const double is = B.radial ? 0.0 : 1.0 / B.s;
#pragma unroll
    for (int k = 0; k < 3; ++k) B.e2[k] = v[k] * is;
    return B;
}

__device__ __forceinline__ void source_ray(const Source& src, int64_t i, double o[3], double d[3]) {
    if (src.origin) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            o[k] = src.origin[3 * i + k];
            d[k] = src.dir[3 * i + k];
        }
    } else {
#pragma unroll
        for (int k = 0; k < 3; ++k) o[k] = src.cam.pos[k];
        camera_dir(src.cam, i, d);
    }
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

// ---------------------------------------------------------------------------
// Counter reset (a kernel rather than a memset so the sequence can be
// captured in a graph).
// ---------------------------------------------------------------------------
__global__ void k_reset(int32_t* ctr) {
    if (threadIdx.x < 8) ctr[threadIdx.x] = 0;
}

// ---------------------------------------------------------------------------
// Set-up and routing.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_setup(Source src, DevScene sc, DevRoute rt, Work w,
                                                  double* out_b) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool valid = i < src.n;
    bool to_q64 = false;
    if (valid) {
        double o[3], dv[3];
        source_ray(src, i, o, dv);
        const Basis B = plane_basis(o, dv, sc.M, sc.r_sky);
        uint8_t path = PATH_NONE, cls = INVALID;
        double phi_end = 0.0, b = 0.0;
        if (B.ok && B.radial) {
            // Radial ray: inward is captured (flat space: straight through
            // the centre to the antipode); outward escapes along e1.
            if (B.c < 0.0) {
                cls = sc.M > 0.0 ? CAPTURED : SKY;
                phi_end = sc.M > 0.0 ? 0.0 : kPi;
            } else {
                cls = SKY;
            }
        } else if (B.ok) {
            const double u0 = 1.0 / B.r0;
            const double w0 = -u0 * B.c / B.s;
            // First integral of Eq. (1): w^2 + u^2 - 2 M u^3 = 1/b^2.
            const double E0 = w0 * w0 + u0 * u0 - 2.0 * sc.M * u0 * u0 * u0;
            b = 1.0 / sqrt(E0);
            const double bc = kBcrit * sc.M;
            w.w0[i] = w0;
            if (w.u0) w.u0[i] = u0;
            w.phi1[i] = sc.has_disk ? first_crossing(B.e1[2], B.e2[2]) : __builtin_inf();
            if (rt.analytic_capture && !sc.has_disk && B.c < 0.0 && b < bc - rt.band) {
                cls = CAPTURED;  // below the potential peak: falls in, no disk to hit
            } else if (rt.precision == 1 && fabs(b - bc) < rt.band) {
                path = PATH_FP64;
                to_q64 = true;
            } else {
                path = rt.precision == 1 ? PATH_FP32 : PATH_FP64;
            }
        }
        w.path[i] = path;
        if (path == PATH_NONE) {
            w.cls[i] = cls;
            w.phi_end[i] = phi_end;
            w.r_hit[i] = 0.0;
            w.steps[i] = 0;
        }
        if (out_b) out_b[i] = b;
    }
    // Wave-aggregated append to the FP64 band queue: one atomic per wavefront
    // that holds band rays (a fraction of a percent of all wavefronts).
    const uint64_t m = __ballot(to_q64);
    if (m) {
        const int leader = __ffsll((unsigned long long)m) - 1;
        int base = 0;
        if (lane_id() == leader) base = atomicAdd(&w.ctr[0], __popcll(m));
        base = __shfl(base, leader);
        if (to_q64) w.q64[base + rank_in(m)] = (int32_t)i;
    }
}

// ---------------------------------------------------------------------------
// Dormand-Prince 5(4) step for y = (u, w), y' = (w, g(u)), g(u) = u (3 M u - 1).
// First-same-as-last: g1 = g(u) comes in, g7 = g(u_new) goes out.  The u
// component of every stage derivative is the stage's w value, so only g is
// evaluated (6 evaluations per step).
// Tableau: Dormand & Prince (1980); Hairer, Norsett & Wanner, Solving ODEs I,
// Sec. II.5.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T g_of(T M3, T u) {
    return u * fma(M3, u, T(-1));
}

template <typename T>
__device__ __forceinline__ void dp45(T M3, T u, T w, T g1, T h, T& un, T& wn, T& g7, T& eu,
                                     T& ew) {
    constexpr T a21 = T(1.0 / 5.0);
    constexpr T a31 = T(3.0 / 40.0), a32 = T(9.0 / 40.0);
    constexpr T a41 = T(44.0 / 45.0), a42 = T(-56.0 / 15.0), a43 = T(32.0 / 9.0);
    constexpr T a51 = T(19372.0 / 6561.0), a52 = T(-25360.0 / 2187.0),
                a53 = T(64448.0 / 6561.0), a54 = T(-212.0 / 729.0);
    constexpr T a61 = T(9017.0 / 3168.0), a62 = T(-355.0 / 33.0), a63 = T(46732.0 / 5247.0),
                a64 = T(49.0 / 176.0), a65 = T(-5103.0 / 18656.0);
    constexpr T b1 = T(35.0 / 384.0), b3 = T(500.0 / 1113.0), b4 = T(125.0 / 192.0),
                b5 = T(-2187.0 / 6784.0), b6 = T(11.0 / 84.0);
    constexpr T e1 = T(71.0 / 57600.0), e3 = T(-71.0 / 16695.0), e4 = T(71.0 / 1920.0),
                e5 = T(-17253.0 / 339200.0), e6 = T(22.0 / 525.0), e7 = T(-1.0 / 40.0);

    const T w1 = w;
    const T u2 = fma(h, a21 * w1, u);
    const T w2 = fma(h, a21 * g1, w);
    const T g2 = g_of(M3, u2);

    const T u3 = fma(h, fma(a32, w2, a31 * w1), u);
    const T w3 = fma(h, fma(a32, g2, a31 * g1), w);
    const T g3 = g_of(M3, u3);

    const T u4 = fma(h, fma(a43, w3, fma(a42, w2, a41 * w1)), u);
    const T w4 = fma(h, fma(a43, g3, fma(a42, g2, a41 * g1)), w);
    const T g4 = g_of(M3, u4);

    const T u5 = fma(h, fma(a54, w4, fma(a53, w3, fma(a52, w2, a51 * w1))), u);
    const T w5 = fma(h, fma(a54, g4, fma(a53, g3, fma(a52, g2, a51 * g1))), w);
    const T g5 = g_of(M3, u5);

    const T u6 = fma(h, fma(a65, w5, fma(a64, w4, fma(a63, w3, fma(a62, w2, a61 * w1)))), u);
    const T w6 = fma(h, fma(a65, g5, fma(a64, g4, fma(a63, g3, fma(a62, g2, a61 * g1)))), w);
    const T g6 = g_of(M3, u6);

    un = fma(h, fma(b6, w6, fma(b5, w5, fma(b4, w4, fma(b3, w3, b1 * w1)))), u);
    wn = fma(h, fma(b6, g6, fma(b5, g5, fma(b4, g4, fma(b3, g3, b1 * g1)))), w);
    g7 = g_of(M3, un);

    eu = h * fma(e7, wn, fma(e6, w6, fma(e5, w5, fma(e4, w4, fma(e3, w3, e1 * w1)))));
    ew = h * fma(e7, g7, fma(e6, g6, fma(e5, g5, fma(e4, g4, fma(e3, g3, e1 * g1)))));
}

// Step-size factor 0.9 err^(-1/5), evaluated in FP32 with the hardware
// log2/exp2 (a heuristic; only the accept test needs full precision).
__device__ __forceinline__ float step_factor(float err) {
    return 0.9f * __builtin_amdgcn_exp2f(-0.2f * __builtin_amdgcn_logf(err));
}

// ---------------------------------------------------------------------------
// Persistent integrator.
// ---------------------------------------------------------------------------
template <typename T>
struct Lane {
    T u, w, g, h, hh;
    double phi, phik;
    int id, attempts, nsteps, it;
    bool rej, refine, active;
};

struct IntegArgs {
    int64_t n;
    const double* u0;         // per-ray u0, or NULL (use u0_uniform)
    double u0_uniform;
    DevScene sc;
    DevTol tol;
    Work w;
    int chunk;
};

template <typename T>
__device__ __forceinline__ void finish(const IntegArgs& a, Lane<T>& L, uint8_t cls, double phi,
                                       double r_hit) {
    a.w.cls[L.id] = cls;
    a.w.phi_end[L.id] = phi;
    a.w.r_hit[L.id] = r_hit;
    a.w.steps[L.id] = L.nsteps;
    L.active = false;
}

// Drains one queue.  VIRTUAL: the queue is the index range [0, total) and a
// ray is taken only if its set-up tag equals `tag`; otherwise queue[] holds
// the ray indices.
template <typename T, bool VIRTUAL>
__device__ void run_queue(const IntegArgs& a, const int32_t* __restrict__ queue, int64_t total,
                          int32_t* head, uint8_t tag, T rtol, T atol, T ntol) {
    const int lane = lane_id();
    const T M3 = T(3.0 * a.sc.M);
    const double twoM = 2.0 * a.sc.M;
    const T usky = T(a.sc.u_sky);
    const T h0 = T(a.tol.h0), hmax = T(a.tol.hmax);
    const double rin = a.sc.rin, rout = a.sc.rout;

    Lane<T> L;
    L.active = false;
    int64_t cnext = 0, cend = 0;
    bool drained = false;

    for (;;) {
        // ---- refill idle lanes from the wavefront's current chunk ---------
        for (int round = 0; round < 2; ++round) {
            const uint64_t need = __ballot(!L.active);
            if (need == 0 || (drained && cnext >= cend)) break;
            if (cnext >= cend) {
                int base = 0;
                if (lane == 0) base = atomicAdd(head, a.chunk);
                base = __shfl(base, 0);
                // base < 0: the 32-bit head wrapped after the queue drained
                if (base < 0 || (int64_t)base >= total) {
                    drained = true;
                    break;
                }
                cnext = base;
                cend = min((int64_t)base + a.chunk, total);
            }
            const int nneed = __popcll(need);
            const int rank = rank_in(need);
            const int64_t avail = cend - cnext;
            if (!L.active && rank < avail) {
                const int64_t pos = cnext + rank;
                const int id = VIRTUAL ? (int)pos : queue[pos];
                if (!VIRTUAL || a.w.path[id] == tag) {
                    L.id = id;
                    L.u = T(a.u0 ? a.u0[id] : a.u0_uniform);
                    L.w = T(a.w.w0[id]);
                    L.g = g_of(M3, L.u);
                    L.h = h0;
                    L.phi = 0.0;
                    L.phik = a.w.phi1[id];
                    L.attempts = 0;
                    L.nsteps = 0;
                    L.it = 0;
                    L.rej = false;
                    L.refine = false;
                    L.active = true;
                }
            }
            cnext += min((int64_t)nneed, avail);
        }
        if (__ballot(L.active) == 0) {
            if (drained) break;
            continue;
        }
        if (!L.active) continue;

        // ---- one step attempt per active lane ------------------------------
        T ht = L.refine ? L.hh : L.h;
        bool land = false;
        if (!L.refine) {
            if (L.attempts >= a.tol.max_steps) {
                finish(a, L, UNRESOLVED, L.phi, 0.0);
                continue;
            }
            ++L.attempts;
            // Shorten a step that would pass the next disk-plane crossing so
            // that it lands on it exactly.
            if (L.phi + (double)ht >= L.phik) {
                ht = T(L.phik - L.phi);
                land = true;
            }
        }
        T un, wn, gn, eu, ew;
        dp45<T>(M3, L.u, L.w, L.g, ht, un, wn, gn, eu, ew);
        ++L.nsteps;

        if (L.refine) {
            // Newton on the step length for u(h) = u_sky, from the last
            // accepted state: h <- h - (u(h) - u_sky) / u'(h).
            const T dh = (un - usky) / wn;
            L.hh -= dh;
            ++L.it;
            if (fabs(dh) < ntol || L.it >= 4) finish(a, L, SKY, L.phi + (double)L.hh, 0.0);
            continue;
        }

        const T su = fma(rtol, fmax(fabs(L.u), fabs(un)), atol);
        const T sw = fma(rtol, fmax(fabs(L.w), fabs(wn)), atol);
        const bool acc = fabs(eu) <= su && fabs(ew) <= sw;
        const float err = fmaxf((float)fabs(eu) * __builtin_amdgcn_rcpf((float)su),
                                (float)fabs(ew) * __builtin_amdgcn_rcpf((float)sw));
        if (!acc) {
            L.h = ht * T(fmaxf(0.2f, step_factor(err)));
            L.rej = true;
            continue;
        }
        const double phin = land ? L.phik : L.phi + (double)ht;
        if (!land) {
            float fac = fminf(5.0f, fmaxf(0.2f, step_factor(err)));
            if (L.rej) fac = fminf(fac, 1.0f);
            L.h = ht * T(fac);
        }
        L.h = fmin(L.h, hmax);
        L.rej = false;

        // Events, in order: disk crossing, horizon, sky sphere, sweep cap.
        if (land) {
            const double r = 1.0 / (double)un;
            if (r >= rin && r <= rout) {
                finish(a, L, DISK, phin, r);
                continue;
            }
            L.phik += kPi;
        }
        if (twoM > 0.0 && twoM * (double)un >= 1.0) {
            finish(a, L, CAPTURED, phin, 0.0);
            continue;
        }
        if (un <= usky && wn < T(0)) {
            const T dh = (un - usky) / wn;
            L.hh = ht - dh;
            if (fabs(dh) < ntol) {
                finish(a, L, SKY, L.phi + (double)L.hh, 0.0);
            } else {
                L.refine = true;  // keep the accepted-from state as the base
                L.it = 1;
            }
            continue;
        }
        L.u = un;
        L.w = wn;
        L.g = gn;
        L.phi = phin;
        if (L.phi > a.tol.max_phi) finish(a, L, UNRESOLVED, L.phi, 0.0);
    }
}

// FP64 mode: one pass over all rays tagged FP64.
__global__ __launch_bounds__(kBlock) void k_integrate_fp64(IntegArgs a) {
    run_queue<double, true>(a, nullptr, a.n, &a.w.ctr[2], PATH_FP64, a.tol.rtol64, a.tol.atol64,
                            a.tol.newton64);
}

// FP32 mode: wavefronts first drain the (small) FP64 band queue, then the
// FP32 rays, in one launch so the band's long rays overlap the FP32 work.
__global__ __launch_bounds__(kBlock) void k_integrate_fp32(IntegArgs a) {
    const int64_t nband = a.w.ctr[0];
    run_queue<double, false>(a, a.w.q64, nband, &a.w.ctr[1], PATH_FP64, a.tol.rtol64,
                             a.tol.atol64, a.tol.newton64);
    run_queue<float, true>(a, nullptr, a.n, &a.w.ctr[2], PATH_FP32, a.tol.rtol32, a.tol.atol32,
                           a.tol.newton32);
}

// ---------------------------------------------------------------------------
// Shading and output.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_shade(Source src, DevScene sc, Work w, float* rgba,
                                                  Out out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= src.n) return;
    double o[3], dv[3];
    source_ray(src, i, o, dv);
    const Basis B = plane_basis(o, dv, sc.M, sc.r_sky);
    const uint8_t cls = w.cls[i];
    const double phi = w.phi_end[i];
    const double r_hit = w.r_hit[i];
    double sphi, cphi;
    sincos(phi, &sphi, &cphi);
    double s[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) s[k] = cphi * B.e1[k] + sphi * B.e2[k];
    if (cls == INVALID) s[0] = s[1] = s[2] = 0.0;

    if (rgba) {
        float4 px = make_float4(0.f, 0.f, 0.f, 1.f);
        if (cls == SKY) {
            const double theta = atan2(hypot(s[0], s[1]), s[2]);
            double varphi = atan2(s[1], s[0]);
            if (varphi < 0.0) varphi += 2.0 * kPi;
            const long parity =
                ((long)floor(theta / sc.cell_rad) + (long)floor(varphi / sc.cell_rad)) & 1L;
            const float g = parity ? 0.1f : 1.0f;
            px = make_float4(g, g, g, 1.f);
        } else if (cls == DISK) {
            const double I = pow(r_hit / sc.rin, sc.power);
            px = make_float4((float)I, (float)(0.6 * I), (float)(0.2 * I), 1.f);
        }
        reinterpret_cast<float4*>(rgba)[i] = px;
    }
    if (out.cls) out.cls[i] = cls;
    if (out.phi_end) out.phi_end[i] = phi;
    if (out.r_hit) out.r_hit[i] = r_hit;
    if (out.steps) out.steps[i] = w.steps[i];
    if (out.path) out.path[i] = w.path[i];
    if (out.exit_dir) {
#pragma unroll
        for (int k = 0; k < 3; ++k) out.exit_dir[3 * i + k] = s[k];
    }
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
    k_reset<<<1, 64, 0, s>>>(ctr);
    return hipGetLastError();
}

hipError_t launch_setup(const Source& src, const DevScene& sc, const DevRoute& rt, const Work& w,
                        double* out_b, hipStream_t s) {
    if (src.n == 0) return hipSuccess;
    k_setup<<<blocks_for(src.n), kBlock, 0, s>>>(src, sc, rt, w, out_b);
    return hipGetLastError();
}

hipError_t launch_integrate(int64_t n, bool explicit_u0, double u0_uniform, const DevScene& sc,
                            const DevTol& tol, int precision, const Work& w, int grid_blocks,
                            int chunk, hipStream_t s) {
    if (n == 0) return hipSuccess;
    IntegArgs a;
    a.n = n;
    a.u0 = explicit_u0 ? w.u0 : nullptr;
    a.u0_uniform = u0_uniform;
    a.sc = sc;
    a.tol = tol;
    a.w = w;
    a.chunk = chunk;
    if (precision == 1)
        k_integrate_fp32<<<grid_blocks, kBlock, 0, s>>>(a);
    else
        k_integrate_fp64<<<grid_blocks, kBlock, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_shade(const Source& src, const DevScene& sc, const Work& w, float* rgba,
                        const Out& out, hipStream_t s) {
    if (src.n == 0) return hipSuccess;
    k_shade<<<blocks_for(src.n), kBlock, 0, s>>>(src, sc, w, rgba, out);
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
