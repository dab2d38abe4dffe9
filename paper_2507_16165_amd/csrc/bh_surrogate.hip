// MLP surrogate of the photon-orbit sweep: training and inference kernels on
// the CDNA4 matrix cores (BF16 in, FP32 accumulate), and its C ABI.
//
// Network (units of M): inputs (b, r0) of an ingoing ray, features
//   f1 = sign(d) ln(1 + |d|/0.05) / 5, d = b - 3 sqrt(3),  f2 = (r0 - 105)/95,
// layers 2 -> 128 -> 128 -> 128 -> 2 with ReLU, outputs y0 (scaled residual of
// the exit azimuth against the first-order weak-field sweep) and y1 (capture
// logit).  Exit azimuth = sweep1(b, r0) + 12/b^2 * y0, with
//   sweep1 = pi - a(R) - a(r0),  a(r) = asin(b/r - (2 - b^2/r^2)/b),  R = 1000.
// Training labels come from the library's own FP64 integrator.
//
// Matrix-core layout.  v_mfma_f32_32x32x16_bf16 takes, per lane l (h = l/32,
// c = l%32), A[c][8h+e] and B[8h+e][c] (e = 0..7) and returns D[i][c] for
// i = 8(r/4) + 4h + r%4 in accumulator register r.  A layer is computed as
// Z^T = W^T H^T (rows = output features, columns = 32 rays).  Registers
// 8s..8s+7 of an output tile hold, per lane, exactly the 8 values a B operand
// needs for one 16-row block of the next layer -- in the K order
// pi(h, e) = e < 4 ? 4h + e : 8 + 4h + (e - 4).  The weights are packed once in
// that permuted order, so the three hidden layers chain in registers with no
// data movement between them.
#include "bh_internal.h"

#include <math.h>
#include <string.h>

#include <vector>

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef short i16x2 __attribute__((ext_vector_type(2)));

namespace bh {

// ---- flat FP32 parameter vector: W1[2][128] b1 W2[128][128] b2 W3 b3 W4[128][2] b4
constexpr int kH = 128;
constexpr int OFF_W1 = 0, OFF_B1 = 256, OFF_W2 = 384, OFF_B2 = OFF_W2 + kH * kH,
              OFF_W3 = OFF_B2 + kH, OFF_B3 = OFF_W3 + kH * kH, OFF_W4 = OFF_B3 + kH,
              OFF_B4 = OFF_W4 + 2 * kH, NPARAM = OFF_B4 + 2;
static_assert(NPARAM == 33666, "parameter count");

// ---- inference pack (bf16, lane order), offsets in bf16 elements
constexpr int PK_P1 = 0;                          // [4 mt][64 lanes][8]
constexpr int PK_P2 = PK_P1 + 4 * 64 * 8;         // [4 mt][8 kt][64][8]
constexpr int PK_P3 = PK_P2 + 4 * 8 * 64 * 8;
constexpr int PK_P4 = PK_P3 + 4 * 8 * 64 * 8;     // [8 kt][64][8]
constexpr int PK_BF16 = PK_P4 + 8 * 64 * 8;       // end of the bf16 part
constexpr int PK_B2 = 0, PK_B3 = 128, PK_B4 = 256, PK_F32 = 288;   // float part

constexpr float kBc = 5.19615242270663188f;
constexpr double kPiD = 3.14159265358979323846;
constexpr double kRsky = 1000.0;

__host__ __device__ inline int perm_k(int h, int e) { return e < 4 ? 4 * h + e : 8 + 4 * h + (e - 4); }

// ln(1 + x) as log2(1 + x) ln 2 from the hardware log2 (about 1 ulp): the
// absolute error, a few 1e-8, is far below the bf16 hi/lo split that carries
// the feature into the network (about 16 bits).
__device__ inline float feature1(float bm) {
    const float d = bm - kBc;
    const float m = __builtin_amdgcn_logf(fmaf(fabsf(d), 20.0f, 1.0f)) * (0.693147181f * 0.2f);
    return d < 0.0f ? -m : m;
}
__device__ inline float feature2(float r0m) { return (r0m - 105.0f) * (1.0f / 95.0f); }

// First-order weak-field sweep from r0 to the sky sphere (M = 1), and the
// residual scale S(b) = 12 / b^2.
__device__ inline double sweep1(double b, double r0) {
    auto a = [b](double r) {
        double x = b / r - (2.0 - b * b / (r * r)) / b;
        x = fmin(1.0, fmax(-1.0, x));
        return asin(x);
    };
    return kPiD - a(kRsky) - a(r0);
}
__device__ inline double res_scale(double b) { return 12.0 / (b * b); }

// ---------------------------------------------------------------------------
// Generic GEMM for training: C = A B (+bias[n]) (relu) (mask: C *= [mask > 0]),
// A: M x K, B: K x N (bf16, arbitrary element strides), FP32 accumulation.
// One wavefront per 32x32 tile; M, N multiples of 32, K multiple of 16.
// ---------------------------------------------------------------------------
struct GemmArgs {
    const bf16* A;
    int64_t a_m, a_k;
    const bf16* B;
    int64_t b_k, b_n;
    int M, N, K;
    const float* bias;
    int relu;
    const bf16* mask;
    int64_t mk_m, mk_n;
    float* Cf;
    int64_t cf_m, cf_n;
    bf16* Cb;
    int64_t cb_m, cb_n;
    // split-K: ksplit > 1 writes FP32 partial tiles of K/ksplit-long slices
    // to part[ks][M][N]; k_gemm_reduce sums them in slice order (so the
    // result does not depend on scheduling) and applies the epilogue.
    int ksplit;
    float* part;
};

// The epilogue of output element (i, j).
__device__ inline void gemm_store(const GemmArgs& g, int64_t i, int64_t j, float v) {
    if (g.bias) v += g.bias[j];
    if (g.relu) v = fmaxf(v, 0.0f);
    if (g.mask && !((float)g.mask[i * g.mk_m + j * g.mk_n] > 0.0f)) v = 0.0f;
    if (g.Cf) g.Cf[i * g.cf_m + j * g.cf_n] = v;
    if (g.Cb) g.Cb[i * g.cb_m + j * g.cb_n] = (bf16)v;
}

__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
    const int wave = (int)((blockIdx.x * 256u + threadIdx.x) >> 6);
    const int tiles_n = g.N >> 5, tiles = (g.M >> 5) * tiles_n;
    if (wave >= tiles * g.ksplit) return;  // whole wavefront
    const int ks = wave / tiles, t = wave % tiles;
    const int tm = t / tiles_n, tn = t % tiles_n;
    const int l = threadIdx.x & 63, h = l >> 5, c = l & 31;
    f32x16 acc = {};
    const int64_t arow = (int64_t)(tm * 32 + c) * g.a_m;
    const int64_t bcol = (int64_t)(tn * 32 + c) * g.b_n;
    const int kc = g.K / g.ksplit;
    for (int k0 = ks * kc; k0 < (ks + 1) * kc; k0 += 16) {
        bf16x8 a, b;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int64_t k = k0 + 8 * h + e;
            a[e] = g.A[arow + k * g.a_k];
            b[e] = g.B[k * g.b_k + bcol];
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int64_t i = tm * 32 + 8 * (r >> 2) + 4 * h + (r & 3), j = tn * 32 + c;
        if (g.ksplit > 1) g.part[((int64_t)ks * g.M + i) * g.N + j] = acc[r];
        else gemm_store(g, i, j, acc[r]);
    }
}

__global__ __launch_bounds__(256) void k_gemm_reduce(GemmArgs g) {
    const int64_t mn = (int64_t)g.M * g.N;
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= mn) return;
    float v = 0.0f;
    for (int ks = 0; ks < g.ksplit; ++ks) v += g.part[ks * mn + idx];
    gemm_store(g, idx / g.N, idx % g.N, v);
}

// ---------------------------------------------------------------------------
// Packing: FP32 master -> bf16 working copies (training GEMMs) and the
// lane-ordered inference pack.
// ---------------------------------------------------------------------------
struct Train {
    bf16* W1ext;   // 32 x 128: rows {w1, w1, w2, w2, b1, 0...}: inputs {f1_hi, f1_lo, f2_hi, f2_lo, 1}
    bf16* W2b;     // 128 x 128
    bf16* W3b;
    bf16* W4pad;   // 128 x 32 (columns 0, 1)
    float* b2r;    // bf16-rounded biases as float
    float* b3r;
    float* b4pad;  // 32
};

__device__ inline float rbf(float x) { return (float)(bf16)x; }

__global__ void k_pack(const float* __restrict__ P, Train t, bf16* pk, float* pkf) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int stride = gridDim.x * blockDim.x;
    for (int i = tid; i < 32 * kH; i += stride) {  // W1ext
        const int row = i / kH, o = i % kH;
        float v = 0.0f;
        if (row <= 1) v = P[OFF_W1 + o];
        else if (row <= 3) v = P[OFF_W1 + kH + o];
        else if (row == 4) v = P[OFF_B1 + o];
        t.W1ext[i] = (bf16)v;
    }
    for (int i = tid; i < kH * kH; i += stride) {
        t.W2b[i] = (bf16)P[OFF_W2 + i];
        t.W3b[i] = (bf16)P[OFF_W3 + i];
    }
    for (int i = tid; i < kH * 32; i += stride) {
        const int k = i / 32, o = i % 32;
        t.W4pad[i] = (bf16)(o < 2 ? P[OFF_W4 + 2 * k + o] : 0.0f);
    }
    for (int i = tid; i < kH; i += stride) {
        t.b2r[i] = rbf(P[OFF_B2 + i]);
        t.b3r[i] = rbf(P[OFF_B3 + i]);
        pkf[PK_B2 + i] = rbf(P[OFF_B2 + i]);
        pkf[PK_B3 + i] = rbf(P[OFF_B3 + i]);
    }
    for (int i = tid; i < 32; i += stride) {
        const float v = i < 2 ? rbf(P[OFF_B4 + i]) : 0.0f;
        t.b4pad[i] = v;
        pkf[PK_B4 + i] = v;
    }
    // inference pack: P1 (layer 1 with the bias row), P2/P3 (hidden layers),
    // P4 (output layer padded to 32 rows), K in the permuted order pi(h, e)
    for (int i = tid; i < 4 * 64 * 8; i += stride) {
        const int e = i % 8, l = (i / 8) % 64, mt = i / 512;
        const int h = l >> 5, o = mt * 32 + (l & 31);
        float v = 0.0f;
        if (h == 0) {
            if (e <= 1) v = P[OFF_W1 + o];
            else if (e <= 3) v = P[OFF_W1 + kH + o];
            else if (e == 4) v = P[OFF_B1 + o];
        }
        pk[PK_P1 + i] = (bf16)v;
    }
    for (int i = tid; i < 4 * 8 * 64 * 8; i += stride) {
        const int e = i % 8, l = (i / 8) % 64, kt = (i / 512) % 8, mt = i / 4096;
        const int in = kt * 16 + perm_k(l >> 5, e), o = mt * 32 + (l & 31);
        pk[PK_P2 + i] = (bf16)P[OFF_W2 + in * kH + o];
        pk[PK_P3 + i] = (bf16)P[OFF_W3 + in * kH + o];
    }
    for (int i = tid; i < 8 * 64 * 8; i += stride) {
        const int e = i % 8, l = (i / 8) % 64, kt = i / 512;
        const int in = kt * 16 + perm_k(l >> 5, e), o = l & 31;
        pk[PK_P4 + i] = (bf16)(o < 2 ? P[OFF_W4 + 2 * in + o] : 0.0f);
    }
}

// ---------------------------------------------------------------------------
// Training: batch preparation, loss, gradient assembly, Adam.
// ---------------------------------------------------------------------------
__device__ inline void split_bf16(float x, bf16& hi, bf16& lo) {
    hi = (bf16)x;
    lo = (bf16)(x - (float)hi);
}

// X1 row: {f1_hi, f1_lo, f2_hi, f2_lo, 1, 0 ...} (32 columns); target, masks.
__global__ void k_prep(int64_t n, const double* b, const double* r0, const double* phi,
                       const uint8_t* cap, bf16* X1, float* tgt, float* esc, float* capf) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const double bb = b[s], rr = r0[s];
    bf16 f1h, f1l, f2h, f2l;
    split_bf16(feature1((float)bb), f1h, f1l);
    split_bf16(feature2((float)rr), f2h, f2l);
    bf16* x = X1 + s * 32;
#pragma unroll
    for (int k = 0; k < 32; ++k) x[k] = (bf16)0.0f;
    x[0] = f1h;
    x[1] = f1l;
    x[2] = f2h;
    x[3] = f2l;
    x[4] = (bf16)1.0f;
    const bool c = cap[s] != 0;
    // regression domain: escaped rays with b >= 10 M
    const bool e = !c && isfinite(phi[s]) && bb >= 10.0;
    esc[s] = e ? 1.0f : 0.0f;
    capf[s] = c ? 1.0f : 0.0f;
    tgt[s] = e ? (float)((phi[s] - sweep1(bb, rr)) / res_scale(bb)) : 0.0f;
}

__global__ void k_zero(float* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

// Loss (1/B) sum [e (y0 - t)^2 + 0.1 BCE(y1, c)] and dY (bf16, B x 32).
__global__ void k_loss(int64_t n, const float* Y, const float* tgt, const float* esc,
                       const float* capf, bf16* dY, float* loss) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float part = 0.0f;
    if (s < n) {
        const float inv = 1.0f / (float)n;
        const float y0 = Y[s * 32], y1 = Y[s * 32 + 1];
        const float r = y0 - tgt[s];
        const float c = capf[s];
        const float bce = fmaxf(y1, 0.0f) - y1 * c + log1pf(expf(-fabsf(y1)));
        part = (esc[s] * r * r + 0.1f * bce) * inv;
        bf16* d = dY + s * 32;
        d[0] = (bf16)(2.0f * esc[s] * r * inv);
        d[1] = (bf16)(0.1f * (1.0f / (1.0f + expf(-y1)) - c) * inv);
        for (int k = 2; k < 32; ++k) d[k] = (bf16)0.0f;
    }
    // wave reduction, one atomic per wavefront
    for (int off = 32; off > 0; off >>= 1) part += __shfl_down(part, off);
    if ((threadIdx.x & 63) == 0) atomicAdd(loss, part);
}

// Gradient vector from the GEMM outputs: gW1ext (32 x 128), gW4pad (128 x 32),
// column sums cs2, cs3 (rows 0 of 32 x 128 GEMMs with a ones operand), cs4.
__global__ void k_assemble(const float* gW1ext, const float* gW4pad, const float* cs2,
                           const float* cs3, const float* cs4, float* G) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kH) {
        G[OFF_W1 + i] = gW1ext[0 * kH + i] + gW1ext[1 * kH + i];
        G[OFF_W1 + kH + i] = gW1ext[2 * kH + i] + gW1ext[3 * kH + i];
        G[OFF_B1 + i] = gW1ext[4 * kH + i];
        G[OFF_B2 + i] = cs2[i];
        G[OFF_B3 + i] = cs3[i];
        G[OFF_W4 + 2 * i] = gW4pad[i * 32];
        G[OFF_W4 + 2 * i + 1] = gW4pad[i * 32 + 1];
    }
    if (i < 2) G[OFF_B4 + i] = cs4[i];
}

// Adam (Kingma & Ba 2015) on the FP32 master: c1 = 1/(1 - beta1^t),
// c2 = 1/(1 - beta2^t).
__global__ void k_adam(int n, float* P, const float* G, float* m, float* v, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = G[i];
    const float mm = b1 * m[i] + (1.0f - b1) * g;
    const float vv = b2 * v[i] + (1.0f - b2) * g * g;
    m[i] = mm;
    v[i] = vv;
    P[i] -= lr * (mm * c1) / (sqrtf(vv * c2) + eps);
}

// ---------------------------------------------------------------------------
// Fused inference: one wavefront evaluates 32 rays through all four layers
// with the operands chained in registers (see the header comment).
// ---------------------------------------------------------------------------
constexpr int kInferThreads = 256;
constexpr int kPackBytes = PK_BF16 * 2 + PK_F32 * 4;

// ReLU of accumulator values off..off+7, rounded to bf16.  Rounding keeps
// the sign, so the ReLU acts on the bf16 bit patterns as a signed 16-bit max
// with 0: one packed integer max per two values, where fmaxf in the default
// IEEE mode costs two float instructions per value (it quiets its input
// first).  A -0 becomes +0; activations are finite.
__device__ inline bf16x8 relu_bf16(const f32x16& acc, int off) {
    uint4 r;
    uint32_t* q = reinterpret_cast<uint32_t*>(&r);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const f32x2 x = {acc[off + 2 * k], acc[off + 2 * k + 1]};
        const i16x2 v = __builtin_bit_cast(i16x2, __builtin_convertvector(x, bf16x2));
        q[k] = __builtin_bit_cast(uint32_t, __builtin_elementwise_max(v, (i16x2)0));
    }
    return __builtin_bit_cast(bf16x8, r);
}

// NT tiles of 32 rays per call: each weight operand read from LDS feeds NT
// matrix-core instructions (NT = 2 halves the LDS traffic per ray).
template <int NT>
__device__ inline void mlp_tiles(const bf16* __restrict__ pk, const float* __restrict__ pkf,
                                 const float* f1, const float* f2, float* y0, float* y1) {
    // Keeps the compiler from hoisting the (loop-invariant) weight reads out
    // of the callers' tile loops: held in registers they would need ~300 VGPRs.
    asm volatile("" ::: "memory");
    const int l = threadIdx.x & 63, h = l >> 5;
    bf16x8 op[NT][8];
    // layer 1: inputs {f1_hi, f1_lo, f2_hi, f2_lo, 1} on the h = 0 half
    {
        const bf16x8* p1 = reinterpret_cast<const bf16x8*>(pk + PK_P1);
        bf16x8 x0[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            bf16 a, b, c, d;
            split_bf16(f1[t], a, b);
            split_bf16(f2[t], c, d);
            const bf16 z = (bf16)0.0f, one = (bf16)1.0f;
            x0[t][0] = h ? z : a;
            x0[t][1] = h ? z : b;
            x0[t][2] = h ? z : c;
            x0[t][3] = h ? z : d;
            x0[t][4] = h ? z : one;
            x0[t][5] = z;
            x0[t][6] = z;
            x0[t][7] = z;
        }
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const bf16x8 w = p1[mt * 64 + l];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                f32x16 acc = {};
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, x0[t], acc, 0, 0, 0);
                op[t][2 * mt] = relu_bf16(acc, 0);
                op[t][2 * mt + 1] = relu_bf16(acc, 8);
            }
        }
    }
    // hidden layers 2 and 3
#pragma unroll
    for (int layer = 0; layer < 2; ++layer) {
        const bf16x8* pw = reinterpret_cast<const bf16x8*>(pk + (layer ? PK_P3 : PK_P2));
        const float* bias = pkf + (layer ? PK_B3 : PK_B2);
        f32x16 acc[NT][4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const float bv = bias[mt * 32 + 8 * (r >> 2) + 4 * h + (r & 3)];
#pragma unroll
                for (int t = 0; t < NT; ++t) acc[t][mt][r] = bv;
            }
        }
        // Weight operands double-buffered: the read of the next one is in
        // flight while the current one feeds the matrix cores.
        bf16x8 w = pw[l];
#pragma unroll
        for (int kt = 0; kt < 8; ++kt) {
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                const int nx = kt * 4 + mt + 1;
                bf16x8 wn = w;
                if (nx < 32) wn = pw[((nx & 3) * 8 + (nx >> 2)) * 64 + l];
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    acc[t][mt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, op[t][kt], acc[t][mt],
                                                                        0, 0, 0);
                w = wn;
            }
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                op[t][2 * mt] = relu_bf16(acc[t][mt], 0);
                op[t][2 * mt + 1] = relu_bf16(acc[t][mt], 8);
            }
        }
    }
    // output layer (rows 0 and 1 of a 32-row tile)
    const bf16x8* p4 = reinterpret_cast<const bf16x8*>(pk + PK_P4);
    f32x16 acc[NT];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const float bv = pkf[PK_B4 + 8 * (r >> 2) + 4 * h + (r & 3)];
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t][r] = bv;
    }
#pragma unroll
    for (int kt = 0; kt < 8; ++kt) {
        const bf16x8 w = p4[kt * 64 + l];
#pragma unroll
        for (int t = 0; t < NT; ++t)
            acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, op[t][kt], acc[t], 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        y0[t] = acc[t][0];  // valid on lanes 0..31 (ray = lane)
        y1[t] = acc[t][1];
    }
}

// Copies the inference pack into LDS (kInferThreads threads, coalesced 16 B
// per thread and step).  All of a thread's loads are issued before its LDS
// stores, so the copy costs about one memory latency, not one per step.
__device__ inline void load_pack(const void* src, void* lds) {
    constexpr int kN = kPackBytes / 16;
    constexpr int kPer = (kN + kInferThreads - 1) / kInferThreads;
    const int4* s = reinterpret_cast<const int4*>(src);
    int4* d = reinterpret_cast<int4*>(lds);
    int4 v[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int i = threadIdx.x + k * kInferThreads;
        if (i < kN) v[k] = s[i];
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int i = threadIdx.x + k * kInferThreads;
        if (i < kN) d[i] = v[k];
    }
    __syncthreads();
}

// Validation / label-side inference: y (n x 2) and the predicted exit azimuth.
__global__ __launch_bounds__(kInferThreads) void k_infer(const void* __restrict__ pack, int64_t n,
                                                         const double* b, const double* r0,
                                                         float* y, double* phi_pred) {
    extern __shared__ __align__(16) unsigned char smem[];
    load_pack(pack, smem);
    const bf16* pk = reinterpret_cast<const bf16*>(smem);
    const float* pkf = reinterpret_cast<const float*>(smem + PK_BF16 * 2);
    const int l = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (kInferThreads / 64);
    const int64_t w0 = (int64_t)blockIdx.x * (kInferThreads / 64) + (threadIdx.x >> 6);
    for (int64_t t = w0; t * 64 < n; t += waves) {
        float f1[2], f2[2], y0[2], y1[2];
        int64_t sidx[2];
        double bb[2], rr[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            sidx[q] = t * 64 + 32 * q + (l & 31);
            const bool ok = sidx[q] < n;
            bb[q] = ok ? b[sidx[q]] : 10.0;
            rr[q] = ok ? r0[sidx[q]] : 100.0;
            f1[q] = feature1((float)bb[q]);
            f2[q] = feature2((float)rr[q]);
        }
        mlp_tiles<2>(pk, pkf, f1, f2, y0, y1);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int64_t s = sidx[q];
            if (s < n && l < 32) {
                if (y) {
                    y[2 * s] = y0[q];
                    y[2 * s + 1] = y1[q];
                }
                if (phi_pred) phi_pred[s] = sweep1(bb[q], rr[q]) + res_scale(bb[q]) * (double)y0[q];
            }
        }
    }
}

// Trust map: per-bin maximum exit error of escaping validation rays (a
// predicted capture counts as an infinite error) and the number of samples.
__global__ void k_trust_acc(int64_t n, const double* b, const double* r0, const double* phi_true,
                            const double* phi_pred, const float* y, unsigned* maxerr,
                            unsigned* count) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n || !isfinite(phi_true[s])) return;
    const int bin = trust_bin((float)b[s], (float)r0[s]);
    if (bin < 0) return;
    float err = (float)fabs(phi_pred[s] - phi_true[s]);
    if (!(y[2 * s + 1] < 0.0f) || !(err == err)) err = 3.0e38f;
    atomicMax(&maxerr[bin], __float_as_uint(err));
    atomicAdd(&count[bin], 1u);
}

__global__ void k_trust_fin(const unsigned* maxerr, const unsigned* count, float thresh,
                            unsigned min_count, uint8_t* trust) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kTrustB * kTrustR) return;
    trust[i] = (count[i] >= min_count && __uint_as_float(maxerr[i]) <= thresh) ? 1 : 0;
}

// Rays for label generation: origin (r0, 0, 0), ingoing direction at angle
// psi to the inward radial with sin psi = u0 / sqrt(1/b^2 + 2 u0^3) (the
// first integral with M = 1, solved for the initial slope).
__global__ void k_pair_rays(int64_t n, const double* b, const double* r0, double* o, double* d) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const double u0 = 1.0 / r0[s], bb = b[s];
    const double sp = u0 / sqrt(1.0 / (bb * bb) + 2.0 * u0 * u0 * u0);
    const double cp = sqrt(fmax(0.0, 1.0 - sp * sp));
    o[3 * s] = r0[s];
    o[3 * s + 1] = 0.0;
    o[3 * s + 2] = 0.0;
    d[3 * s] = sp <= 1.0 ? -cp : __builtin_nan("");
    d[3 * s + 1] = sp;
    d[3 * s + 2] = 0.0;
}

// Label records from the traced classes: captured flag, exit azimuth (NaN
// unless the ray reached the sky sphere).
__global__ void k_labels_finish(int64_t n, uint8_t* cls_cap, double* phi) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const uint8_t c = cls_cap[s];
    if (c != SKY) phi[s] = __builtin_nan("");
    cls_cap[s] = c == CAPTURED ? 1 : 0;
}

// ---------------------------------------------------------------------------
// Render path: the surrogate list that set-up fills (kSlices slices of ray
// indices with {b, w0}).  Tiles of 32 listed rays are dealt to wavefronts in
// pairs, round-robin (every tile costs the same); a wavefront loads its next
// pair's entries before it evaluates the current one.  The exit azimuth goes straight
// into the result record.  A ray whose capture logit disagrees with b > b_c is
// handed back to the FP32 integrator by restoring its start record.
// ---------------------------------------------------------------------------
struct SurRender {
    int64_t slice_cap;  // entries per slice of the list
    Work w;
    float r0m;     // camera distance / M
    float inv_r0m; // M / camera distance
    double inv_M;  // 1/M
    // batches: each listed ray's request (w.rq) selects these constants
    // instead of the three above; NULL for a single render
    const SurReq* req;
};

// The render path's exit azimuth in FP32 (its error budget is 1e-4 rad):
// first-order sweep plus the scaled network output.  ib = 1/b (hardware
// reciprocal, 1 ulp), ir0 = 1/r0; with q = b/r, a(r) = asin(q - (2 - q^2)/b).
__device__ inline float sweep1f(float b, float ib, float ir0) {
    auto a = [ib](float q) {
        const float x = q - (2.0f - q * q) * ib;
        return asinf(fminf(1.0f, fmaxf(-1.0f, x)));
    };
    return 3.14159265f - a(b * (1.0f / 1000.0f)) - a(b * ir0);
}

// BATCH: FP32 batch records (rec32 / res32, no path byte), per-ray inv_r0m.
template <bool BATCH>
__device__ inline void sur_finish(const SurRender& a, int id, double w0, float bm, float y0,
                                  float y1, float inv_r0m) {
    if (!(y1 < 0.0f)) {
        if constexpr (BATCH) {
            a.w.rec32[id] = make_float2((float)w0, a.w.rec32[id].y);
        } else {
            a.w.rec[id] = make_double2(w0, a.w.rec[id].y);
            a.w.path[id] = PATH_FP32;
        }
        return;
    }
    const float ib = __builtin_amdgcn_rcpf(bm);
    const float phi = sweep1f(bm, ib, inv_r0m) + (12.0f * ib * ib) * y0;
    // SKY, no integration steps (an FP32 record's zero r_hit is the class)
    if constexpr (BATCH) {
        a.w.res32[id] = make_float2(phi, 0.0f);
    } else {
        a.w.res[id] = make_double2((double)phi, 0.0);
        a.w.clst[id] = 0;
    }
}

// Entry of listed ray j of tile t: tiles are numbered over the slices in
// order; first[s] is the first tile of slice s (first[kSurSlices] = all
// tiles), cnt[s] its length.  Lanes past the end of their slice read the
// slice's first entry.
struct SurEntry {
    int64_t slot;
    bool valid;
};

// `slice` is the caller's last slice (tiles of a wavefront only increase):
// it walks forward to the last slice with first[s] <= t.
__device__ inline SurEntry sur_entry(const int* cnt, const int* first, int64_t slice_cap,
                                     int64_t t, int lane, int& slice) {
    int lo = slice;
    while (lo + 1 < kSurSlices && first[lo + 1] <= t) ++lo;
    slice = lo;
    const int64_t j = (t - first[lo]) * 32 + lane;
    const bool valid = j < cnt[lo];
    return {lo * slice_cap + (valid ? j : 0), valid};
}

// A wavefront evaluates two tiles per pass (tiles 2p and 2p + 1 of pair p):
// each weight operand read from LDS then feeds two matrix-core instructions.
// With one tile per pass the four SIMDs of a CU need about 128 B of LDS reads
// per clock at the matrix-core rate, the whole LDS bandwidth.
template <bool BATCH>
__global__ __launch_bounds__(kInferThreads) __attribute__((amdgpu_waves_per_eu(2)))
void k_sur_render(const void* __restrict__ pack, SurRender a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_cnt[kSurSlices], s_first[kSurSlices + 1];
    if (threadIdx.x < kSurSlices) s_cnt[threadIdx.x] = a.w.ctr[kCtrSur + threadIdx.x * kCtrStride];
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int q = 0; q < kSurSlices; ++q) {
            s_first[q] = t;
            t += (s_cnt[q] + 31) / 32;
        }
        s_first[kSurSlices] = t;
    }
    __syncthreads();
    const int64_t tiles = s_first[kSurSlices];
    const int64_t pairs = (tiles + 1) / 2;
    constexpr int wpb = kInferThreads / 64;
    if ((int64_t)blockIdx.x * wpb >= pairs) return;  // block-uniform: nothing for this block
    load_pack(pack, smem);
    const bf16* pk = reinterpret_cast<const bf16*>(smem);
    const float* pkf = reinterpret_cast<const float*>(smem + PK_BF16 * 2);
    const int l = threadIdx.x & 63;
    const float f2v = feature2(a.r0m);
    const int64_t nw = (int64_t)gridDim.x * wpb;
    int64_t p = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6);
    int slice = 0;
    // Entries of the two tiles of pair q (a tile past the list is not valid).
    auto fetch = [&](int64_t q, SurEntry (&e)[2], int (&id)[2], double2 (&rec)[2]) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            e[k] = SurEntry{0, false};
            id[k] = 0;
            rec[k] = make_double2(10.0, 0.0);
            const int64_t t = 2 * q + k;
            if (q < pairs && t < tiles) {
                e[k] = sur_entry(s_cnt, s_first, a.slice_cap, t, l & 31, slice);
                id[k] = a.w.qsur[e[k].slot];
                rec[k] = a.w.qsurrec[e[k].slot];
            }
        }
    };
    SurEntry e[2];
    int id[2];
    double2 rec[2];
    fetch(p, e, id, rec);
    for (; p < pairs; p += nw) {
        // next pair's entries in flight while this one is evaluated
        SurEntry en[2];
        int idn[2];
        double2 recn[2];
        fetch(p + nw, en, idn, recn);
        float bm[2], f1[2], f2[2] = {f2v, f2v}, y0[2], y1[2], ir0[2] = {a.inv_r0m, a.inv_r0m};
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            if constexpr (BATCH) {
                // the ray's request (an invalid lane reads entry 0: its
                // values are computed and dropped)
                const SurReq q = a.req[a.w.rq[id[k]]];
                bm[k] = (float)(rec[k].x * q.inv_M);
                f2[k] = feature2(q.r0m);
                ir0[k] = q.inv_r0m;
            } else {
                bm[k] = (float)(rec[k].x * a.inv_M);
            }
            f1[k] = feature1(bm[k]);
        }
        mlp_tiles<2>(pk, pkf, f1, f2, y0, y1);
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            if (l < 32 && e[k].valid)
                sur_finish<BATCH>(a, id[k], rec[k].y, bm[k], y0[k], y1[k], ir0[k]);
            e[k] = en[k];
            id[k] = idn[k];
            rec[k] = recn[k];
        }
    }
}

// Two blocks per CU (the weights fill ~66 KB of LDS per block); blocks beyond
// the list's tiles return at once.
static unsigned sur_grid(int64_t n, int cus) {
    int64_t g = (int64_t)cus * 2;
    const int64_t need = (n + 64 * (kInferThreads / 64) - 1) / (64 * (kInferThreads / 64));
    if (g > need) g = need > 0 ? need : 1;
    return (unsigned)g;
}

hipError_t launch_surrogate_render(int64_t n, const Work& w, const void* pack, double M,
                                   double r_cam, int cus, hipStream_t s) {
    SurRender a;
    a.slice_cap = sur_slice_cap(n);
    a.w = w;
    a.r0m = (float)(r_cam / M);
    a.inv_r0m = (float)(M / r_cam);
    a.inv_M = 1.0 / M;
    a.req = nullptr;
    k_sur_render<false><<<sur_grid(n, cus), kInferThreads, kPackBytes, s>>>(pack, a);
    return hipGetLastError();
}

hipError_t launch_surrogate_render_batch(int64_t n, const Work& w, const void* pack,
                                         const SurReq* req, int cus, hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (!w.rec32 || !w.res32 || !w.rq || !req) return hipErrorInvalidValue;
    SurRender a;
    a.slice_cap = sur_slice_cap(n);
    a.w = w;
    a.r0m = 105.0f;  // unused: each ray's request gives its constants
    a.inv_r0m = 0.0f;
    a.inv_M = 0.0;
    a.req = req;
    k_sur_render<true><<<sur_grid(n, cus), kInferThreads, kPackBytes, s>>>(pack, a);
    return hipGetLastError();
}

}  // namespace bh

// ===========================================================================
// C ABI
// ===========================================================================
using namespace bh;

struct bh_surrogate {
    int device = 0;
    int64_t max_batch = 0;
    void* base = nullptr;
    float* P = nullptr;     // master
    float* m = nullptr;
    float* v = nullptr;
    float* G = nullptr;     // last gradient
    Train t{};
    bf16* pk = nullptr;     // inference pack (bf16 part), followed by the float part
    float* pkf = nullptr;
    uint8_t* trust = nullptr;
    unsigned* tacc = nullptr;  // 2 x kTrustB*kTrustR (max error bits, counts)
    // training scratch
    bf16 *X1 = nullptr, *H1 = nullptr, *H2 = nullptr, *H3 = nullptr;
    bf16 *dY = nullptr, *dZ1 = nullptr, *dZ2 = nullptr, *dZ3 = nullptr, *ones = nullptr;
    float *Y = nullptr, *tgt = nullptr, *esc = nullptr, *capf = nullptr;
    float *gW1ext = nullptr, *gW4pad = nullptr, *cs = nullptr;  // cs: 3 x 32 x 128
    float* loss = nullptr;
    float* part = nullptr;  // split-K partial products, kMaxSplit x 128 x 128
    // label scratch (grown on demand)
    void* lab = nullptr;
    int64_t lab_cap = 0;
    int step = 0;
    int trusted = 0;
    unsigned version = 0;  // changes with the parameters and the trust map
    int cus = 256;
};

namespace {

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

// Split-K for the weight-gradient products (K = batch, at most 128 x 128
// outputs: too few tiles to fill the chip): slices of >= 256, at most
// kMaxSplit of them.
constexpr int kMaxSplit = 16;

hipError_t gemm(GemmArgs g, hipStream_t s, float* part) {
    const int tiles = (g.M / 32) * (g.N / 32);
    g.ksplit = 1;
    g.part = part;
    if (g.K >= 1024 && (int64_t)g.M * g.N <= kH * kH) {
        while (g.ksplit < kMaxSplit && g.K / (2 * g.ksplit) >= 256 &&
               (g.K / 16) % (2 * g.ksplit) == 0)
            g.ksplit *= 2;
    }
    const int waves = tiles * g.ksplit;
    k_gemm<<<(waves + 3) / 4, 256, 0, s>>>(g);
    if (g.ksplit > 1) {
        const int64_t mn = (int64_t)g.M * g.N;
        k_gemm_reduce<<<(unsigned)((mn + 255) / 256), 256, 0, s>>>(g);
    }
    return hipGetLastError();
}

GemmArgs gemm_args(const bf16* A, int64_t a_m, int64_t a_k, const bf16* B, int64_t b_k,
                   int64_t b_n, int M, int N, int K) {
    GemmArgs g;
    memset(&g, 0, sizeof g);
    g.A = A;
    g.a_m = a_m;
    g.a_k = a_k;
    g.B = B;
    g.b_k = b_k;
    g.b_n = b_n;
    g.M = M;
    g.N = N;
    g.K = K;
    return g;
}

hipError_t repack(bh_surrogate* s, hipStream_t st) {
    k_pack<<<64, 256, 0, st>>>(s->P, s->t, s->pk, s->pkf);
    return hipGetLastError();
}

#define HIPCHK(x, what)                                 \
    do {                                                \
        hipError_t e_ = (x);                            \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

}  // namespace

extern "C" {

bh_status bh_surrogate_create(const float* params, int64_t count, int64_t max_batch,
                              bh_surrogate** out) {
    if (!out) return fail(BH_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!params || count != NPARAM)
        return fail(BH_ERR_ARG, "params must hold %d floats", NPARAM);
    if (max_batch < 32 || max_batch % 32 != 0 || max_batch > (1 << 24))
        return fail(BH_ERR_ARG, "max_batch must be a positive multiple of 32 (<= 2^24)");
    bh_surrogate* s = new bh_surrogate();
    HIPCHK(hipGetDevice(&s->device), "hipGetDevice");
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, s->device) == hipSuccess &&
        cus > 0)
        s->cus = cus;
    s->max_batch = max_batch;
    const int64_t B = max_batch;
    const size_t szP = al(NPARAM * 4);
    size_t total = 4 * szP;
    total += al(32 * kH * 2) + 2 * al(kH * kH * 2) + al(kH * 32 * 2) + 2 * al(kH * 4) + al(32 * 4);
    total += al(kPackBytes) + al(kTrustB * kTrustR) + al(2 * kTrustB * kTrustR * 4);
    total += al(B * 32 * 2) + 3 * al(B * kH * 2) + al(B * 32 * 2) + 3 * al(B * kH * 2) + al(B * 2);
    total += al(B * 32 * 4) + 3 * al(B * 4) + al(32 * kH * 4) + al(kH * 32 * 4) + al(3 * 32 * kH * 4) +
             256;
    total += al((size_t)kMaxSplit * kH * kH * 4);
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, total);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        return fail(BH_ERR_NOMEM, "surrogate buffers (%zu bytes)", total);
    }
    s->base = p;
    char* c = (char*)p;
    auto take = [&c](size_t n) {
        void* r = c;
        c += al(n);
        return r;
    };
    s->P = (float*)take(NPARAM * 4);
    s->m = (float*)take(NPARAM * 4);
    s->v = (float*)take(NPARAM * 4);
    s->G = (float*)take(NPARAM * 4);
    s->t.W1ext = (bf16*)take(32 * kH * 2);
    s->t.W2b = (bf16*)take(kH * kH * 2);
    s->t.W3b = (bf16*)take(kH * kH * 2);
    s->t.W4pad = (bf16*)take(kH * 32 * 2);
    s->t.b2r = (float*)take(kH * 4);
    s->t.b3r = (float*)take(kH * 4);
    s->t.b4pad = (float*)take(32 * 4);
    s->pk = (bf16*)take(kPackBytes);
    s->pkf = (float*)((char*)s->pk + PK_BF16 * 2);
    s->trust = (uint8_t*)take(kTrustB * kTrustR);
    s->tacc = (unsigned*)take(2 * kTrustB * kTrustR * 4);
    s->X1 = (bf16*)take(B * 32 * 2);
    s->H1 = (bf16*)take(B * kH * 2);
    s->H2 = (bf16*)take(B * kH * 2);
    s->H3 = (bf16*)take(B * kH * 2);
    s->dY = (bf16*)take(B * 32 * 2);
    s->dZ1 = (bf16*)take(B * kH * 2);
    s->dZ2 = (bf16*)take(B * kH * 2);
    s->dZ3 = (bf16*)take(B * kH * 2);
    s->ones = (bf16*)take(B * 2);
    s->Y = (float*)take(B * 32 * 4);
    s->tgt = (float*)take(B * 4);
    s->esc = (float*)take(B * 4);
    s->capf = (float*)take(B * 4);
    s->part = (float*)take((size_t)kMaxSplit * kH * kH * 4);
    s->gW1ext = (float*)take(32 * kH * 4);
    s->gW4pad = (float*)take(kH * 32 * 4);
    s->cs = (float*)take(3 * 32 * kH * 4);
    s->loss = (float*)c;
    std::vector<bf16> ones(B, (bf16)1.0f);
    HIPCHK(hipMemcpy(s->ones, ones.data(), B * 2, hipMemcpyHostToDevice), "upload");
    HIPCHK(hipMemcpy(s->P, params, NPARAM * 4, hipMemcpyHostToDevice), "upload");
    HIPCHK(hipMemset(s->m, 0, NPARAM * 4), "memset");
    HIPCHK(hipMemset(s->v, 0, NPARAM * 4), "memset");
    HIPCHK(hipMemset(s->G, 0, NPARAM * 4), "memset");
    HIPCHK(hipMemset(s->trust, 0, kTrustB * kTrustR), "memset");
    HIPCHK(repack(s, nullptr), "pack");
    HIPCHK(hipDeviceSynchronize(), "sync");
    *out = s;
    return BH_OK;
}

bh_status bh_surrogate_destroy(bh_surrogate* s) {
    if (!s) return BH_OK;
    (void)hipDeviceSynchronize();
    if (s->base) (void)hipFree(s->base);
    if (s->lab) (void)hipFree(s->lab);
    delete s;
    return BH_OK;
}

bh_status bh_surrogate_params(const bh_surrogate* s, int which, float* host, int64_t count) {
    if (!s || !host || count != NPARAM) return fail(BH_ERR_ARG, "need a handle and %d floats", NPARAM);
    const float* src = which == 0 ? s->P : which == 1 ? s->G : which == 2 ? s->m : which == 3 ? s->v
                                                                                               : nullptr;
    if (!src) return fail(BH_ERR_ARG, "which must be 0 (params), 1 (grad), 2 (m) or 3 (v)");
    HIPCHK(hipDeviceSynchronize(), "sync");
    HIPCHK(hipMemcpy(host, src, NPARAM * 4, hipMemcpyDeviceToHost), "download");
    return BH_OK;
}

bh_status bh_surrogate_set_params(bh_surrogate* s, const float* params, const float* m,
                                  const float* v, int step) {
    if (!s || !params) return fail(BH_ERR_ARG, "need a handle and params");
    HIPCHK(hipDeviceSynchronize(), "sync");
    HIPCHK(hipMemcpy(s->P, params, NPARAM * 4, hipMemcpyHostToDevice), "upload");
    if (m) HIPCHK(hipMemcpy(s->m, m, NPARAM * 4, hipMemcpyHostToDevice), "upload");
    if (v) HIPCHK(hipMemcpy(s->v, v, NPARAM * 4, hipMemcpyHostToDevice), "upload");
    s->step = step;
    // the trust map was validated on the old parameters: renders stop routing
    // to the network until a map is built (or set) for these
    s->trusted = 0;
    ++s->version;
    HIPCHK(repack(s, nullptr), "pack");
    HIPCHK(hipDeviceSynchronize(), "sync");
    return BH_OK;
}

bh_status bh_surrogate_train_step(bh_surrogate* s, const double* b, const double* r0,
                                  const double* phi_exit, const uint8_t* captured, int64_t n,
                                  const bh_adam* hp, float* loss_out, void* stream) {
    if (!s || !b || !r0 || !phi_exit || !captured)
        return fail(BH_ERR_ARG, "handle and batch arrays are required");
    if (n < 32 || n % 32 != 0 || n > s->max_batch)
        return fail(BH_ERR_ARG, "batch must be a multiple of 32 in [32, max_batch]");
    hipStream_t st = (hipStream_t)stream;
    const int nb = (int)((n + 255) / 256);
    k_zero<<<1, 64, 0, st>>>(s->loss, 1);
    k_prep<<<nb, 256, 0, st>>>(n, b, r0, phi_exit, captured, s->X1, s->tgt, s->esc, s->capf);
    HIPCHK(hipGetLastError(), "prep");
    const int N = (int)n;
    // forward
    GemmArgs g = gemm_args(s->X1, 32, 1, s->t.W1ext, kH, 1, N, kH, 32);
    g.relu = 1; g.Cb = s->H1; g.cb_m = kH; g.cb_n = 1;
    HIPCHK(gemm(g, st, s->part), "gemm");
    g = gemm_args(s->H1, kH, 1, s->t.W2b, kH, 1, N, kH, kH);
    g.bias = s->t.b2r; g.relu = 1; g.Cb = s->H2; g.cb_m = kH; g.cb_n = 1;
    HIPCHK(gemm(g, st, s->part), "gemm");
    g = gemm_args(s->H2, kH, 1, s->t.W3b, kH, 1, N, kH, kH);
    g.bias = s->t.b3r; g.relu = 1; g.Cb = s->H3; g.cb_m = kH; g.cb_n = 1;
    HIPCHK(gemm(g, st, s->part), "gemm");
    g = gemm_args(s->H3, kH, 1, s->t.W4pad, 32, 1, N, 32, kH);
    g.bias = s->t.b4pad; g.Cf = s->Y; g.cf_m = 32; g.cf_n = 1;
    HIPCHK(gemm(g, st, s->part), "gemm");
    k_loss<<<nb, 256, 0, st>>>(n, s->Y, s->tgt, s->esc, s->capf, s->dY, s->loss);
    HIPCHK(hipGetLastError(), "loss");
    // backward: dZ3 = (dY W4^T) * [H3 > 0]
    g = gemm_args(s->dY, 32, 1, s->t.W4pad, 1, 32, N, kH, 32);
    g.mask = s->H3; g.mk_m = kH; g.mk_n = 1; g.Cb = s->dZ3; g.cb_m = kH; g.cb_n = 1;
    HIPCHK(gemm(g, st, s->part), "gemm");
    g = gemm_args(s->H3, 1, kH, s->dY, 32, 1, kH, 32, N);  // gW4pad = H3^T dY
    g.Cf = s->gW4pad; g.cf_m = 32; g.cf_n = 1;
    HIPCHK(gemm(g, st, s->part), "gemm");
    g = gemm_args(s->dZ3, kH, 1, s->t.W3b, 1, kH, N, kH, kH);  // dZ2
    g.mask = s->H2; g.mk_m = kH; g.mk_n = 1; g.Cb = s->dZ2; g.cb_m = kH; g.cb_n = 1;
    HIPCHK(gemm(g, st, s->part), "gemm");
    g = gemm_args(s->H2, 1, kH, s->dZ3, kH, 1, kH, kH, N);  // gW3 = H2^T dZ3
    g.Cf = s->G + OFF_W3; g.cf_m = kH; g.cf_n = 1;
    HIPCHK(gemm(g, st, s->part), "gemm");
    g = gemm_args(s->dZ2, kH, 1, s->t.W2b, 1, kH, N, kH, kH);  // dZ1
    g.mask = s->H1; g.mk_m = kH; g.mk_n = 1; g.Cb = s->dZ1; g.cb_m = kH; g.cb_n = 1;
    HIPCHK(gemm(g, st, s->part), "gemm");
    g = gemm_args(s->H1, 1, kH, s->dZ2, kH, 1, kH, kH, N);  // gW2 = H1^T dZ2
    g.Cf = s->G + OFF_W2; g.cf_m = kH; g.cf_n = 1;
    HIPCHK(gemm(g, st, s->part), "gemm");
    g = gemm_args(s->X1, 1, 32, s->dZ1, kH, 1, 32, kH, N);  // gW1ext = X1^T dZ1
    g.Cf = s->gW1ext; g.cf_m = kH; g.cf_n = 1;
    HIPCHK(gemm(g, st, s->part), "gemm");
    // bias gradients: column sums through a ones operand (row 0 of the result)
    const bf16* cols[3] = {s->dZ2, s->dZ3, s->dY};
    const int ncol[3] = {kH, kH, 32};
    for (int q = 0; q < 3; ++q) {
        g = gemm_args(s->ones, 0, 1, cols[q], ncol[q], 1, 32, ncol[q], N);
        g.Cf = s->cs + q * 32 * kH; g.cf_m = ncol[q]; g.cf_n = 1;
        HIPCHK(gemm(g, st, s->part), "gemm");
    }
    k_assemble<<<1, kH, 0, st>>>(s->gW1ext, s->gW4pad, s->cs, s->cs + 32 * kH, s->cs + 2 * 32 * kH,
                                 s->G);
    HIPCHK(hipGetLastError(), "assemble");
    if (hp && hp->lr > 0.0f) {
        s->step += 1;
        s->trusted = 0;  // new parameters: the trust map no longer applies
        ++s->version;
        const float c1 = 1.0f / (1.0f - powf(hp->beta1, (float)s->step));
        const float c2 = 1.0f / (1.0f - powf(hp->beta2, (float)s->step));
        k_adam<<<(NPARAM + 255) / 256, 256, 0, st>>>(NPARAM, s->P, s->G, s->m, s->v, hp->lr,
                                                     hp->beta1, hp->beta2, hp->eps, c1, c2);
        HIPCHK(hipGetLastError(), "adam");
        HIPCHK(repack(s, st), "pack");
    }
    if (loss_out) HIPCHK(hipMemcpyAsync(loss_out, s->loss, 4, hipMemcpyDeviceToDevice, st), "copy");
    return BH_OK;
}

bh_status bh_surrogate_infer(const bh_surrogate* s, const double* b, const double* r0, int64_t n,
                             float* y, double* phi_pred, void* stream) {
    if (!s || !b || !r0 || n < 0) return fail(BH_ERR_ARG, "handle, b and r0 are required");
    if (n == 0) return BH_OK;
    const size_t lds = kPackBytes;
    int64_t g = (int64_t)s->cus * 2, need = (n + 255) / 256;
    if (g > need) g = need;
    k_infer<<<(unsigned)g, kInferThreads, lds, (hipStream_t)stream>>>(s->pk, n, b, r0, y, phi_pred);
    HIPCHK(hipGetLastError(), "infer");
    return BH_OK;
}

bh_status bh_surrogate_labels(bh_surrogate* s, const double* b, const double* r0, int64_t n,
                              double* phi_exit, uint8_t* captured, void* stream) {
    if (!s || !b || !r0 || !phi_exit || !captured || n < 0)
        return fail(BH_ERR_ARG, "handle and arrays are required");
    if (n == 0) return BH_OK;
    hipStream_t st = (hipStream_t)stream;
    if (n > s->lab_cap) {
        HIPCHK(hipStreamSynchronize(st), "sync");
        if (s->lab) (void)hipFree(s->lab);
        s->lab = nullptr;
        s->lab_cap = 0;
        if (hipMalloc(&s->lab, (size_t)n * 6 * 8) != hipSuccess) {
            (void)hipGetLastError();
            return fail(BH_ERR_NOMEM, "label scratch");
        }
        s->lab_cap = n;
    }
    double* o = (double*)s->lab;
    double* d = o + 3 * n;
    k_pair_rays<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, b, r0, o, d);
    HIPCHK(hipGetLastError(), "pair rays");
    bh_scene sc;
    memset(&sc, 0, sizeof sc);
    sc.M = 1.0;
    sc.r_sky = 1000.0;
    sc.checker_deg = 10.0;
    bh_options opt;
    bh_default_options(&opt);
    opt.analytic_capture = 0;  // labels come from integration
    bh_ray_out out;
    memset(&out, 0, sizeof out);
    out.cls = captured;  // class codes; converted below
    out.phi_end = phi_exit;
    bh_status stt = bh_trace_rays(o, d, n, &sc, &opt, &out, stream);
    if (stt != BH_OK) return stt;
    k_labels_finish<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, captured, phi_exit);
    HIPCHK(hipGetLastError(), "labels");
    return BH_OK;
}

bh_status bh_surrogate_build_trust(bh_surrogate* s, const double* b, const double* r0,
                                   const double* phi_true, int64_t n, float max_err,
                                   int min_count, float* y_scratch, double* phi_scratch,
                                   void* stream) {
    if (!s || !b || !r0 || !phi_true || !y_scratch || !phi_scratch || n < 1 || min_count < 1)
        return fail(BH_ERR_ARG, "handle, arrays, n >= 1 and min_count >= 1 are required");
    hipStream_t st = (hipStream_t)stream;
    bh_status stt = bh_surrogate_infer(s, b, r0, n, y_scratch, phi_scratch, stream);
    if (stt != BH_OK) return stt;
    HIPCHK(hipMemsetAsync(s->tacc, 0, 2 * kTrustB * kTrustR * 4, st), "memset");
    k_trust_acc<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, b, r0, phi_true, phi_scratch,
                                                             y_scratch, s->tacc,
                                                             s->tacc + kTrustB * kTrustR);
    k_trust_fin<<<(kTrustB * kTrustR + 255) / 256, 256, 0, st>>>(s->tacc, s->tacc + kTrustB * kTrustR,
                                                                 max_err, (unsigned)min_count,
                                                                 s->trust);
    HIPCHK(hipGetLastError(), "trust");
    s->trusted = 1;
    ++s->version;
    return BH_OK;
}

bh_status bh_surrogate_trust(const bh_surrogate* s, uint8_t* host_map, int64_t count) {
    if (!s || !host_map || count != kTrustB * kTrustR)
        return fail(BH_ERR_ARG, "map needs %d bytes", kTrustB * kTrustR);
    HIPCHK(hipDeviceSynchronize(), "sync");
    HIPCHK(hipMemcpy(host_map, s->trust, count, hipMemcpyDeviceToHost), "download");
    return BH_OK;
}

bh_status bh_surrogate_set_trust(bh_surrogate* s, const uint8_t* host_map, int64_t count) {
    if (!s || !host_map || count != kTrustB * kTrustR)
        return fail(BH_ERR_ARG, "map needs %d bytes", kTrustB * kTrustR);
    HIPCHK(hipDeviceSynchronize(), "sync");
    HIPCHK(hipMemcpy(s->trust, host_map, count, hipMemcpyHostToDevice), "upload");
    s->trusted = 1;
    ++s->version;
    return BH_OK;
}

}  // extern "C"

namespace bh {
const uint8_t* surrogate_trust(const bh_surrogate* s) { return s && s->trusted ? s->trust : nullptr; }
unsigned surrogate_version(const bh_surrogate* s) { return s ? s->version : 0u; }
const void* surrogate_pack(const bh_surrogate* s) { return s ? s->pk : nullptr; }
}  // namespace bh
