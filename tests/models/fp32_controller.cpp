// A scalar model of the FP32 integrator's step-size controller, for the
// design test tests/test_fp32_controller_model.py (not the oracle, and not
// part of the library).  Each ray is integrated in the scaled variable
// v = 3M u of Eq. (1), v'' + v = v^2, with the Dormand-Prince 5(4) step in
// float (the published tableau), the error norm max_i |e_i| / (atol + rtol
// max(|y_i|, |y_new,i|)), the controller factor s err^(-1/5) clamped to
// [0.2, 5] with no growth after a rejection, steps shortened to land on
// disk-plane crossings, and the sky crossing refined by Newton re-steps
// until the last correction is below 1e-3 rad.  Each ray's tolerance grows
// with its distance from the critical impact parameter as the GPU's FP32
// rays' do: rtol and atol times f = clamp(|b - 3 sqrt(3) M| / 0.5 M, 1,
// growth), first step h0 f^(1/5).  The reference run uses double at rtol
// 1e-12 with safety 0.9.
//
// stdin: "v0 w0 phi1" per ray (scaled start value and slope, first crossing).
// argv: safety h0 rtol growth [...]; one JSON line per variant on stdout:
// mean accepted, rejected and Newton steps per ray, the largest exit azimuth
// error and disk-radius error against the reference, and the number of class
// differences, all of them and those outside the disk-edge zone (a DISK side
// whose radius lies within 1e-4 r of an edge).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

namespace {

constexpr double kPi = 3.14159265358979323846;
// sky at 1000 M, disk 6-30 M, in v = 3M / r
constexpr double kVsky = 3.0 / 1000.0, kVin = 3.0 / 6.0, kVout = 3.0 / 30.0;

struct Ray { double v0, w0, phi1; };

// Tolerance factor of a ray (M = 1): 9 / b^2 = w^2 + v^2 - (2/3) v^3.
double growth_of(const Ray& r, double growth) {
    const double b = 3.0 / std::sqrt(r.w0 * r.w0 + r.v0 * r.v0 * (1.0 - 2.0 * r.v0 / 3.0));
    return std::fmin(std::fmax(std::fabs(b - 3.0 * std::sqrt(3.0)) / 0.5, 1.0), growth);
}
bool near_edge(double r) {
    return std::fabs(r - 6.0) < 1e-4 * 6.0 || std::fabs(r - 30.0) < 1e-4 * 30.0;
}
struct Res { int cls; double phi, r; int acc, rej, newt; };

template <typename T> T G(T x) { return std::fma(x, x, -x); }

template <typename T>
void step(T v, T w, T g1, T h, T& vn, T& wn, T& g7, T& ev, T& ew) {
    const double a21 = 1.0 / 5, a31 = 3.0 / 40, a32 = 9.0 / 40, a41 = 44.0 / 45, a42 = -56.0 / 15,
                 a43 = 32.0 / 9, a51 = 19372.0 / 6561, a52 = -25360.0 / 2187,
                 a53 = 64448.0 / 6561, a54 = -212.0 / 729, a61 = 9017.0 / 3168,
                 a62 = -355.0 / 33, a63 = 46732.0 / 5247, a64 = 49.0 / 176,
                 a65 = -5103.0 / 18656;
    const double b1 = 35.0 / 384, b3 = 500.0 / 1113, b4 = 125.0 / 192, b5 = -2187.0 / 6784,
                 b6 = 11.0 / 84;
    const double e1 = 71.0 / 57600, e3 = -71.0 / 16695, e4 = 71.0 / 1920,
                 e5 = -17253.0 / 339200, e6 = 22.0 / 525, e7 = -1.0 / 40;
    // stage values in the standard form: v_k = v + h sum a w_j, w_k = w + h sum a g_j
    T k1v = w, k1w = g1;
    T v2 = v + h * T(a21) * k1v, w2 = w + h * T(a21) * k1w;
    T k2v = w2, k2w = G(v2);
    T v3 = v + h * (T(a31) * k1v + T(a32) * k2v), w3 = w + h * (T(a31) * k1w + T(a32) * k2w);
    T k3v = w3, k3w = G(v3);
    T v4 = v + h * (T(a41) * k1v + T(a42) * k2v + T(a43) * k3v);
    T w4 = w + h * (T(a41) * k1w + T(a42) * k2w + T(a43) * k3w);
    T k4v = w4, k4w = G(v4);
    T v5 = v + h * (T(a51) * k1v + T(a52) * k2v + T(a53) * k3v + T(a54) * k4v);
    T w5 = w + h * (T(a51) * k1w + T(a52) * k2w + T(a53) * k3w + T(a54) * k4w);
    T k5v = w5, k5w = G(v5);
    T v6 = v + h * (T(a61) * k1v + T(a62) * k2v + T(a63) * k3v + T(a64) * k4v + T(a65) * k5v);
    T w6 = w + h * (T(a61) * k1w + T(a62) * k2w + T(a63) * k3w + T(a64) * k4w + T(a65) * k5w);
    T k6v = w6, k6w = G(v6);
    vn = v + h * (T(b1) * k1v + T(b3) * k3v + T(b4) * k4v + T(b5) * k5v + T(b6) * k6v);
    wn = w + h * (T(b1) * k1w + T(b3) * k3w + T(b4) * k4w + T(b5) * k5w + T(b6) * k6w);
    T k7v = wn, k7w = G(vn);
    g7 = k7w;
    ev = h * (T(e1) * k1v + T(e3) * k3v + T(e4) * k4v + T(e5) * k5v + T(e6) * k6v + T(e7) * k7v);
    ew = h * (T(e1) * k1w + T(e3) * k3w + T(e4) * k4w + T(e5) * k5w + T(e6) * k6w + T(e7) * k7w);
}

template <typename T>
Res trace(const Ray& r, double safety, double h0, double rtol_d, double ntol) {
    Res o{3, 0.0, 0.0, 0, 0, 0};
    T v = T(r.v0), w = T(r.w0), g = G(v), h = T(h0), phi = T(0), phik = T(r.phi1);
    const T rtol = T(rtol_d), atol = T(rtol_d * kVsky);
    bool rej = false;
    for (int it = 0; it < 100000; ++it) {
        T ht = h;
        bool land = false;
        if (phi + ht >= phik) { ht = phik - phi; land = true; }
        T vn, wn, gn, ev, ew;
        step<T>(v, w, g, ht, vn, wn, gn, ev, ew);
        const T sv = rtol * std::fmax(std::fabs(v), std::fabs(vn)) + atol;
        const T sw = rtol * std::fmax(std::fabs(w), std::fabs(wn)) + atol;
        const bool fits = std::fabs(ev) <= sv && std::fabs(ew) <= sw;
        const double err = std::fmax(std::fabs((double)ev / sv), std::fabs((double)ew / sw));
        double fac = safety * std::pow(err, -0.2);
        if (!(fac == fac)) fac = 0.2;
        if (!fits) {
            ++o.rej;
            rej = true;
            h = T(std::fmin(1.0, ht * std::fmax(fac, 0.2)));
            continue;
        }
        ++o.acc;
        fac = std::fmin(std::fmax(fac, 0.2), rej ? 1.0 : 5.0);
        const T phin = land ? phik : phi + ht;
        if (land && vn >= T(kVout) && vn <= T(kVin)) {
            o.cls = 2; o.r = 3.0 / (double)vn; o.phi = (double)phin;
            return o;
        }
        if (vn >= T(1.5)) { o.cls = 1; o.phi = (double)phin; return o; }
        if (vn <= T(kVsky) && wn < T(0)) {
            T hh = ht, vv = vn, ww = wn;
            for (int k = 0; k < 4; ++k) {
                const T dh = (vv - T(kVsky)) / ww;
                hh -= dh;
                if (std::fabs((double)dh) < ntol || k == 3) break;
                T a, b, c;
                step<T>(v, w, g, hh, vv, ww, a, b, c);
                ++o.newt;
            }
            o.cls = 0; o.phi = (double)(phi + hh);
            return o;
        }
        if (land) phik += T(kPi);
        v = vn; w = wn; g = gn; phi = phin;
        if (!land) h = T(std::fmin(1.0, ht * fac));
        rej = false;
        if (phi > 8 * kPi) return o;
    }
    return o;
}

}  // namespace

int main(int argc, char** argv) {
    std::vector<Ray> rays;
    Ray r;
    while (std::scanf("%lf %lf %lf", &r.v0, &r.w0, &r.phi1) == 3) rays.push_back(r);
    std::vector<Res> ref(rays.size());
    for (size_t i = 0; i < rays.size(); ++i) ref[i] = trace<double>(rays[i], 0.9, 1e-2, 1e-12, 1e-15);
    for (int a = 1; a + 3 < argc; a += 4) {
        const double s = std::atof(argv[a]), h0 = std::atof(argv[a + 1]), rt = std::atof(argv[a + 2]);
        const double growth = std::atof(argv[a + 3]);
        long acc = 0, rej = 0, newt = 0, mism = 0, mism_out = 0;
        double emax = 0.0, rmax = 0.0;
        for (size_t i = 0; i < rays.size(); ++i) {
            const double f = growth_of(rays[i], growth);
            const Res o = trace<float>(rays[i], s, f > 1.0 ? h0 * std::pow(f, 0.2) : h0, rt * f, 1e-3);
            acc += o.acc; rej += o.rej; newt += o.newt;
            if (o.cls != ref[i].cls) {
                ++mism;
                const double rd = ref[i].cls == 2 ? ref[i].r : o.r;
                if (!(((ref[i].cls == 2) != (o.cls == 2)) && near_edge(rd))) ++mism_out;
                continue;
            }
            if (o.cls == 0) emax = std::fmax(emax, std::fabs(o.phi - ref[i].phi));
            if (o.cls == 2) rmax = std::fmax(rmax, std::fabs(o.r / ref[i].r - 1.0));
        }
        const double n = (double)rays.size();
        std::printf("{\"safety\": %g, \"h0\": %g, \"rtol\": %g, \"growth\": %g, \"accepted\": %.4f, "
                    "\"rejected\": %.4f, \"newton\": %.4f, \"max_phi_err\": %.3e, \"max_r_rel\": %.3e, "
                    "\"class_diff\": %ld, \"class_diff_outside_edge_zone\": %ld}\n",
                    s, h0, rt, growth, acc / n, rej / n, newt / n, emax, rmax, mism, mism_out);
    }
    return 0;
}
