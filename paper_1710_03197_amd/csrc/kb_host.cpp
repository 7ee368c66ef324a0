// Host-side float64 mathematics of the plan: the Kaiser-Bessel interpolation
// kernel (the alternative kernel the paper lists in Section 4.1, item 6, used
// in place of its default min-max interpolator), its Fourier transform for
// the scaling stage S (Section 2.1 "Scaling"), the per-tap polynomial fit the
// GPU evaluates, FFT twiddles and the radix schedule of the oversampled FFT
// (Section 2.1 "Oversampled FFT").
#include <cmath>
#include <cstring>

#include "nufft_internal.h"

namespace nufft {

namespace {
constexpr double kPi = 3.14159265358979323846;
}

// Beatty, Nishimura and Pauly's shape parameter for width J and
// oversampling sigma.
double kb_beta(int J, double sigma) {
    double a = (double(J) / sigma) * (sigma - 0.5);
    return kPi * std::sqrt(a * a - 0.8);
}

// I0 by its power series; every term is positive, so there is no
// cancellation for the arguments used here (z <= beta < 60).
double kb_i0(double z) {
    double q = 0.25 * z * z, term = 1.0, sum = 1.0;
    for (int k = 1; k < 1000; ++k) {
        term *= q / (double(k) * double(k));
        sum += term;
        if (term < 1e-19 * sum) break;
    }
    return sum;
}

static double i1_over_z(double z) {
    double q = 0.25 * z * z, term = 0.5, sum = 0.5;
    for (int k = 1; k < 1000; ++k) {
        term *= q / (double(k) * double(k + 1));
        sum += term;
        if (term < 1e-19 * sum) break;
    }
    return sum;
}

double kb_phi(double t, int J, double beta) {
    double r = 2.0 * t / J;
    double s = 1.0 - r * r;
    if (s < 0.0) return 0.0;
    return kb_i0(beta * std::sqrt(s));
}

double kb_dphi(double t, int J, double beta) {
    double r = 2.0 * t / J;
    double s = 1.0 - r * r;
    if (s < 0.0) return 0.0;
    return -(4.0 * beta * beta * t / (double(J) * J)) * i1_over_z(beta * std::sqrt(s));
}

// Fourier transform of the kernel on [-J/2, J/2]:
// J sinh(sqrt(b^2 - (pi J xi)^2)) / sqrt(b^2 - (pi J xi)^2), sin form past the root.
double kb_ft(double xi, int J, double beta) {
    double a = kPi * J * xi;
    double r = beta * beta - a * a;
    if (r > 0.0) {
        double q = std::sqrt(r);
        return J * std::sinh(q) / q;
    }
    if (r < 0.0) {
        double q = std::sqrt(-r);
        return J * std::sin(q) / q;
    }
    return double(J);
}

// Chebyshev interpolant of g on [-1, 1] at deg+1 first-kind nodes, returned
// as monomial coefficients in z (float64).
template <class F>
static void cheb_fit(F g, int deg, double *mono) {
    int n = deg + 1;
    double a[kMaxPolyDeg + 1];
    double fz[kMaxPolyDeg + 1];
    double zk[kMaxPolyDeg + 1];
    for (int k = 0; k < n; ++k) {
        zk[k] = std::cos(kPi * (k + 0.5) / n);
        fz[k] = g(zk[k]);
    }
    for (int m = 0; m < n; ++m) {
        double s = 0.0;
        for (int k = 0; k < n; ++k) s += fz[k] * std::cos(m * kPi * (k + 0.5) / n);
        a[m] = s * 2.0 / n;
    }
    a[0] *= 0.5;
    // T_m as monomials: T_0 = 1, T_1 = z, T_{m+1} = 2 z T_m - T_{m-1}.
    double Tm1[kMaxPolyDeg + 2] = {0}, Tm[kMaxPolyDeg + 2] = {0}, Tn[kMaxPolyDeg + 2];
    for (int k = 0; k <= deg; ++k) mono[k] = 0.0;
    Tm1[0] = 1.0;  // T_0
    Tm[1] = 1.0;   // T_1
    mono[0] += a[0];
    if (deg >= 1) mono[1] += a[1];
    for (int m = 2; m <= deg; ++m) {
        for (int k = 0; k <= deg; ++k) {
            double v = -Tm1[k];
            if (k >= 1) v += 2.0 * Tm[k - 1];
            Tn[k] = v;
        }
        for (int k = 0; k <= deg; ++k) mono[k] += a[m] * Tn[k];
        std::memcpy(Tm1, Tm, sizeof(Tm));
        std::memcpy(Tm, Tn, sizeof(Tm));
    }
}

static double horner64(const double *c, int deg, double z) {
    double v = c[deg];
    for (int k = deg - 1; k >= 0; --k) v = v * z + c[k];
    return v;
}

// Fit w_j(z) = phi(t), t = (z+1)/2 + J/2 - 1 - j, for every tap j, with
// the lowest degree whose float64 error is below `tol` (relative to the peak
// of the fitted function).
template <class F>
static int fit_taps(int J, F fn, double peak, double tol, std::vector<float> *out) {
    for (int deg = 4; deg <= kMaxPolyDeg; ++deg) {
        std::vector<double> c(size_t(J) * (deg + 1));
        double err = 0.0;
        for (int j = 0; j < J; ++j) {
            auto g = [&](double z) { return fn((z + 1.0) * 0.5 + 0.5 * J - 1.0 - j); };
            cheb_fit(g, deg, &c[size_t(j) * (deg + 1)]);
            for (int s = 0; s <= 400; ++s) {
                double z = -1.0 + 2.0 * s / 400.0;
                double e = std::fabs(horner64(&c[size_t(j) * (deg + 1)], deg, z) - g(z));
                if (e > err) err = e;
            }
        }
        if (err <= tol * peak) {
            out->resize(c.size());
            for (size_t i = 0; i < c.size(); ++i) (*out)[i] = float(c[i]);
            return deg;
        }
    }
    return -1;
}

bool kb_fit(int J, double beta, AxisKernel *out) {
    const double p0 = kb_phi(0.0, J, beta);
    out->beta = beta;
    auto phi = [&](double t) { return kb_phi(t, J, beta); };
    auto dphi = [&](double t) { return kb_dphi(t, J, beta); };
    double dpeak = 0.0;
    for (int s = 0; s <= 2000; ++s) {
        double t = -0.5 * J + J * s / 2000.0;
        dpeak = std::fmax(dpeak, std::fabs(dphi(t)));
    }
    out->deg = fit_taps(J, phi, p0, 2e-9, &out->coef);
    out->deg_d = fit_taps(J, dphi, dpeak, 2e-9, &out->dcoef);
    return out->deg > 0 && out->deg_d > 0;
}

void kb_eval_fit(const AxisKernel &k, int J, float f, float *w, float *dw) {
    float z = 2.0f * f - 1.0f;
    for (int j = 0; j < J; ++j) {
        const float *c = &k.coef[size_t(j) * (k.deg + 1)];
        float v = c[k.deg];
        for (int q = k.deg - 1; q >= 0; --q) v = std::fmaf(v, z, c[q]);
        w[j] = v;
        if (dw) {
            const float *cd = &k.dcoef[size_t(j) * (k.deg_d + 1)];
            float u = cd[k.deg_d];
            for (int q = k.deg_d - 1; q >= 0; --q) u = std::fmaf(u, z, cd[q]);
            dw[j] = u;
        }
    }
}

std::vector<float> coef_rows(const std::vector<float> &coef, int J, int deg, int jp, int *nq) {
    const int rows = (deg + 1 + 1) / 2 * 2;
    std::vector<float> out(size_t(rows) * jp, 0.0f);
    for (int r = 0; r < rows; ++r) {
        const int q = rows - 1 - r;
        if (q > deg) continue;
        for (int j = 0; j < J; ++j) out[size_t(r) * jp + j] = coef[size_t(j) * (deg + 1) + q];
    }
    *nq = rows;
    return out;
}

std::vector<float> kb_scaling(int N, int K, int J, double beta) {
    std::vector<float> s(N);
    for (int i = 0; i < N; ++i) s[i] = float(1.0 / kb_ft(double(i - N / 2) / K, J, beta));
    return s;
}

std::vector<float2> twiddles(int K) {
    std::vector<float2> tw(K);
    for (int e = 0; e < K; ++e) {
        double ang = 2.0 * kPi * double(e) / double(K);
        tw[e] = make_float2(float(std::cos(ang)), float(-std::sin(ang)));
    }
    return tw;
}

bool radix_plan(int K, RadixPlan *rp) {
    rp->n = 0;
    int rem = K;
    const int order[] = {8, 4, 2, 3, 5};
    for (int r : order) {
        while (rem % r == 0) {
            if (rp->n >= kMaxPasses) return false;
            rp->r[rp->n++] = r;
            rem /= r;
        }
    }
    return rem == 1;
}

}  // namespace nufft
