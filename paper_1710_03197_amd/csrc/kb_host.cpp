// Host-side float64 mathematics of the plan: the Kaiser-Bessel interpolation
// kernel (the alternative kernel the paper lists in Section 4.1, item 6, used
// in place of its default min-max interpolator), its Fourier transform for
// the scaling stage S (Section 2.1 "Scaling"), the per-tap polynomial fit the
// GPU evaluates, FFT twiddles and the radix schedule of the oversampled FFT
// (Section 2.1 "Oversampled FFT").
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>

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

// Fit w_j(z) = fn(j, f), f = (z+1)/2 the window's fractional offset, for
// every tap j, with the lowest degree whose float64 error is below `tol`
// (relative to the peak of the fitted function).
template <class F>
static int fit_taps_jf(int J, F fn, double peak, double tol, std::vector<float> *out) {
    for (int deg = 4; deg <= kMaxPolyDeg; ++deg) {
        std::vector<double> c(size_t(J) * (deg + 1));
        double err = 0.0;
        for (int j = 0; j < J; ++j) {
            auto g = [&](double z) { return fn(j, (z + 1.0) * 0.5); };
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

// The Kaiser-Bessel taps are one function of the tap offset
// t = f + J/2 - 1 - j.
template <class F>
static int fit_taps(int J, F fn, double peak, double tol, std::vector<float> *out) {
    return fit_taps_jf(J, [&](int j, double f) { return fn(f + 0.5 * J - 1.0 - j); }, peak, tol, out);
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

// ---- min-max interpolator (Section 2.1 "Interpolation", after Fessler and
// Sutton).  With the scaling factors s_n = g(n + 1/2), g(m) = 1/Phi(m/K),
// n in [-N/2, N/2), the worst-case-optimal coefficients c = T^-1 r factor as
// c_j = e^{i gamma t_j / 2} c'_j with c' real:
//   c' = T'^-1 R'(t),  T'_jl = sum_m g(m)^2 cos(gamma (j - l) m),
//   R'(t)_j = sum_m g(m) cos(gamma t_j m),  gamma = 2 pi / K,
// m over the symmetric half-integers n + 1/2, t_j = f + J/2 - 1 - j.  The
// phase e^{i gamma t_j / 2} = e^{i omega / 2} e^{-i pi k / K} (k = k0 + j
// unwrapped) is applied by the kernels: e^{-i pi k / K} on the grid (FFT
// passes, half_phase) with a sign for taps that wrap past K, e^{i omega / 2}
// per sample.
std::vector<float> minmax_scaling(int N, int K, int J, double beta) {
    std::vector<float> s(N);
    for (int i = 0; i < N; ++i) s[i] = float(1.0 / kb_ft((double(i - N / 2) + 0.5) / K, J, beta));
    return s;
}

std::vector<float2> half_phase(int K) {
    std::vector<float2> p(K);
    for (int k = 0; k < K; ++k) {
        const double a = -kPi * double(k) / double(K);
        p[k] = make_float2(float(std::cos(a)), float(std::sin(a)));
    }
    return p;
}

// Solve A x = b (n x n, row-major) by Gaussian elimination with partial
// pivoting; A and b are overwritten.
static bool solve_dense(int n, std::vector<double> &A, std::vector<double> &b) {
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(A[size_t(r) * n + c]) > std::fabs(A[size_t(piv) * n + c])) piv = r;
        if (A[size_t(piv) * n + c] == 0.0) return false;
        if (piv != c) {
            for (int k = 0; k < n; ++k) std::swap(A[size_t(c) * n + k], A[size_t(piv) * n + k]);
            std::swap(b[c], b[piv]);
        }
        for (int r = c + 1; r < n; ++r) {
            const double f = A[size_t(r) * n + c] / A[size_t(c) * n + c];
            for (int k = c; k < n; ++k) A[size_t(r) * n + k] -= f * A[size_t(c) * n + k];
            b[r] -= f * b[c];
        }
    }
    for (int c = n - 1; c >= 0; --c) {
        double v = b[c];
        for (int k = c + 1; k < n; ++k) v -= A[size_t(c) * n + k] * b[k];
        b[c] = v / A[size_t(c) * n + c];
    }
    return true;
}

bool minmax_fit(int N, int K, int J, double beta, AxisKernel *out) {
    std::vector<double> g(N), m(N);
    for (int i = 0; i < N; ++i) {
        m[i] = double(i - N / 2) + 0.5;
        g[i] = 1.0 / kb_ft(m[i] / K, J, beta);
    }
    const double gam = 2.0 * kPi / K;
    std::vector<double> T(size_t(J) * J);
    for (int j = 0; j < J; ++j)
        for (int l = 0; l < J; ++l) {
            double v = 0.0;
            for (int i = 0; i < N; ++i) v += g[i] * g[i] * std::cos(gam * (j - l) * m[i]);
            T[size_t(j) * J + l] = v;
        }
    bool ok = true;
    // c'(f) for all taps at once, memoised: the fit asks for every tap at the
    // same offsets
    std::map<double, std::vector<double>> memo;
    auto coef = [&](int j, double f) {
        auto it = memo.find(f);
        if (it == memo.end()) {
            std::vector<double> A = T, r(J);
            for (int l = 0; l < J; ++l) {
                const double t = f + 0.5 * J - 1.0 - l;
                double v = 0.0;
                for (int i = 0; i < N; ++i) v += g[i] * std::cos(gam * t * m[i]);
                r[l] = v;
            }
            if (!solve_dense(J, A, r)) ok = false;
            it = memo.emplace(f, std::move(r)).first;
        }
        return it->second[j];
    };
    double peak = 0.0;
    for (int s = 0; s <= 200; ++s)
        for (int j = 0; j < J; ++j) peak = std::fmax(peak, std::fabs(coef(j, s / 200.0)));
    out->beta = beta;
    out->deg = fit_taps_jf(J, coef, peak, 2e-9, &out->coef);
    // no derivative fit: the trajectory gradient is Kaiser-Bessel only
    out->deg_d = 1;
    out->dcoef.assign(size_t(J) * 2, 0.0f);
    return ok && out->deg > 0;
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

bool radix_plan(int K, RadixPlan *rp, int schedule) {
    rp->n = 0;
    int rem = K;
    // radices taken greedily in this order (schedule 3: schedule 0's passes
    // run in reverse)
    static const int orders[3][5] = {{8, 4, 2, 3, 5}, {4, 8, 2, 3, 5}, {3, 5, 8, 4, 2}};
    if (schedule < 0 || schedule > 3) return false;
    for (int r : orders[schedule == 3 ? 0 : schedule]) {
        while (rem % r == 0) {
            if (rp->n >= kMaxPasses) return false;
            rp->r[rp->n++] = r;
            rem /= r;
        }
    }
    if (rem != 1) return false;
    if (schedule == 3) std::reverse(rp->r, rp->r + rp->n);
    auto magic = [](int D) { return D > 1 ? 0xFFFFFFFFu / unsigned(D) + 1u : 0u; };
    int Ns = 1;
    for (int p = 0; p < rp->n; ++p) {
        rp->span[p] = K / (Ns * rp->r[p]);
        rp->m_ns[p] = magic(Ns);
        rp->m_nbl[p] = magic(K / rp->r[p]);
        Ns *= rp->r[p];
    }
    return true;
}

}  // namespace nufft
