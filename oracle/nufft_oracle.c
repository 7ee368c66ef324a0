/*
 * FP64 CPU oracle for the NUFFT pair A = V F S and A^H = S^H F^H V^H
 * (paper Section 2.1: Eq. A = VFS; scaling, oversampled FFT with zero
 * padding, interpolation; Section 2.1 "Adjoint PyNUFFT", Eq. A^H = S^H F^H V^H).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU library is checked against.  It shares no code, header or table with the
 * GPU library; only tests, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.
 *
 * Conventions (readings of points the paper leaves open):
 *  - C order (last axis fastest), as the paper's C-order CSR interpolator.
 *  - Image index i_a in [0, N_a) stands for n_a = i_a - N_a/2; it lands on grid
 *    index q_a = n_a mod K_a (zero padding without any index list).
 *  - Forward kernel e^{-i omega.n}; both FFTs unnormalised; the adjoint is the
 *    exact conjugate transpose of the forward.
 *  - Interpolation kernel: Kaiser-Bessel, phi(t) = I0(beta*sqrt(1-(2t/J)^2)) for
 *    |t| <= J/2, with Beatty's beta = pi*sqrt((J/sigma)^2 (sigma-1/2)^2 - 0.8),
 *    sigma_a = K_a/N_a.  The paper's default is the min-max kernel; it lists
 *    Kaiser-Bessel among the alternatives (Section 4.1, item 6).
 *  - Scaling S(n) = prod_a 1/Phi_a(n_a/K_a), Phi the continuous Fourier
 *    transform of phi: Phi(xi) = J sinh(sqrt(b^2-(pi J xi)^2))/sqrt(...).
 *  - Window: u = omega * (K/(2 pi)) with one FP64 multiply (no FMA), first tap
 *    k0 = floor(u - J/2) + 1, taps k0..k0+J-1 wrapped modulo K.
 *
 * Everything is complex double; omega arrives as doubles that were widened
 * exactly from the float32 coordinates the GPU path sees.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define ORC_PI 3.14159265358979323846

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ kernel */

/* Beatty, Nishimura, Pauly (IEEE TMI 2005) choice of the KB shape. */
double orc_kb_beta(int J, double sigma) {
    double a = ((double)J / sigma) * (sigma - 0.5);
    return ORC_PI * sqrt(a * a - 0.8);
}

/* Modified Bessel I0 by its power series sum_k ((z/2)^k / k!)^2. */
double orc_i0(double z) {
    double q = 0.25 * z * z, term = 1.0, sum = 1.0;
    for (int k = 1; k < 500; ++k) {
        term *= q / ((double)k * (double)k);
        sum += term;
        if (term < 1e-18 * sum) break;
    }
    return sum;
}

/* I1(z)/z = sum_k (z/2)^{2k} / (2 k! (k+1)!), equal to 1/2 at z = 0. */
double orc_i1_over_z(double z) {
    double q = 0.25 * z * z, term = 0.5, sum = 0.5;
    for (int k = 1; k < 500; ++k) {
        term *= q / ((double)k * (double)(k + 1));
        sum += term;
        if (term < 1e-18 * sum) break;
    }
    return sum;
}

double orc_kb_phi(double t, int J, double beta) {
    double r = 2.0 * t / (double)J;
    double s = 1.0 - r * r;
    if (s < 0.0) return 0.0;
    return orc_i0(beta * sqrt(s));
}

/* d phi / d t = -(4 beta^2 t / J^2) * I1(z)/z, z = beta sqrt(1-(2t/J)^2). */
double orc_kb_dphi(double t, int J, double beta) {
    double r = 2.0 * t / (double)J;
    double s = 1.0 - r * r;
    if (s < 0.0) return 0.0;
    double z = beta * sqrt(s);
    return -(4.0 * beta * beta * t / ((double)J * (double)J)) * orc_i1_over_z(z);
}

/* Continuous Fourier transform of phi: int phi(t) e^{-2 pi i xi t} dt. */
double orc_kb_ft(double xi, int J, double beta) {
    double a = ORC_PI * (double)J * xi;
    double r = beta * beta - a * a;
    if (r > 0.0) {
        double q = sqrt(r);
        return (double)J * sinh(q) / q;
    } else if (r < 0.0) {
        double q = sqrt(-r);
        return (double)J * sin(q) / q;
    }
    return (double)J;
}

static void axis_betas(int d, const int64_t *N, const int64_t *K, int J, double *beta) {
    for (int a = 0; a < d; ++a) beta[a] = orc_kb_beta(J, (double)K[a] / (double)N[a]);
}

/* Scaling factors s_a(i) = 1/Phi_a((i - N_a/2)/K_a), concatenated over axes. */
void orc_scaling(int d, const int64_t *N, const int64_t *K, int J, double *s_out) {
    double beta[3];
    axis_betas(d, N, K, J, beta);
    int64_t off = 0;
    for (int a = 0; a < d; ++a) {
        for (int64_t i = 0; i < N[a]; ++i) {
            double n = (double)(i - N[a] / 2);
            s_out[off + i] = 1.0 / orc_kb_ft(n / (double)K[a], J, beta[a]);
        }
        off += N[a];
    }
}

/* --------------------------------------------------------------------- FFT */

/* Smallest prime factor. */
static int64_t small_factor(int64_t n) {
    for (int64_t p = 2; p * p <= n; ++p)
        if (n % p == 0) return p;
    return n;
}

/* Recursive mixed-radix decimation in time over any length n.
 * out[k] = sum_q in[q*istride] * W^{q k}, W = tw[.] with tw[e] = e^{sign 2 pi i e / ntop},
 * and the current length n = ntop / twstep.  The p outputs X[k + s m]
 * (s < p) overwrite exactly the p partial results at r m + k (r < p). */
static void fft_rec(int64_t n, const cplx *in, int64_t istride, cplx *out,
                    const cplx *tw, int64_t ntop, int64_t twstep) {
    if (n == 1) {
        out[0] = in[0];
        return;
    }
    int64_t p = small_factor(n), m = n / p;
    for (int64_t r = 0; r < p; ++r)
        fft_rec(m, in + r * istride, istride * p, out + r * m, tw, ntop, twstep * p);
    cplx tmp[64];
    cplx *t = (p <= 64) ? tmp : (cplx *)malloc(sizeof(cplx) * (size_t)p);
    for (int64_t k = 0; k < m; ++k) {
        for (int64_t r = 0; r < p; ++r) t[r] = out[r * m + k];
        for (int64_t s = 0; s < p; ++s) {
            cplx acc = 0.0;
            int64_t kk = k + s * m;
            for (int64_t r = 0; r < p; ++r) {
                int64_t e = (r * kk) % n;
                acc += t[r] * tw[e * twstep];
            }
            out[kk] = acc;
        }
    }
    if (t != tmp) free(t);
    (void)ntop;
}

/* Unnormalised DFT along one axis of a C-order array of the given shape:
 * a[.., k, ..] <- sum_q a[.., q, ..] e^{sign 2 pi i q k / L}. */
void orc_fft_axis(int d, const int64_t *shape, int axis, cplx *a, int sign) {
    int64_t L = shape[axis], outer = 1, inner = 1;
    for (int b = 0; b < axis; ++b) outer *= shape[b];
    for (int b = axis + 1; b < d; ++b) inner *= shape[b];
    cplx *tw = (cplx *)malloc(sizeof(cplx) * (size_t)L);
    for (int64_t e = 0; e < L; ++e) {
        double ang = (double)sign * 2.0 * ORC_PI * (double)e / (double)L;
        tw[e] = cos(ang) + I * sin(ang);
    }
    int64_t lines = outer * inner;
#pragma omp parallel
    {
        cplx *buf = (cplx *)malloc(sizeof(cplx) * (size_t)L);
        cplx *res = (cplx *)malloc(sizeof(cplx) * (size_t)L);
#pragma omp for schedule(static)
        for (int64_t l = 0; l < lines; ++l) {
            int64_t o = l / inner, c = l % inner;
            cplx *base = a + o * L * inner + c;
            for (int64_t q = 0; q < L; ++q) buf[q] = base[q * inner];
            fft_rec(L, buf, 1, res, tw, L, 1);
            for (int64_t q = 0; q < L; ++q) base[q * inner] = res[q];
        }
        free(buf);
        free(res);
    }
    free(tw);
}

void orc_fftn(int d, const int64_t *shape, cplx *a, int sign) {
    for (int ax = 0; ax < d; ++ax) orc_fft_axis(d, shape, ax, a, sign);
}

/* ------------------------------------------------------------ S and pad/crop */

static int64_t prod(int d, const int64_t *v) {
    int64_t p = 1;
    for (int a = 0; a < d; ++a) p *= v[a];
    return p;
}

static int64_t wrap(int64_t k, int64_t K) {
    int64_t r = k % K;
    return r < 0 ? r + K : r;
}

/* g = 0 on the K grid, g[n mod K] = S(n) x_n  (scaling, then zero padding). */
void orc_pad_scale(int d, const int64_t *N, const int64_t *K, int J, const cplx *x, cplx *g) {
    int64_t nN = prod(d, N), nK = prod(d, K);
    int64_t ssz = 0;
    for (int a = 0; a < d; ++a) ssz += N[a];
    double *s = (double *)malloc(sizeof(double) * (size_t)ssz);
    orc_scaling(d, N, K, J, s);
    memset(g, 0, sizeof(cplx) * (size_t)nK);
    for (int64_t lin = 0; lin < nN; ++lin) {
        int64_t rem = lin, q = 0, off = ssz;
        double sc = 1.0;
        int64_t idx[3];
        for (int a = d - 1; a >= 0; --a) {
            idx[a] = rem % N[a];
            rem /= N[a];
        }
        off = 0;
        for (int a = 0; a < d; ++a) {
            sc *= s[off + idx[a]];
            off += N[a];
            q = q * K[a] + wrap(idx[a] - N[a] / 2, K[a]);
        }
        g[q] = sc * x[lin];
    }
    free(s);
}

/* x_n = S(n) H[n mod K]  (crop, then scaling: the adjoint of pad_scale). */
void orc_crop_scale(int d, const int64_t *N, const int64_t *K, int J, const cplx *H, cplx *x) {
    int64_t nN = prod(d, N);
    int64_t ssz = 0;
    for (int a = 0; a < d; ++a) ssz += N[a];
    double *s = (double *)malloc(sizeof(double) * (size_t)ssz);
    orc_scaling(d, N, K, J, s);
    for (int64_t lin = 0; lin < nN; ++lin) {
        int64_t rem = lin, q = 0, off = 0;
        double sc = 1.0;
        int64_t idx[3];
        for (int a = d - 1; a >= 0; --a) {
            idx[a] = rem % N[a];
            rem /= N[a];
        }
        for (int a = 0; a < d; ++a) {
            sc *= s[off + idx[a]];
            off += N[a];
            q = q * K[a] + wrap(idx[a] - N[a] / 2, K[a]);
        }
        x[lin] = sc * H[q];
    }
    free(s);
}

/* ------------------------------------------------------------ V and V^H */

typedef struct {
    int64_t k0[3];   /* first tap per axis (unwrapped) */
    double w[3][32]; /* phi(u_a - k0_a - j) */
    double dw[3][32];/* phi'(u_a - k0_a - j) */
} window_t;

static void make_window(int d, const int64_t *K, int J, const double *beta,
                        const double *om_m, int want_deriv, window_t *win) {
    for (int a = 0; a < d; ++a) {
        double C = (double)K[a] / (2.0 * ORC_PI);
        volatile double u = om_m[a] * C; /* one rounded multiply */
        double base = floor(u - 0.5 * (double)J) + 1.0;
        win->k0[a] = (int64_t)base;
        for (int j = 0; j < J; ++j) {
            double t = u - (base + (double)j);
            win->w[a][j] = orc_kb_phi(t, J, beta[a]);
            if (want_deriv) win->dw[a][j] = orc_kb_dphi(t, J, beta[a]);
        }
    }
}

/* Row-major offset of tap (j_0..j_{d-1}) and its weight product. */
static void tap_iter(int d, const int64_t *K, int J, int64_t t, const window_t *win,
                     int64_t *cell, int64_t *row0, int *jj) {
    int64_t rem = t, c = 0;
    for (int a = d - 1; a >= 0; --a) {
        jj[a] = (int)(rem % J);
        rem /= J;
    }
    for (int a = 0; a < d; ++a) {
        int64_t k = wrap(win->k0[a] + jj[a], K[a]);
        if (a == 0) *row0 = k;
        c = c * K[a] + k;
    }
    *cell = c;
}

/* y_m = sum over the J^d taps of prod_a phi(u_{m,a} - k_a) * G[k mod K]. */
void orc_interp(int d, const int64_t *N, const int64_t *K, int J, int64_t M,
                const double *om, const cplx *G, cplx *y) {
    double beta[3];
    axis_betas(d, N, K, J, beta);
    int64_t taps = 1;
    for (int a = 0; a < d; ++a) taps *= J;
#pragma omp parallel for schedule(static)
    for (int64_t m = 0; m < M; ++m) {
        window_t win;
        make_window(d, K, J, beta, om + m * d, 0, &win);
        cplx acc = 0.0;
        for (int64_t t = 0; t < taps; ++t) {
            int64_t cell, row0;
            int jj[3];
            tap_iter(d, K, J, t, &win, &cell, &row0, jj);
            double w = 1.0;
            for (int a = 0; a < d; ++a) w *= win.w[a][jj[a]];
            acc += w * G[cell];
        }
        y[m] = acc;
    }
}

/* h = 0; h[k mod K] += prod_a phi(u_{m,a} - k_a) y_m for every sample and tap.
 * Parallel over slabs of the slowest grid axis: each thread owns its rows and
 * visits the samples in order, so the result does not depend on the thread count
 * schedule beyond that fixed order. */
void orc_grid(int d, const int64_t *N, const int64_t *K, int J, int64_t M,
              const double *om, const cplx *y, cplx *h) {
    double beta[3];
    axis_betas(d, N, K, J, beta);
    int64_t nK = prod(d, K);
    memset(h, 0, sizeof(cplx) * (size_t)nK);
    int64_t taps = 1;
    for (int a = 0; a < d; ++a) taps *= J;
#pragma omp parallel
    {
        int nt = 1, tid = 0;
#ifdef _OPENMP
        nt = omp_get_num_threads();
        tid = omp_get_thread_num();
#endif
        int64_t lo = K[0] * tid / nt, hi = K[0] * (tid + 1) / nt;
        for (int64_t m = 0; m < M; ++m) {
            window_t win;
            /* cheap reject: does the axis-0 window touch [lo, hi)? */
            double C = (double)K[0] / (2.0 * ORC_PI);
            volatile double u0 = om[m * d] * C;
            int64_t k00 = (int64_t)(floor(u0 - 0.5 * (double)J) + 1.0);
            int touch = 0;
            for (int j = 0; j < J; ++j) {
                int64_t r = wrap(k00 + j, K[0]);
                if (r >= lo && r < hi) touch = 1;
            }
            if (!touch) continue;
            make_window(d, K, J, beta, om + m * d, 0, &win);
            for (int64_t t = 0; t < taps; ++t) {
                int64_t cell, row0;
                int jj[3];
                tap_iter(d, K, J, t, &win, &cell, &row0, jj);
                if (row0 < lo || row0 >= hi) continue;
                double w = 1.0;
                for (int a = 0; a < d; ++a) w *= win.w[a][jj[a]];
                h[cell] += w * y[m];
            }
        }
    }
}

/* ------------------------------------------------------------ whole transforms */

/* y = V F S x.  g_out / G_out (K^d each) receive the padded scaled image and its
 * FFT when non-NULL. */
void orc_forward(int d, const int64_t *N, const int64_t *K, int J, int64_t M,
                 const double *om, const cplx *x, cplx *y, cplx *g_out, cplx *G_out) {
    int64_t nK = prod(d, K);
    cplx *G = (cplx *)malloc(sizeof(cplx) * (size_t)nK);
    orc_pad_scale(d, N, K, J, x, G);
    if (g_out) memcpy(g_out, G, sizeof(cplx) * (size_t)nK);
    orc_fftn(d, K, G, -1);
    if (G_out) memcpy(G_out, G, sizeof(cplx) * (size_t)nK);
    orc_interp(d, N, K, J, M, om, G, y);
    free(G);
}

/* x = S^H F^H V^H y.  h_out / H_out receive the gridded samples and their
 * inverse FFT when non-NULL. */
void orc_adjoint(int d, const int64_t *N, const int64_t *K, int J, int64_t M,
                 const double *om, const cplx *y, cplx *x, cplx *h_out, cplx *H_out) {
    int64_t nK = prod(d, K);
    cplx *h = (cplx *)malloc(sizeof(cplx) * (size_t)nK);
    orc_grid(d, N, K, J, M, om, y, h);
    if (h_out) memcpy(h_out, h, sizeof(cplx) * (size_t)nK);
    orc_fftn(d, K, h, +1);
    if (H_out) memcpy(H_out, h, sizeof(cplx) * (size_t)nK);
    orc_crop_scale(d, N, K, J, h, x);
    free(h);
}

/* Derivative of y_m = V(omega) G with respect to omega_{m,a}, contracted with
 * the torch-convention output gradient gy (dL/dRe y + i dL/dIm y):
 *   gom[m,a] += Re( conj(gy_m) * (K_a / 2 pi) *
 *                   sum_taps phi'(u_a - k_a) prod_{b != a} phi(u_b - k_b) G[k] ).
 * Accumulates, so calls for several coils (each with its own G) sum. */
void orc_grad_points(int d, const int64_t *N, const int64_t *K, int J, int64_t M,
                     const double *om, const cplx *G, const cplx *gy, double *gom) {
    double beta[3];
    axis_betas(d, N, K, J, beta);
    int64_t taps = 1;
    for (int a = 0; a < d; ++a) taps *= J;
#pragma omp parallel for schedule(static)
    for (int64_t m = 0; m < M; ++m) {
        window_t win;
        make_window(d, K, J, beta, om + m * d, 1, &win);
        cplx D[3] = {0.0, 0.0, 0.0};
        for (int64_t t = 0; t < taps; ++t) {
            int64_t cell, row0;
            int jj[3];
            tap_iter(d, K, J, t, &win, &cell, &row0, jj);
            for (int a = 0; a < d; ++a) {
                double w = win.dw[a][jj[a]];
                for (int b = 0; b < d; ++b)
                    if (b != a) w *= win.w[b][jj[b]];
                D[a] += w * G[cell];
            }
        }
        for (int a = 0; a < d; ++a) {
            double C = (double)K[a] / (2.0 * ORC_PI);
            gom[m * d + a] += creal(conj(gy[m]) * D[a]) * C;
        }
    }
}

/* Circulant-embedding product of the normal operator (paper Section 2.1,
 * "Self-adjoint NUFFT": A^H A applied without the interpolator in the loop):
 *   out[n] = sum_{n'} p[n - n'] x[n'],   n, n' in [-N/2, N/2)^d,
 * with the point-spread function p stored centred on [-N, N)^d (array index
 * Delta_a + N_a, shape 2N).  Plain direct sum, O(N^d * N^d). */
void orc_toeplitz_conv(int d, const int64_t *N, const cplx *p, const cplx *x, cplx *out) {
    int64_t nN = prod(d, N);
    int64_t P[3] = {1, 1, 1};
    for (int a = 0; a < d; ++a) P[a] = 2 * N[a];
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < nN; ++e) {
        int64_t i[3] = {0, 0, 0};
        int64_t r = e;
        for (int a = d - 1; a >= 0; --a) {
            i[a] = r % N[a];
            r /= N[a];
        }
        cplx acc = 0.0;
        for (int64_t f = 0; f < nN; ++f) {
            int64_t j[3] = {0, 0, 0};
            int64_t s = f;
            for (int a = d - 1; a >= 0; --a) {
                j[a] = s % N[a];
                s /= N[a];
            }
            /* Delta = n - n' = i - j; centred index Delta + N */
            int64_t idx = 0;
            for (int a = 0; a < d; ++a) idx = idx * P[a] + (i[a] - j[a] + N[a]);
            acc += p[idx] * x[f];
        }
        out[e] = acc;
    }
}
