// HIP kernels for gfx950 (CDNA4, wave64) of the NUFFT pair
//   A   = V F S        (paper Section 2.1, Eq. A = VFS)
//   A^H = S^H F^H V^H  (Section 2.1 "Adjoint PyNUFFT")
//
// Stage map:
//   k_first_pass   S + zero padding + FFT along the contiguous last axis
//                  (Section 2.1 "Scaling", "Oversampled FFT"); the pad is index
//                  arithmetic on the load, never a materialised array.
//   k_strided_pass FFT along a strided axis, zero-padded input rows (forward) or
//                  cropped output rows (adjoint, the copy after the IFFT).
//   k_last_pass    inverse FFT along the last axis + crop + S^H + coil combine
//                  (Section 2.2, multi-coil: sum_i conj(c_i) A^H y_i).
//   k_interp       V, a gather of J^d taps per sample (Section 2.1
//                  "Interpolation"), samples visited in grid-tile order.
//   k_grid         V^H (gridding), output driven: a workgroup owns one grid tile,
//                  accumulates the clipped windows of the samples that reach it
//                  with LDS float atomics and writes the tile once, so no memset
//                  and no global atomics are needed; crowded tiles are split into
//                  chunks whose partial tiles k_reduce_partials sums in chunk
//                  order.  The LDS atomics commit in arrival order, so the last
//                  bits may differ from run to run.
//   k_grad         trajectory gradient through the derivative of the kernel.
//
// All arithmetic is float32 with float32 accumulation; window positions are
// float64 (u = omega * K/(2 pi) as one rounded multiply).
#include <hipcub/hipcub.hpp>

#include "nufft_internal.h"

namespace nufft {
namespace {

// ------------------------------------------------------------ complex helpers
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ __forceinline__ float2 cmulcj(float2 a, float2 b) {
    return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 mul_negi(float2 a) { return make_float2(a.y, -a.x); }

// ------------------------------------------------------------ small DFTs (e^{-2 pi i / R})
template <int R>
__device__ __forceinline__ void dft(float2 *v);

template <>
__device__ __forceinline__ void dft<2>(float2 *v) {
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <>
__device__ __forceinline__ void dft<3>(float2 *v) {
    const float c = 0.86602540378443864676f;  // sin(2 pi / 3)
    float2 s = cadd(v[1], v[2]), dd = csub(v[1], v[2]);
    float2 m = make_float2(v[0].x - 0.5f * s.x, v[0].y - 0.5f * s.y);
    v[0] = cadd(v[0], s);
    v[1] = make_float2(m.x + c * dd.y, m.y - c * dd.x);
    v[2] = make_float2(m.x - c * dd.y, m.y + c * dd.x);
}

template <>
__device__ __forceinline__ void dft<4>(float2 *v) {
    float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    float2 t2 = cadd(v[1], v[3]), t3 = mul_negi(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
}

template <>
__device__ __forceinline__ void dft<5>(float2 *v) {
    const float c1 = 0.30901699437494742410f, c2 = -0.80901699437494742410f;
    const float s1 = 0.95105651629515357212f, s2 = 0.58778525229247312917f;
    float2 p1 = cadd(v[1], v[4]), m1 = csub(v[1], v[4]);
    float2 p2 = cadd(v[2], v[3]), m2 = csub(v[2], v[3]);
    float2 x0 = v[0];
    float2 A1 = make_float2(x0.x + c1 * p1.x + c2 * p2.x, x0.y + c1 * p1.y + c2 * p2.y);
    float2 B1 = make_float2(s1 * m1.x + s2 * m2.x, s1 * m1.y + s2 * m2.y);
    float2 A2 = make_float2(x0.x + c2 * p1.x + c1 * p2.x, x0.y + c2 * p1.y + c1 * p2.y);
    float2 B2 = make_float2(s2 * m1.x - s1 * m2.x, s2 * m1.y - s1 * m2.y);
    v[0] = make_float2(x0.x + p1.x + p2.x, x0.y + p1.y + p2.y);
    v[1] = make_float2(A1.x + B1.y, A1.y - B1.x);
    v[4] = make_float2(A1.x - B1.y, A1.y + B1.x);
    v[2] = make_float2(A2.x + B2.y, A2.y - B2.x);
    v[3] = make_float2(A2.x - B2.y, A2.y + B2.x);
}

template <>
__device__ __forceinline__ void dft<8>(float2 *v) {
    const float r2 = 0.70710678118654752440f;
    float2 e[4] = {v[0], v[2], v[4], v[6]};
    float2 o[4] = {v[1], v[3], v[5], v[7]};
    dft<4>(e);
    dft<4>(o);
    // o[k] *= e^{-2 pi i k / 8}
    float2 o1 = make_float2((o[1].x + o[1].y) * r2, (o[1].y - o[1].x) * r2);
    float2 o2 = mul_negi(o[2]);
    float2 o3 = make_float2((o[3].y - o[3].x) * r2, -(o[3].x + o[3].y) * r2);
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
}

// ------------------------------------------------------------ Stockham passes in LDS
// Element (line, q) of the tile lives at s[line * LS + q * ES].  STRIDED tiles
// keep lines adjacent (ES = number of lines) so a wavefront's lanes walk
// across lines; contiguous tiles keep each line contiguous (ES = 1).
constexpr int kEPT = kFftTileElems / kFftThreads;  // complex elements per thread

template <int R, bool INV, bool STRIDED>
__device__ __forceinline__ void radix_pass(float2 *s, int nlines, int K, int LS, int ES, int Ns,
                                           const float2 *__restrict__ tw) {
    constexpr int NB = (kEPT + R - 1) / R;
    const int nbl = K / R;
    const int total = nlines * nbl;
    float2 v[NB][R];
    int lidx[NB], jidx[NB];
#pragma unroll
    for (int it = 0; it < NB; ++it) {
        const int b = threadIdx.x + it * kFftThreads;
        lidx[it] = 0;
        jidx[it] = 0;
        if (b < total) {
            int line, j;
            if (STRIDED) {
                line = b % nlines;
                j = b / nlines;
            } else {
                j = b % nbl;
                line = b / nbl;
            }
            lidx[it] = line;
            jidx[it] = j;
            const float2 *p = s + line * LS + j * ES;
#pragma unroll
            for (int r = 0; r < R; ++r) v[it][r] = p[r * nbl * ES];
        }
    }
    __syncthreads();
    const int span = K / (Ns * R);
#pragma unroll
    for (int it = 0; it < NB; ++it) {
        const int b = threadIdx.x + it * kFftThreads;
        if (b < total) {
            const int j = jidx[it];
            const int k = j % Ns;
            const int step = k * span;
#pragma unroll
            for (int r = 1; r < R; ++r) {
                float2 w = tw[r * step];
                if (INV) w.y = -w.y;
                v[it][r] = cmul(v[it][r], w);
            }
            if (INV) {
#pragma unroll
                for (int r = 0; r < R; ++r) v[it][r].y = -v[it][r].y;
            }
            dft<R>(v[it]);
            if (INV) {
#pragma unroll
                for (int r = 0; r < R; ++r) v[it][r].y = -v[it][r].y;
            }
            const int idxD = (j / Ns) * Ns * R + k;
            float2 *q = s + lidx[it] * LS + idxD * ES;
#pragma unroll
            for (int r = 0; r < R; ++r) q[r * Ns * ES] = v[it][r];
        }
    }
    __syncthreads();
}

template <bool INV, bool STRIDED>
__device__ void lds_fft(float2 *s, int nlines, int K, int LS, int ES, const RadixPlan &rp,
                        const float2 *__restrict__ tw) {
    int Ns = 1;
    for (int p = 0; p < rp.n; ++p) {
        const int R = rp.r[p];
        switch (R) {
            case 8: radix_pass<8, INV, STRIDED>(s, nlines, K, LS, ES, Ns, tw); break;
            case 4: radix_pass<4, INV, STRIDED>(s, nlines, K, LS, ES, Ns, tw); break;
            case 2: radix_pass<2, INV, STRIDED>(s, nlines, K, LS, ES, Ns, tw); break;
            case 3: radix_pass<3, INV, STRIDED>(s, nlines, K, LS, ES, Ns, tw); break;
            case 5: radix_pass<5, INV, STRIDED>(s, nlines, K, LS, ES, Ns, tw); break;
            default: break;
        }
        Ns *= R;
    }
}

// Product of the scaling factors of the leading axes of image row r
// (row-major over axes 0..d-2).
__device__ __forceinline__ float row_scale(int d, const int *Nax, const float *const *scale, int64_t r) {
    float sc = 1.0f;
    for (int a = d - 2; a >= 0; --a) {
        int64_t i = r % Nax[a];
        r /= Nax[a];
        sc *= scale[a][i];
    }
    return sc;
}

// Grid position of image index i on an axis of image size N and grid size K
// (n = i - N/2 wrapped modulo K), and its inverse (-1 in the zero gap).
__device__ __forceinline__ int pad_pos(int i, int N, int K) { return i < N / 2 ? K - N / 2 + i : i - N / 2; }
__device__ __forceinline__ int src_row(int q, int N, int K) {
    if (q < N / 2) return q + N / 2;
    if (q >= K - N / 2) return q - (K - N / 2);
    return -1;
}

// ------------------------------------------------------------ FFT kernels
__global__ __launch_bounds__(kFftThreads) void k_first_pass(FirstPassArgs a, int lines_per_wg) {
    extern __shared__ float2 s[];
    const int K = a.K, N = a.N;
    const int64_t total = int64_t(a.B) * a.C * a.rows;
    const int64_t l0 = int64_t(blockIdx.x) * lines_per_wg;
    const int nl = int(min(int64_t(lines_per_wg), total - l0));
    const float *slast = a.scale[a.d - 1];
    for (int e = threadIdx.x; e < nl * K; e += kFftThreads) {
        const int lw = e / K, q = e - lw * K;
        float2 v = make_float2(0.f, 0.f);
        const int i = src_row(q, N, K);
        if (i >= 0) {
            const int64_t l = l0 + lw;
            const int64_t g = l / a.rows, r = l - g * a.rows;
            const int64_t b = g / a.C;
            const int64_t c = g - b * a.C;
            v = a.x[(b * a.rows + r) * N + i];
            const float sc = row_scale(a.d, a.Nax, a.scale, r) * slast[i];
            v = cscale(v, sc);
            if (a.coils) v = cmul(v, a.coils[(c * a.rows + r) * N + i]);
        }
        s[e] = v;
    }
    __syncthreads();
    lds_fft<false, false>(s, nl, K, K, 1, a.rp, a.tw);
    float2 *out = a.out + l0 * K;
    for (int e = threadIdx.x; e < nl * K; e += kFftThreads) out[e] = s[e];
}

template <bool INV>
__global__ __launch_bounds__(kFftThreads) void k_strided_pass(StridedPassArgs a, int W, int64_t ntc) {
    extern __shared__ float2 s[];
    const int K = a.K;
    const int64_t bid = blockIdx.x;
    const int64_t ct = bid % ntc;
    const int64_t rest = bid / ntc;
    const int64_t o = rest % a.outer;
    const int64_t g = rest / a.outer;
    const int64_t c0 = ct * W;
    const int wv = int(min(int64_t(W), a.inner - c0));
    const float2 *in = a.in + ((g * a.outer + o) * a.Lin) * a.inner + c0;
    float2 *out = a.out + ((g * a.outer + o) * a.Lout) * a.inner + c0;
    for (int e = threadIdx.x; e < K * W; e += kFftThreads) {
        const int q = e / W, w = e - q * W;
        float2 v = make_float2(0.f, 0.f);
        if (w < wv) {
            const int i = (a.Lin == K) ? q : src_row(q, a.Lin, K);
            if (i >= 0) v = in[int64_t(i) * a.inner + w];
        }
        s[e] = v;
    }
    __syncthreads();
    lds_fft<INV, true>(s, W, K, 1, W, a.rp, a.tw);
    for (int e = threadIdx.x; e < a.Lout * W; e += kFftThreads) {
        const int i = e / W, w = e - i * W;
        if (w < wv) {
            const int q = (a.Lout == K) ? i : pad_pos(i, a.Lout, K);
            out[int64_t(i) * a.inner + w] = s[q * W + w];
        }
    }
}

constexpr int kMaxOutPerThread = kFftTileElems / kFftThreads;

__global__ __launch_bounds__(kFftThreads) void k_last_pass(LastPassArgs a, int rows_per_wg, int coils_per_round) {
    extern __shared__ float2 s[];
    const int K = a.K, N = a.N, C = a.C;
    const int64_t nrt = (a.rows + rows_per_wg - 1) / rows_per_wg;
    const int64_t b = blockIdx.x / nrt;
    const int64_t r0 = (blockIdx.x % nrt) * rows_per_wg;
    const int nr = int(min(int64_t(rows_per_wg), a.rows - r0));
    float2 acc[kMaxOutPerThread];
#pragma unroll
    for (int it = 0; it < kMaxOutPerThread; ++it) acc[it] = make_float2(0.f, 0.f);
    for (int c0 = 0; c0 < C; c0 += coils_per_round) {
        const int nc = min(coils_per_round, C - c0);
        const int nl = nr * nc;
        for (int e = threadIdx.x; e < nl * K; e += kFftThreads) {
            const int lw = e / K, q = e - lw * K;
            const int rr = lw / nc, cc = lw - rr * nc;
            s[e] = a.in[((b * C + c0 + cc) * a.rows + r0 + rr) * K + q];
        }
        __syncthreads();
        lds_fft<true, false>(s, nl, K, K, 1, a.rp, a.tw);
#pragma unroll
        for (int it = 0; it < kMaxOutPerThread; ++it) {
            const int e = threadIdx.x + it * kFftThreads;
            if (e < nr * N) {
                const int rr = e / N, i = e - rr * N;
                const int q = pad_pos(i, N, K);
                float2 v = make_float2(0.f, 0.f);
                for (int cc = 0; cc < nc; ++cc) {
                    float2 t = s[(rr * nc + cc) * K + q];
                    if (a.coils) t = cmulcj(a.coils[(int64_t(c0 + cc) * a.rows + r0 + rr) * N + i], t);
                    v = cadd(v, t);
                }
                acc[it] = cadd(acc[it], v);
            }
        }
        __syncthreads();
    }
    const float *slast = a.scale[a.d - 1];
#pragma unroll
    for (int it = 0; it < kMaxOutPerThread; ++it) {
        const int e = threadIdx.x + it * kFftThreads;
        if (e < nr * N) {
            const int rr = e / N, i = e - rr * N;
            const float sc = row_scale(a.d, a.Nax, a.scale, r0 + rr) * slast[i];
            a.x[(b * a.rows + r0 + rr) * N + i] = cscale(acc[it], sc);
        }
    }
}

// ------------------------------------------------------------ interpolation window
// First tap k0 = floor(u - J/2) + 1 with u = omega * K/(2 pi) in float64, the
// J wrapped grid indices and the offset f = u - k0 - (J/2 - 1) in [0, 1).
template <int J>
__device__ __forceinline__ float window_pos(const SampleGeom &geo, int ax, float om, int *kk) {
    const double u = __dmul_rn(double(om), geo.C[ax]);
    const double k0 = floor(u - 0.5 * J) + 1.0;
    const float f = float(u - k0 - (0.5 * J - 1.0));
    const int K = geo.K[ax];
    long long kw = static_cast<long long>(k0) % K;
    if (kw < 0) kw += K;
#pragma unroll
    for (int j = 0; j < J; ++j) {
        int k = int(kw) + j;
        kk[j] = k >= K ? k - K : k;
    }
    return f;
}

// w_j(f): per-tap polynomial in z = 2f - 1 (Horner, float32).
template <int J>
__device__ __forceinline__ void window_weights(const float *__restrict__ coef, int deg, float f, float *w) {
    const float z = 2.0f * f - 1.0f;
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const float *c = coef + j * (deg + 1);
        float v = c[deg];
        for (int q = deg - 1; q >= 0; --q) v = fmaf(v, z, c[q]);
        w[j] = v;
    }
}

// ------------------------------------------------------------ V (gather)
template <int J, int DIM>
__global__ __launch_bounds__(256) void k_interp(InterpArgs a) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= a.M) return;
    float w[DIM][J];
    int kk[DIM][J];
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) {
        const float f = window_pos<J>(a.geo, ax, a.om_sorted[i * DIM + ax], kk[ax]);
        window_weights<J>(a.geo.coef[ax], a.geo.deg[ax], f, w[ax]);
    }
    const int64_t m = a.perm[i];
    for (int g = 0; g < a.grids; ++g) {
        const float2 *G = a.G + int64_t(g) * a.grid_elems;
        float2 acc = make_float2(0.f, 0.f);
        if constexpr (DIM == 1) {
#pragma unroll
            for (int j = 0; j < J; ++j) acc = cadd(acc, cscale(G[kk[0][j]], w[0][j]));
        } else if constexpr (DIM == 2) {
            const int64_t K1 = a.geo.K[1];
#pragma unroll
            for (int j0 = 0; j0 < J; ++j0) {
                const float2 *row = G + int64_t(kk[0][j0]) * K1;
                float2 rs = make_float2(0.f, 0.f);
#pragma unroll
                for (int j1 = 0; j1 < J; ++j1) rs = cadd(rs, cscale(row[kk[1][j1]], w[1][j1]));
                acc = cadd(acc, cscale(rs, w[0][j0]));
            }
        } else {
            const int64_t K1 = a.geo.K[1], K2 = a.geo.K[2];
            for (int j0 = 0; j0 < J; ++j0) {
                float2 ps = make_float2(0.f, 0.f);
#pragma unroll
                for (int j1 = 0; j1 < J; ++j1) {
                    const float2 *row = G + (int64_t(kk[0][j0]) * K1 + kk[1][j1]) * K2;
                    float2 rs = make_float2(0.f, 0.f);
#pragma unroll
                    for (int j2 = 0; j2 < J; ++j2) rs = cadd(rs, cscale(row[kk[2][j2]], w[2][j2]));
                    ps = cadd(ps, cscale(rs, w[1][j1]));
                }
                acc = cadd(acc, cscale(ps, w[0][j0]));
            }
        }
        a.y[int64_t(g) * a.M + m] = acc;
    }
}

// ------------------------------------------------------------ V^H (output-driven gridding)
template <int J, int DIM>
__global__ __launch_bounds__(256) void k_grid(GridArgs a) {
    extern __shared__ float acc_lds[];
    float *are = acc_lds;
    float *aim = acc_lds + a.tile_cells;
    __shared__ int seg_start[kMaxNeighbors];
    __shared__ int seg_pre[kMaxNeighbors + 1];
    __shared__ int nseg_s;
    const GridItem it = a.items[blockIdx.x];
    const int g = blockIdx.y;
    for (int e = threadIdx.x; e < a.tile_cells; e += blockDim.x) {
        are[e] = 0.f;
        aim[e] = 0.f;
    }
    int tc[DIM];
    {
        int t = it.tile;
#pragma unroll
        for (int ax = DIM - 1; ax >= 0; --ax) {
            tc[ax] = t % a.nt[ax];
            t /= a.nt[ax];
        }
    }
    if (threadIdx.x == 0) {
        int n = 0, pre = 0;
        int r[DIM];
#pragma unroll
        for (int ax = 0; ax < DIM; ++ax) r[ax] = 0;
        while (true) {
            int bin = 0;
#pragma unroll
            for (int ax = 0; ax < DIM; ++ax) {
                int bt = tc[ax] - r[ax];
                if (bt < 0) bt += a.nt[ax];
                bin = bin * a.nt[ax] + bt;
            }
            const int s0 = a.bin_start[bin], s1 = a.bin_start[bin + 1];
            seg_start[n] = s0;
            seg_pre[n] = pre;
            pre += s1 - s0;
            ++n;
            int ax = DIM - 1;
            while (ax >= 0) {
                if (++r[ax] < a.R[ax]) break;
                r[ax] = 0;
                --ax;
            }
            if (ax < 0) break;
        }
        seg_pre[n] = pre;
        nseg_s = n;
    }
    __syncthreads();
    const int nseg = nseg_s;
    const int total = seg_pre[nseg];
    const int f0 = it.chunk * a.chunk;
    const int f1 = min(total, f0 + a.chunk);
    const float2 *y = a.y + int64_t(g) * a.M;
    int base[DIM];
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) base[ax] = tc[ax] * a.T[ax];
    for (int f = f0 + threadIdx.x; f < f1; f += blockDim.x) {
        int n = 0;
        while (n + 1 < nseg && seg_pre[n + 1] <= f) ++n;
        const int64_t i = seg_start[n] + (f - seg_pre[n]);
        int loc[DIM][J];
        float fo[DIM];
        bool hit = true;
#pragma unroll
        for (int ax = 0; ax < DIM; ++ax) {
            int kk[J];
            fo[ax] = window_pos<J>(a.geo, ax, a.om_sorted[i * DIM + ax], kk);
            bool any = false;
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const int l = kk[j] - base[ax];
                const bool in = (l >= 0) && (l < a.T[ax]);
                loc[ax][j] = in ? l : -1;
                any = any || in;
            }
            hit = hit && any;
        }
        if (!hit) continue;
        float w[DIM][J];
#pragma unroll
        for (int ax = 0; ax < DIM; ++ax) window_weights<J>(a.geo.coef[ax], a.geo.deg[ax], fo[ax], w[ax]);
        const float2 v = y[a.perm[i]];
        if constexpr (DIM == 1) {
#pragma unroll
            for (int j = 0; j < J; ++j) {
                if (loc[0][j] < 0) continue;
                atomicAdd(&are[loc[0][j]], w[0][j] * v.x);
                atomicAdd(&aim[loc[0][j]], w[0][j] * v.y);
            }
        } else if constexpr (DIM == 2) {
            const int T1 = a.T[1];
#pragma unroll
            for (int j0 = 0; j0 < J; ++j0) {
                if (loc[0][j0] < 0) continue;
                const float2 v0 = cscale(v, w[0][j0]);
                const int rb = loc[0][j0] * T1;
#pragma unroll
                for (int j1 = 0; j1 < J; ++j1) {
                    if (loc[1][j1] < 0) continue;
                    atomicAdd(&are[rb + loc[1][j1]], w[1][j1] * v0.x);
                    atomicAdd(&aim[rb + loc[1][j1]], w[1][j1] * v0.y);
                }
            }
        } else {
            const int T1 = a.T[1], T2 = a.T[2];
            for (int j0 = 0; j0 < J; ++j0) {
                if (loc[0][j0] < 0) continue;
                const float2 v0 = cscale(v, w[0][j0]);
#pragma unroll
                for (int j1 = 0; j1 < J; ++j1) {
                    if (loc[1][j1] < 0) continue;
                    const float2 v1 = cscale(v0, w[1][j1]);
                    const int rb = (loc[0][j0] * T1 + loc[1][j1]) * T2;
#pragma unroll
                    for (int j2 = 0; j2 < J; ++j2) {
                        if (loc[2][j2] < 0) continue;
                        atomicAdd(&are[rb + loc[2][j2]], w[2][j2] * v1.x);
                        atomicAdd(&aim[rb + loc[2][j2]], w[2][j2] * v1.y);
                    }
                }
            }
        }
    }
    __syncthreads();
    if (it.nchunks == 1) {
        float2 *h = a.h + int64_t(g) * a.grid_elems;
        for (int e = threadIdx.x; e < a.tile_cells; e += blockDim.x) {
            int rem = e;
            int64_t idx = 0;
            int l[DIM];
#pragma unroll
            for (int ax = DIM - 1; ax >= 0; --ax) {
                l[ax] = rem % a.T[ax];
                rem /= a.T[ax];
            }
#pragma unroll
            for (int ax = 0; ax < DIM; ++ax) idx = idx * a.geo.K[ax] + base[ax] + l[ax];
            h[idx] = make_float2(are[e], aim[e]);
        }
    } else {
        float2 *p = a.partials + (int64_t(g) * a.n_slots + it.slot + it.chunk) * a.tile_cells;
        for (int e = threadIdx.x; e < a.tile_cells; e += blockDim.x) p[e] = make_float2(are[e], aim[e]);
    }
}

__global__ __launch_bounds__(256) void k_reduce_partials(ReduceArgs a) {
    const HotTile ht = a.hot[blockIdx.x];
    const int g = blockIdx.y;
    int tc[kMaxDim];
    {
        int t = ht.tile;
        for (int ax = a.d - 1; ax >= 0; --ax) {
            tc[ax] = t % a.nt[ax];
            t /= a.nt[ax];
        }
    }
    const float2 *p = a.partials + (int64_t(g) * a.n_slots + ht.slot) * a.tile_cells;
    float2 *h = a.h + int64_t(g) * a.grid_elems;
    for (int e = threadIdx.x; e < a.tile_cells; e += blockDim.x) {
        float2 acc = make_float2(0.f, 0.f);
        for (int c = 0; c < ht.nchunks; ++c) acc = cadd(acc, p[int64_t(c) * a.tile_cells + e]);
        int rem = e;
        int l[kMaxDim];
        for (int ax = a.d - 1; ax >= 0; --ax) {
            l[ax] = rem % a.T[ax];
            rem /= a.T[ax];
        }
        int64_t idx = 0;
        for (int ax = 0; ax < a.d; ++ax) idx = idx * a.K[ax] + tc[ax] * a.T[ax] + l[ax];
        h[idx] = acc;
    }
}

// ------------------------------------------------------------ trajectory gradient
template <int J, int DIM>
__global__ __launch_bounds__(256) void k_grad(GradArgs a) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= a.M) return;
    float w[DIM][J], dw[DIM][J];
    int kk[DIM][J];
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) {
        const float f = window_pos<J>(a.geo, ax, a.om_sorted[i * DIM + ax], kk[ax]);
        window_weights<J>(a.geo.coef[ax], a.geo.deg[ax], f, w[ax]);
        window_weights<J>(a.geo.dcoef[ax], a.geo.deg_d[ax], f, dw[ax]);
    }
    const int64_t m = a.perm[i];
    float gsum[DIM];
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) gsum[ax] = 0.f;
    for (int g = 0; g < a.grids; ++g) {
        const float2 *G = a.G + int64_t(g) * a.grid_elems;
        float2 D[DIM];
#pragma unroll
        for (int ax = 0; ax < DIM; ++ax) D[ax] = make_float2(0.f, 0.f);
        if constexpr (DIM == 1) {
#pragma unroll
            for (int j = 0; j < J; ++j) D[0] = cadd(D[0], cscale(G[kk[0][j]], dw[0][j]));
        } else if constexpr (DIM == 2) {
            const int64_t K1 = a.geo.K[1];
#pragma unroll
            for (int j0 = 0; j0 < J; ++j0) {
                const float2 *row = G + int64_t(kk[0][j0]) * K1;
                float2 rs = make_float2(0.f, 0.f), rsd = make_float2(0.f, 0.f);
#pragma unroll
                for (int j1 = 0; j1 < J; ++j1) {
                    const float2 gv = row[kk[1][j1]];
                    rs = cadd(rs, cscale(gv, w[1][j1]));
                    rsd = cadd(rsd, cscale(gv, dw[1][j1]));
                }
                D[0] = cadd(D[0], cscale(rs, dw[0][j0]));
                D[1] = cadd(D[1], cscale(rsd, w[0][j0]));
            }
        } else {
            const int64_t K1 = a.geo.K[1], K2 = a.geo.K[2];
            for (int j0 = 0; j0 < J; ++j0) {
                float2 P = make_float2(0.f, 0.f), P1 = P, P2 = P;
#pragma unroll
                for (int j1 = 0; j1 < J; ++j1) {
                    const float2 *row = G + (int64_t(kk[0][j0]) * K1 + kk[1][j1]) * K2;
                    float2 rs = make_float2(0.f, 0.f), rsd = rs;
#pragma unroll
                    for (int j2 = 0; j2 < J; ++j2) {
                        const float2 gv = row[kk[2][j2]];
                        rs = cadd(rs, cscale(gv, w[2][j2]));
                        rsd = cadd(rsd, cscale(gv, dw[2][j2]));
                    }
                    P = cadd(P, cscale(rs, w[1][j1]));
                    P1 = cadd(P1, cscale(rs, dw[1][j1]));
                    P2 = cadd(P2, cscale(rsd, w[1][j1]));
                }
                D[0] = cadd(D[0], cscale(P, dw[0][j0]));
                D[1] = cadd(D[1], cscale(P1, w[0][j0]));
                D[2] = cadd(D[2], cscale(P2, w[0][j0]));
            }
        }
        const float2 gy = a.gy[int64_t(g) * a.M + m];
#pragma unroll
        for (int ax = 0; ax < DIM; ++ax) gsum[ax] += gy.x * D[ax].x + gy.y * D[ax].y;
    }
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) a.gom[m * DIM + ax] = gsum[ax] * float(a.geo.C[ax]);
}

// ------------------------------------------------------------ plan-time binning
__global__ __launch_bounds__(256) void k_bin_keys(BinArgs a) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= a.M) return;
    int key = 0;
    bool bad = false;
    for (int ax = 0; ax < a.d; ++ax) {
        const float om = a.om[i * a.d + ax];
        int tile = 0;
        if (!isfinite(om)) {
            bad = true;
        } else {
            const double u = __dmul_rn(double(om), a.C[ax]);
            if (fabs(u) > 1.0e15) {
                bad = true;
            } else {
                const double k0 = floor(u - 0.5 * a.J) + 1.0;
                long long kw = static_cast<long long>(k0) % a.K[ax];
                if (kw < 0) kw += a.K[ax];
                tile = int(kw) / a.T[ax];
            }
        }
        key = key * a.nt[ax] + tile;
    }
    if (bad) atomicOr(a.flag, 1);
    a.keys[i] = key;
    atomicAdd(&a.counts[key], 1);
}

__global__ void k_iota(int *v, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) v[i] = int(i);
}

__global__ void k_permute_points(const float *om, const int *perm, int64_t M, int d, float *out) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= M) return;
    const int64_t m = perm[i];
    for (int ax = 0; ax < d; ++ax) out[i * d + ax] = om[m * d + ax];
}

// ------------------------------------------------------------ template dispatch
template <template <int, int> class Fn, int J>
struct DimDispatch {
    template <class... Args>
    static hipError_t run(int d, Args &&...args) {
        switch (d) {
            case 1: return Fn<J, 1>::go(args...);
            case 2: return Fn<J, 2>::go(args...);
            case 3: return Fn<J, 3>::go(args...);
            default: return hipErrorInvalidValue;
        }
    }
};

template <template <int, int> class Fn, class... Args>
hipError_t dispatch_jd(int J, int d, Args &&...args) {
    switch (J) {
#define NUFFT_J_CASE(JJ) \
    case JJ: return DimDispatch<Fn, JJ>::run(d, args...);
        NUFFT_J_CASE(2)
        NUFFT_J_CASE(3)
        NUFFT_J_CASE(4)
        NUFFT_J_CASE(5)
        NUFFT_J_CASE(6)
        NUFFT_J_CASE(7)
        NUFFT_J_CASE(8)
        NUFFT_J_CASE(9)
        NUFFT_J_CASE(10)
        NUFFT_J_CASE(11)
        NUFFT_J_CASE(12)
        NUFFT_J_CASE(13)
        NUFFT_J_CASE(14)
        NUFFT_J_CASE(15)
        NUFFT_J_CASE(16)
#undef NUFFT_J_CASE
        default: return hipErrorInvalidValue;
    }
}

template <int J, int DIM>
struct InterpLaunch {
    static hipError_t go(const InterpArgs &a, hipStream_t s) {
        if (a.M == 0) return hipSuccess;
        const int64_t blocks = (a.M + 255) / 256;
        hipLaunchKernelGGL((k_interp<J, DIM>), dim3(unsigned(blocks)), dim3(256), 0, s, a);
        return hipGetLastError();
    }
};

template <int J, int DIM>
struct GridLaunch {
    static hipError_t go(const GridArgs &a, hipStream_t s) {
        if (a.n_items == 0) return hipSuccess;
        const size_t lds = size_t(a.tile_cells) * 2 * sizeof(float);
        hipLaunchKernelGGL((k_grid<J, DIM>), dim3(unsigned(a.n_items), unsigned(a.grids)), dim3(256), lds, s, a);
        return hipGetLastError();
    }
};

template <int J, int DIM>
struct GradLaunch {
    static hipError_t go(const GradArgs &a, hipStream_t s) {
        if (a.M == 0) return hipSuccess;
        const int64_t blocks = (a.M + 255) / 256;
        hipLaunchKernelGGL((k_grad<J, DIM>), dim3(unsigned(blocks)), dim3(256), 0, s, a);
        return hipGetLastError();
    }
};

}  // namespace

// ------------------------------------------------------------ launchers
hipError_t launch_first_pass(const FirstPassArgs &a, hipStream_t s) {
    const int64_t total = int64_t(a.B) * a.C * a.rows;
    if (total == 0) return hipSuccess;
    const int lpw = max(1, kFftTileElems / a.K);
    const int64_t blocks = (total + lpw - 1) / lpw;
    const size_t lds = size_t(lpw) * a.K * sizeof(float2);
    hipLaunchKernelGGL(k_first_pass, dim3(unsigned(blocks)), dim3(kFftThreads), lds, s, a, lpw);
    return hipGetLastError();
}

hipError_t launch_strided_pass(const StridedPassArgs &a, hipStream_t s) {
    if (a.grids * a.outer * a.inner == 0) return hipSuccess;
    int W = max(1, kFftTileElems / a.K);
    if (int64_t(W) > a.inner) W = int(a.inner);
    const int64_t ntc = (a.inner + W - 1) / W;
    const int64_t blocks = ntc * a.outer * a.grids;
    const size_t lds = size_t(W) * a.K * sizeof(float2);
    if (a.inverse)
        hipLaunchKernelGGL(k_strided_pass<true>, dim3(unsigned(blocks)), dim3(kFftThreads), lds, s, a, W, ntc);
    else
        hipLaunchKernelGGL(k_strided_pass<false>, dim3(unsigned(blocks)), dim3(kFftThreads), lds, s, a, W, ntc);
    return hipGetLastError();
}

hipError_t launch_last_pass(const LastPassArgs &a, hipStream_t s) {
    if (int64_t(a.B) * a.rows == 0) return hipSuccess;
    int rows_per_wg, coils_per_round;
    if (a.C * a.K <= kFftTileElems) {
        coils_per_round = a.C;
        rows_per_wg = max(1, kFftTileElems / (a.C * a.K));
    } else {
        rows_per_wg = 1;
        coils_per_round = max(1, kFftTileElems / a.K);
    }
    // at most kMaxOutPerThread outputs per thread
    while (rows_per_wg > 1 && rows_per_wg * a.N > kMaxOutPerThread * kFftThreads) --rows_per_wg;
    if (int64_t(rows_per_wg) > a.rows) rows_per_wg = int(a.rows);
    const int64_t nrt = (a.rows + rows_per_wg - 1) / rows_per_wg;
    const int64_t blocks = nrt * a.B;
    const size_t lds = size_t(rows_per_wg) * coils_per_round * a.K * sizeof(float2);
    hipLaunchKernelGGL(k_last_pass, dim3(unsigned(blocks)), dim3(kFftThreads), lds, s, a, rows_per_wg,
                       coils_per_round);
    return hipGetLastError();
}

hipError_t launch_interp(const InterpArgs &a, hipStream_t s) {
    return dispatch_jd<InterpLaunch>(a.geo.J, a.geo.d, a, s);
}

hipError_t launch_grid(const GridArgs &a, hipStream_t s) {
    return dispatch_jd<GridLaunch>(a.geo.J, a.geo.d, a, s);
}

hipError_t launch_reduce_partials(const ReduceArgs &a, hipStream_t s) {
    if (a.n_hot == 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_partials, dim3(unsigned(a.n_hot), unsigned(a.grids)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_grad(const GradArgs &a, hipStream_t s) {
    return dispatch_jd<GradLaunch>(a.geo.J, a.geo.d, a, s);
}

hipError_t launch_bin_keys(const BinArgs &a, hipStream_t s) {
    if (a.M == 0) return hipSuccess;
    const int64_t blocks = (a.M + 255) / 256;
    hipLaunchKernelGGL(k_bin_keys, dim3(unsigned(blocks)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_iota(int *v, int64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_iota, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, v, n);
    return hipGetLastError();
}

hipError_t launch_permute_points(const float *om, const int *perm, int64_t M, int d, float *om_sorted,
                                 hipStream_t s) {
    if (M == 0) return hipSuccess;
    hipLaunchKernelGGL(k_permute_points, dim3(unsigned((M + 255) / 256)), dim3(256), 0, s, om, perm, M, d,
                       om_sorted);
    return hipGetLastError();
}

hipError_t sort_pairs(const int *keys_in, int *keys_out, const int *vals_in, int *vals_out, int64_t n,
                      int key_bits, hipStream_t s) {
    if (n == 0) return hipSuccess;
    size_t temp = 0;
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, temp, keys_in, keys_out, vals_in, vals_out,
                                                      int(n), 0, key_bits, s);
    if (e != hipSuccess) return e;
    void *buf = nullptr;
    e = hipMalloc(&buf, temp > 0 ? temp : 1);
    if (e != hipSuccess) return e;
    e = hipcub::DeviceRadixSort::SortPairs(buf, temp, keys_in, keys_out, vals_in, vals_out, int(n), 0,
                                           key_bits, s);
    hipError_t e2 = hipStreamSynchronize(s);
    (void)hipFree(buf);
    return e != hipSuccess ? e : e2;
}

}  // namespace nufft
