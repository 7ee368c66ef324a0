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
//   k_grid_blk     V^H (gridding) in 3D on the matrix cores by 4 x 4 blocks;
//   k_grid_mfma    by row tiles (2D and other 16-cell tiles);
//   k_grid         on the vector ALUs (other tiles).  All output driven: a
//                  work item owns one grid tile and walks the samples that
//                  reach it (staged in LDS), so the tile is written once with
//                  plain stores: no memset, no atomics, a fixed summation
//                  order; crowded tiles are split into chunks whose partial
//                  tiles k_reduce_partials (or the first inverse FFT pass)
//                  sums in a fixed order.
//   k_grad         trajectory gradient through the derivative of the kernel.
//
// All arithmetic is float32 with float32 accumulation; window positions are
// float64 (u = omega * K/(2 pi) as one rounded multiply).
#include <hip/hip_ext.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <mutex>
#include <type_traits>

#include "nufft_internal.h"

namespace nufft {
namespace {

// Every kernel launch of the library: a launch inside a timed stage carries the
// stage's start and stop events.
template <typename K, typename... Args>
void launch_kernel(K kernel, dim3 grid, dim3 block, size_t lds, hipStream_t s, Args... args) {
    LaunchEvents *ev = g_launch_events;
    if (ev && !ev->used) {
        ev->used = true;
        hipExtLaunchKernelGGL(kernel, grid, block, uint32_t(lds), s, ev->start, ev->stop, 0u, args...);
    } else {
        hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
    }
}

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

// floor(e / D) for a divisor D >= 1 fixed per launch: q = floor(e m / 2^32)
// with m = ceil(2^32 / D) is exact whenever e (D - 1) < 2^32, since the error
// e (m D - 2^32) / (D 2^32) then stays below 1/D.  One high multiply instead
// of an integer division.  Every use here divides tile positions (< 4096) by
// at most 4096, or a column index c < K_1 K_2 by K_2 with K_1 K_2^2 < 2^32
// (checked when the plan is made).
struct FastDiv {
    unsigned m;
    int d;
    __device__ __forceinline__ FastDiv() : m(0u), d(1) {}
    __device__ __forceinline__ explicit FastDiv(int D) : m(D > 1 ? 0xFFFFFFFFu / unsigned(D) + 1u : 0u), d(D) {}
    __device__ __forceinline__ FastDiv(unsigned magic, int D) : m(magic), d(D) {}  // magic made on the host
    __device__ __forceinline__ int div(int e) const { return d > 1 ? int(__umulhi(unsigned(e), m)) : e; }
    __device__ __forceinline__ int rem(int e, int q) const { return e - __umul24(q, d); }
};

// ------------------------------------------------------------ Stockham passes in LDS
// Element (line, q) of a tile lives at s[line * LS + q * ES].  STRIDED tiles
// keep lines adjacent (ES = number of lines) so a wavefront's lanes walk
// across lines; contiguous tiles keep each line contiguous (ES = 1).  A tile
// holds at most THREADS * kEPT complex elements; a thread handles up to
// ceil(kEPT / R) butterflies of radix R per pass.  Twiddles e^{-2 pi i e / K}
// are staged in LDS (tw) once per workgroup.
constexpr int kEPT = 8;  // complex elements per thread

// KC > 0: the line length KC and sub-transform length NSC of this pass are
// compile-time constants (the common grid sizes), so its index arithmetic
// folds; the same operations in the same order as the run-time form.
template <int THREADS, int R, bool INV, bool STRIDED, int KC = 0, int NSC = 0>
__device__ __forceinline__ void radix_pass(float2 *s, int nlines, int K_, int LS, int ES, int Ns_, int span_,
                                           unsigned m_ns, unsigned m_nbl, const float2 *tw) {
    constexpr int NB = (kEPT + R - 1) / R;
    const int K = KC > 0 ? KC : K_;
    const int Ns = KC > 0 ? NSC : Ns_;
    const int span = KC > 0 ? KC / ((NSC > 0 ? NSC : 1) * R) : span_;
    const int nbl = K / R;
    const int total = nlines * nbl;
    // (the line count's magic is made per pass: kept across passes it costs
    // the strided passes about 20 registers)
    const FastDiv by_line = STRIDED ? FastDiv(nlines) : FastDiv(m_nbl, nbl), by_ns(m_ns, Ns);
    float2 v[NB][R];
    int lidx[NB], jidx[NB];
#pragma unroll
    for (int it = 0; it < NB; ++it) {
        const int b = threadIdx.x + it * THREADS;
        lidx[it] = 0;
        jidx[it] = 0;
        if (b < total) {
            int line, j;
            if (STRIDED) {
                j = by_line.div(b);
                line = by_line.rem(b, j);
            } else if constexpr (KC > 0) {
                line = b / (KC / R);
                j = b - line * (KC / R);
            } else {
                line = by_line.div(b);
                j = by_line.rem(b, line);
            }
            lidx[it] = line;
            jidx[it] = j;
            const float2 *p = s + line * LS + j * ES;
#pragma unroll
            for (int r = 0; r < R; ++r) v[it][r] = p[r * nbl * ES];
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < NB; ++it) {
        const int b = threadIdx.x + it * THREADS;
        if (b < total) {
            const int j = jidx[it];
            int jq, k;
            if constexpr (KC > 0) {
                jq = j / NSC;
                k = j - jq * NSC;
            } else {
                jq = by_ns.div(j);
                k = by_ns.rem(j, jq);
            }
            const int step = __umul24(k, span);
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
            const int idxD = __umul24(jq, Ns * R) + k;
            float2 *q = s + lidx[it] * LS + idxD * ES;
#pragma unroll
            for (int r = 0; r < R; ++r) q[r * Ns * ES] = v[it][r];
        }
    }
    __syncthreads();
}

template <int THREADS, bool INV, bool STRIDED>
__device__ void lds_fft(float2 *s, int nlines, int K, int LS, int ES, const RadixPlan &rp, const float2 *tw) {
    // the grid sizes of the common workloads (and their Toeplitz 2N grids)
    // with their radix plans spelled out at compile time
    if (K == 512 && rp.n == 3 && rp.r[0] == 8 && rp.r[1] == 8 && rp.r[2] == 8) {
        radix_pass<THREADS, 8, INV, STRIDED, 512, 1>(s, nlines, K, LS, ES, 1, 0, 0u, 0u, tw);
        radix_pass<THREADS, 8, INV, STRIDED, 512, 8>(s, nlines, K, LS, ES, 8, 0, 0u, 0u, tw);
        radix_pass<THREADS, 8, INV, STRIDED, 512, 64>(s, nlines, K, LS, ES, 64, 0, 0u, 0u, tw);
        return;
    }
    if (K == 256 && rp.n == 3 && rp.r[0] == 8 && rp.r[1] == 8 && rp.r[2] == 4) {
        radix_pass<THREADS, 8, INV, STRIDED, 256, 1>(s, nlines, K, LS, ES, 1, 0, 0u, 0u, tw);
        radix_pass<THREADS, 8, INV, STRIDED, 256, 8>(s, nlines, K, LS, ES, 8, 0, 0u, 0u, tw);
        radix_pass<THREADS, 4, INV, STRIDED, 256, 64>(s, nlines, K, LS, ES, 64, 0, 0u, 0u, tw);
        return;
    }
    int Ns = 1;
    for (int p = 0; p < rp.n; ++p) {
        const int R = rp.r[p];
        const int sp = rp.span[p];
        const unsigned mn = rp.m_ns[p], mb = rp.m_nbl[p];
        switch (R) {
            case 8: radix_pass<THREADS, 8, INV, STRIDED>(s, nlines, K, LS, ES, Ns, sp, mn, mb, tw); break;
            case 4: radix_pass<THREADS, 4, INV, STRIDED>(s, nlines, K, LS, ES, Ns, sp, mn, mb, tw); break;
            case 2: radix_pass<THREADS, 2, INV, STRIDED>(s, nlines, K, LS, ES, Ns, sp, mn, mb, tw); break;
            case 3: radix_pass<THREADS, 3, INV, STRIDED>(s, nlines, K, LS, ES, Ns, sp, mn, mb, tw); break;
            case 5: radix_pass<THREADS, 5, INV, STRIDED>(s, nlines, K, LS, ES, Ns, sp, mn, mb, tw); break;
            default: break;
        }
        Ns *= R;
    }
}

// Twiddles into LDS.  A workgroup's tile holds at least one whole line, so a
// thread stages at most kEPT of the K twiddles; every load is issued before
// the first LDS write, so the staging costs one memory round trip.
template <int THREADS>
struct TwiddleStage {
    float2 v[kEPT];
    __device__ __forceinline__ void load(const float2 *__restrict__ tw, int K) {
#pragma unroll
        for (int u = 0; u < kEPT; ++u) {
            const int e = threadIdx.x + u * THREADS;
            if (e < K) v[u] = tw[e];
        }
    }
    __device__ __forceinline__ void store(float2 *tw_lds, int K) const {
#pragma unroll
        for (int u = 0; u < kEPT; ++u) {
            const int e = threadIdx.x + u * THREADS;
            if (e < K) tw_lds[e] = v[u];
        }
    }
};


// Product of the scaling factors of the leading axes of image row r
// (row-major over axes 0..d-2), 32-bit index arithmetic.
__device__ __forceinline__ float row_scale(int d, const int *Nax, const float *const *scale, int r) {
    float sc = 1.0f;
    for (int a = d - 2; a >= 0; --a) {
        const int i = r % Nax[a];
        r /= Nax[a];
        sc *= scale[a][i];
    }
    return sc;
}

// row_scale with its loads issued at load() and the product formed at value(),
// so the loads overlap other work.
struct RowScale {
    float f[kMaxDim - 1];
    int n;
    __device__ __forceinline__ void load(int d, const int *Nax, const float *const *scale, int r) {
        n = d - 1;
#pragma unroll
        for (int a = kMaxDim - 2; a >= 0; --a) {
            if (a < n) {
                const int i = r % Nax[a];
                r /= Nax[a];
                f[a] = scale[a][i];
            }
        }
    }
    __device__ __forceinline__ float value() const {
        float sc = 1.0f;
#pragma unroll
        for (int a = kMaxDim - 2; a >= 0; --a)
            if (a < n) sc *= f[a];
        return sc;
    }
};

// Grid position of image index i on an axis of image size N and grid size K
// (n = i - N/2 wrapped modulo K), and its inverse (-1 in the zero gap).
__device__ __forceinline__ int pad_pos(int i, int N, int K) { return i < N / 2 ? K - N / 2 + i : i - N / 2; }
__device__ __forceinline__ int src_row(int q, int N, int K) {
    if (q < N / 2) return q + N / 2;
    if (q >= K - N / 2) return q - (K - N / 2);
    return -1;
}

// ------------------------------------------------------------ FFT kernels
// Dynamic LDS layout of every FFT kernel: [K twiddles][tile].
template <int THREADS>
__device__ __forceinline__ void first_pass_body(const FirstPassArgs &a, int lines_per_wg, int64_t bx) {
    extern __shared__ float2 lds[];
    const int K = a.K, N = a.N;
    float2 *tw = lds;
    float2 *s = lds + K;
    const int64_t total = int64_t(a.B) * a.C * a.rows;
    const int64_t l0 = bx * lines_per_wg;
    const int nl = int(min(int64_t(lines_per_wg), total - l0));  // 1..64
    // Line `lane` of the workgroup, known to that lane of every wavefront: the
    // image and coil row offsets and the product of the leading axes' scaling
    // factors (applied after the FFT, which is linear along the line).
    const int lane = threadIdx.x & 63;
    int xb = 0, cb = 0;
    RowScale rsf;
    {
        const int64_t l = l0 + min(lane, nl - 1);
        const int g = int(l / a.rows);
        const int r = int(l - int64_t(g) * a.rows);
        const int b = g / a.C;
        const int c = g - b * a.C;
        rsf.load(a.d, a.Nax, a.scale, r);  // consumed after the FFT
        xb = (b * int(a.rows) + r) * N;
        cb = (c * int(a.rows) + r) * N;
    }
    TwiddleStage<THREADS> tws;
    tws.load(a.tw, K);
    // the tile holds nl * K <= THREADS * kEPT elements: every load is issued
    // before the first use
    const int ne = nl * K;
    const FastDiv byK(K);
    const float *slast = a.scale[a.d - 1];
    // (loads land in registers without a default value, so no copy waits for
    // them; `live` marks the elements that read the image)
    // (branch-free: indices are clamped into the row and `live` marks the
    // elements that really read the image, so no load waits on another)
    float2 xv[kEPT], cv[kEPT];
    float sv[kEPT];
    unsigned live = 0;
#pragma unroll
    for (int u = 0; u < kEPT; ++u) {
        const int e = min(int(threadIdx.x) + u * THREADS, ne - 1);
        const int lw = byK.div(e);
        const int i = src_row(byK.rem(e, lw), N, K);
        live |= (int(threadIdx.x) + u * THREADS < ne && i >= 0) ? 1u << u : 0u;
        const int ic = max(i, 0);
        // one grid per image row without coils: line l reads image row l
        const int xbl = a.C == 1 ? int(l0 + lw) * N : __shfl(xb, lw);
        xv[u] = a.x[xbl + ic];
        sv[u] = slast[ic];
        if (a.coils) cv[u] = a.coils[__shfl(cb, lw) + ic];
    }
    // values first, without branches (one wait for all loads), then the writes
#pragma unroll
    for (int u = 0; u < kEPT; ++u) {
        float2 v = cscale(xv[u], sv[u]);
        if (a.coils) v = cmul(v, cv[u]);
        xv[u] = (live & (1u << u)) ? v : make_float2(0.f, 0.f);
    }
    tws.store(tw, K);
#pragma unroll
    for (int u = 0; u < kEPT; ++u) {
        const int e = threadIdx.x + u * THREADS;
        if (e < ne) s[e] = xv[u];
    }
    __syncthreads();
    lds_fft<THREADS, false, false>(s, nl, K, K, 1, a.rp, tw);
    const float rs = rsf.value();
    float2 *out = a.out + l0 * K;
    float2 pv[kEPT], mv[kEPT];
#pragma unroll
    for (int u = 0; u < kEPT; ++u) {
        const int e = min(int(threadIdx.x) + u * THREADS, ne - 1);
        const int lw = byK.div(e);
        const int q = byK.rem(e, lw);
        if (a.phase) pv[u] = a.phase[q];
        if (a.mult) mv[u] = a.mult[((l0 + lw) % a.rows) * K + q];
    }
#pragma unroll
    for (int u = 0; u < kEPT; ++u) {
        const int e = min(int(threadIdx.x) + u * THREADS, ne - 1);
        float2 v = s[e];
        if (a.d > 1) v = cscale(v, __shfl(rs, byK.div(e)));  // row scale of the element's line
        if (a.phase) v = cmul(v, pv[u]);
        if (a.mult) v = cmul(v, mv[u]);
        pv[u] = v;
    }
#pragma unroll
    for (int u = 0; u < kEPT; ++u) {
        const int e = threadIdx.x + u * THREADS;
        if (e < ne) out[e] = pv[u];
    }
}

template <int THREADS>
__global__ __launch_bounds__(THREADS) void k_first_pass(FirstPassArgs a, int lines_per_wg) {
    first_pass_body<THREADS>(a, lines_per_wg, blockIdx.x);
}

// Many problems in one launch: workgroup b runs block blocks[b].y of problem
// blocks[b].x, whose arguments sit in jobs[blocks[b].x].
template <int THREADS>
__global__ __launch_bounds__(THREADS) void k_first_pass_multi(const FirstJob *__restrict__ jobs,
                                                             const int4 *__restrict__ blocks) {
    const int4 b = blocks[blockIdx.x];
    const FirstJob &j = jobs[b.x];
    first_pass_body<THREADS>(j.a, j.lpw, b.y);
}

// SPLIT (inverse only): the first inverse pass of an adjoint whose split
// gridding tiles are still partial tiles (its own instantiation, so the
// common passes keep their register budget).
template <int THREADS, bool INV, bool SPLIT>
__device__ __forceinline__ void strided_pass_body(const StridedPassArgs &a, int W, int64_t ntc, int64_t bid) {
    extern __shared__ float2 lds[];
    const int K = a.K;
    float2 *tw = lds;
    float2 *s = lds + K;
    const int64_t ct = bid % ntc;
    const int64_t rest = bid / ntc;
    const int64_t o = rest % a.outer;
    const int64_t g = rest / a.outer;
    const int64_t c0 = ct * W;
    const int wv = int(min(int64_t(W), a.inner - c0));
    const float2 *in = a.in + ((g * a.outer + o) * a.Lin) * a.inner + c0;
    float2 *out = a.out + ((g * a.outer + o) * a.Lout) * a.inner + c0;
    TwiddleStage<THREADS> tws;
    tws.load(a.tw, K);
    // the tile holds K * W <= THREADS * kEPT elements
    const int ne = K * W;
    const FastDiv byW(W);
    // (no default values in the load registers, so no copy waits for a load;
    // `live` marks the elements that read the input)
    float2 v[kEPT], mv[kEPT], pv[kEPT];
    unsigned live = 0;
    if constexpr (!SPLIT) {
#pragma unroll
        for (int u = 0; u < kEPT; ++u) {
            const int e = threadIdx.x + u * THREADS;
            const int q = byW.div(min(e, ne - 1));
            const int w = e - __umul24(q, W);
            // forward: grid row q takes image row src_row (zero rows when Lin < K,
            // the centring shift when Lin == K); inverse: the input is the grid
            const int i = INV ? q : src_row(q, a.Lin, K);
            if (e < ne && w < wv && i >= 0) {
                live |= 1u << u;
                v[u] = in[int64_t(i) * a.inner + w];
                if (a.mult) mv[u] = a.mult[(o * a.Lin + i) * a.inner + c0 + w];
                if (INV && a.phase) pv[u] = a.phase[q];
            }
        }
    } else {
        // First inverse pass of the adjoint: a cell of a split gridding tile is
        // the sum of its partial tiles in chunk order (the order, hence the bits,
        // of k_reduce_partials).  Grid row q on axis 0, column c0 + w over the
        // remaining axes; the input and the cell's split entry are loaded
        // together, the partial tiles after that.
        const FastDiv byT0(a.T[0]), byT1(a.T[1]), byT2(a.d > 2 ? a.T[2] : 1), byK2(a.d > 2 ? a.Kax[2] : 1);
        int2 sp[kEPT];
        int cellv[kEPT];
#pragma unroll
        for (int u = 0; u < kEPT; ++u) {
            const int e = min(int(threadIdx.x) + u * THREADS, ne - 1);
            const int q = byW.div(e);
            const int w = min(e - __umul24(q, W), wv - 1);
            const int i = INV ? q : max(src_row(q, a.Lin, K), 0);
            live |= (int(threadIdx.x) + u * THREADS < ne && e - __umul24(q, W) < wv &&
                     (INV || src_row(q, a.Lin, K) >= 0)) ? 1u << u : 0u;
            // grid coordinates of the cell: k0 = q, then the column's axes
            const int c = int(c0) + w;
            int k1 = c, k2 = 0;
            if (a.d > 2) {
                k1 = byK2.div(c);
                k2 = byK2.rem(c, k1);
            }
            const int t0 = byT0.div(q), t1 = byT1.div(k1);
            int tile = t0 * a.nt[1] + t1;
            int cell = byT0.rem(q, t0) * a.T[1] + byT1.rem(k1, t1);
            if (a.d > 2) {
                const int t2 = byT2.div(k2);
                tile = tile * a.nt[2] + t2;
                cell = cell * a.T[2] + byT2.rem(k2, t2);
            }
            v[u] = in[int64_t(i) * a.inner + w];
            sp[u] = a.split_of_tile[tile];
            cellv[u] = cell;
            if (INV && a.phase) pv[u] = a.phase[q];  // (never with a Toeplitz product)
        }
#pragma unroll
        for (int u = 0; u < kEPT; ++u) {
            const int n = sp[u].y;
            if (n > 0) {
                const float2 *pp = a.partials + (g * a.n_slots + sp[u].x) * a.tile_cells + cellv[u];
                // kReduceLanes interleaved sums (chunk c into sum c mod
                // kReduceLanes, in chunk order), then added in lane order
                float2 acc[kReduceLanes];
#pragma unroll
                for (int j = 0; j < kReduceLanes; ++j) acc[j] = make_float2(0.f, 0.f);
                for (int k0 = 0; k0 < n; k0 += kReduceLanes) {
                    float2 t[kReduceLanes];
#pragma unroll
                    for (int j = 0; j < kReduceLanes; ++j)
                        if (k0 + j < n) t[j] = pp[int64_t(k0 + j) * a.tile_cells];
#pragma unroll
                    for (int j = 0; j < kReduceLanes; ++j)
                        if (k0 + j < n) acc[j] = cadd(acc[j], t[j]);
                }
#pragma unroll
                for (int j = 1; j < kReduceLanes; ++j) acc[0] = cadd(acc[0], acc[j]);
                v[u] = acc[0];
            }
        }
    }
    // values first, without branches (one wait for all loads), then the writes
#pragma unroll
    for (int u = 0; u < kEPT; ++u) {
        float2 x = v[u];
        if (!SPLIT && a.mult) x = cmul(x, mv[u]);
        if (INV && a.phase) x = cmulcj(pv[u], x);
        v[u] = (live & (1u << u)) ? x : make_float2(0.f, 0.f);
    }
    tws.store(tw, K);
#pragma unroll
    for (int u = 0; u < kEPT; ++u) {
        const int e = threadIdx.x + u * THREADS;
        if (e < ne) s[e] = v[u];
    }
    __syncthreads();
    lds_fft<THREADS, INV, true>(s, W, K, 1, W, a.rp, tw);
    // Lout * W <= K * W outputs
    const int no = a.Lout * W;
    if (!INV && a.phase) {
#pragma unroll
        for (int u = 0; u < kEPT; ++u) {
            const int e = min(int(threadIdx.x) + u * THREADS, no - 1);
            pv[u] = a.phase[byW.div(e)];
        }
    }
    // values first, without branches, then the writes
#pragma unroll
    for (int u = 0; u < kEPT; ++u) {
        const int e = min(int(threadIdx.x) + u * THREADS, no - 1);
        const int i = byW.div(e);
        const int q = INV ? pad_pos(i, a.Lout, K) : i;
        float2 x = s[__umul24(q, W) + byW.rem(e, i)];
        if (!INV && a.phase) x = cmul(x, pv[u]);
        v[u] = x;
    }
#pragma unroll
    for (int u = 0; u < kEPT; ++u) {
        const int e = threadIdx.x + u * THREADS;
        const int i = byW.div(min(e, no - 1));
        const int w = e - __umul24(i, W);
        if (e < no && w < wv) out[int64_t(i) * a.inner + w] = v[u];
    }
}

template <int THREADS, bool INV, bool SPLIT>
__global__ __launch_bounds__(THREADS) void k_strided_pass(StridedPassArgs a, int W, int64_t ntc) {
    strided_pass_body<THREADS, INV, SPLIT>(a, W, ntc, blockIdx.x);
}

template <int THREADS, bool INV, bool SPLIT>
__global__ __launch_bounds__(THREADS) void k_strided_pass_multi(const StridedJob *__restrict__ jobs,
                                                               const int4 *__restrict__ blocks) {
    const int4 b = blocks[blockIdx.x];
    const StridedJob &j = jobs[b.x];
    strided_pass_body<THREADS, INV, SPLIT>(j.a, j.W, j.ntc, b.y);
}

template <int THREADS>
__device__ __forceinline__ void last_pass_body(const LastPassArgs &a, int rows_per_wg, int coils_per_round, int64_t bx) {
    extern __shared__ float2 lds[];
    __shared__ float rsc[kMaxLinesPerWg];
    const int K = a.K, N = a.N, C = a.C;
    float2 *tw = lds;
    float2 *s = lds + K;
    const int64_t nrt = (a.rows + rows_per_wg - 1) / rows_per_wg;
    const int64_t b = bx / nrt;
    const int64_t r0 = (bx % nrt) * rows_per_wg;
    const int nr = int(min(int64_t(rows_per_wg), a.rows - r0));
    TwiddleStage<THREADS> tws;
    tws.load(a.tw, K);
    const float *slast = a.scale[a.d - 1];
    if (coils_per_round >= C) {
        const FastDiv byK(K), byN(N), byC(C);
        // all coils of the rows in one tile (nr * C * K <= THREADS * kEPT
        // elements, nr * N outputs): every load is issued before the first use.
        // Lane rr (< nr <= 64) of every wavefront holds row rr's scaling factor.
        RowScale rsf;
        rsf.load(a.d, a.Nax, a.scale, int(r0) + min(int(threadIdx.x & 63), nr - 1));
        const int nl = nr * C;
        const int ne = nl * K;
        float2 v[kEPT], pv[kEPT];
#pragma unroll
        for (int u = 0; u < kEPT; ++u) {
            const int e = min(int(threadIdx.x) + u * THREADS, ne - 1);  // (clamped: every load is in bounds)
            const int lw = byK.div(e);
            const int q = byK.rem(e, lw);
            const int rr = byC.div(lw), cc = byC.rem(lw, rr);
            v[u] = a.in[((b * C + cc) * a.rows + r0 + rr) * K + q];
            if (a.phase) pv[u] = a.phase[q];
        }
        if (a.phase) {
#pragma unroll
            for (int u = 0; u < kEPT; ++u) v[u] = cmulcj(pv[u], v[u]);
        }
        tws.store(tw, K);
#pragma unroll
        for (int u = 0; u < kEPT; ++u) {
            const int e = threadIdx.x + u * THREADS;
            if (e < ne) s[e] = v[u];
        }
        __syncthreads();
        lds_fft<THREADS, true, false>(s, nl, K, K, 1, a.rp, tw);
        const float rs = rsf.value();
        const int no = nr * N;
        float sv[kEPT];
#pragma unroll
        for (int u = 0; u < kEPT; ++u) {
            const int e = min(int(threadIdx.x) + u * THREADS, no - 1);
            sv[u] = slast[byN.rem(e, byN.div(e))];
        }
        // values first (one wait for the scaling-factor loads), then the writes
        float2 res[kEPT];
#pragma unroll
        for (int u = 0; u < kEPT; ++u) {
            const int e = min(int(threadIdx.x) + u * THREADS, no - 1);
            const int rr = byN.div(e), i = byN.rem(e, rr);
            const int q = pad_pos(i, N, K);
            float2 sum = make_float2(0.f, 0.f);
            if (a.coils) {
#pragma unroll 1
                for (int cc = 0; cc < C; ++cc)
                    sum = cadd(sum, cmulcj(a.coils[(int64_t(cc) * a.rows + r0 + rr) * N + i], s[(rr * C + cc) * K + q]));
            } else {
#pragma unroll 1
                for (int cc = 0; cc < C; ++cc) sum = cadd(sum, s[(rr * C + cc) * K + q]);
            }
            res[u] = cscale(sum, __shfl(rs, rr) * sv[u]);
        }
#pragma unroll
        for (int u = 0; u < kEPT; ++u) {
            const int e = threadIdx.x + u * THREADS;
            const int rr = byN.div(min(e, no - 1)), i = e - __umul24(rr, N);
            if (e < no) a.x[(b * a.rows + r0 + rr) * N + i] = res[u];
        }
        return;
    }
    // more coils than one tile holds (C * K > the tile): rounds of
    // coils_per_round coils summed in LDS accumulators after the tile
    tws.store(tw, K);
    if (threadIdx.x < nr) rsc[threadIdx.x] = row_scale(a.d, a.Nax, a.scale, int(r0) + threadIdx.x);
    float2 *acc = s + rows_per_wg * coils_per_round * K;
    for (int e = threadIdx.x; e < nr * N; e += THREADS) acc[e] = make_float2(0.f, 0.f);
    for (int c0 = 0; c0 < C; c0 += coils_per_round) {
        const int nc = min(coils_per_round, C - c0);
        const int nl = nr * nc;
        for (int e = threadIdx.x; e < nl * K; e += THREADS) {
            const int lw = e / K, q = e - lw * K;
            const int rr = lw / nc, cc = lw - rr * nc;
            float2 v = a.in[((b * C + c0 + cc) * a.rows + r0 + rr) * K + q];
            if (a.phase) v = cmulcj(a.phase[q], v);
            s[e] = v;
        }
        __syncthreads();
        lds_fft<THREADS, true, false>(s, nl, K, K, 1, a.rp, tw);
        for (int e = threadIdx.x; e < nr * N; e += THREADS) {
            const int rr = e / N, i = e - rr * N;
            const int q = pad_pos(i, N, K);
            float2 sum = make_float2(0.f, 0.f);
            for (int cc = 0; cc < nc; ++cc) {
                float2 t = s[(rr * nc + cc) * K + q];
                if (a.coils) t = cmulcj(a.coils[(int64_t(c0 + cc) * a.rows + r0 + rr) * N + i], t);
                sum = cadd(sum, t);
            }
            acc[e] = cadd(acc[e], sum);
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < nr * N; e += THREADS) {
        const int rr = e / N, i = e - rr * N;
        a.x[(b * a.rows + r0 + rr) * N + i] = cscale(acc[e], rsc[rr] * slast[i]);
    }
}

template <int THREADS>
__global__ __launch_bounds__(THREADS) void k_last_pass(LastPassArgs a, int rows_per_wg, int coils_per_round) {
    last_pass_body<THREADS>(a, rows_per_wg, coils_per_round, blockIdx.x);
}

template <int THREADS>
__global__ __launch_bounds__(THREADS) void k_last_pass_multi(const LastJob *__restrict__ jobs,
                                                            const int4 *__restrict__ blocks) {
    const int4 b = blocks[blockIdx.x];
    const LastJob &j = jobs[b.x];
    last_pass_body<THREADS>(j.a, j.rpw, j.cpr, b.y);
}

// ------------------------------------------------------------ interpolation window
// k0 mod K for an integer-valued k0 (|k0| <= 1e15, checked when the plan is
// made).  Trajectories inside [-pi, pi) give |k0| <= K/2 + J/2 < K, handled
// without the 64-bit division the general case needs.
__device__ __forceinline__ int wrap_first_tap(double k0, int K) {
    const double Kd = double(K);
    if (k0 >= 0.0 && k0 < Kd) return int(k0);
    if (k0 < 0.0 && k0 >= -Kd) return int(k0) + K;
    long long kw = static_cast<long long>(k0) % K;
    if (kw < 0) kw += K;
    return int(kw);
}


// First tap k0 = floor(u - J/2) + 1 with u = omega * K/(2 pi) in float64, the
// J wrapped grid indices and the offset f = u - k0 - (J/2 - 1) in [0, 1).
template <int J>
__device__ __forceinline__ float window_pos(const SampleGeom &geo, int ax, float om, int *kk) {
    const double u = __dmul_rn(double(om), geo.C[ax]);
    const double k0 = floor(u - 0.5 * J) + 1.0;
    const float f = float(u - k0 - (0.5 * J - 1.0));
    const int K = geo.K[ax];
    const int kw = wrap_first_tap(k0, K);
#pragma unroll
    for (int j = 0; j < J; ++j) {
        int k = kw + j;
        kk[j] = k >= K ? k - K : k;
    }
    return f;
}

// Min-max interpolator: the coefficients are c_j = e^{i gamma t_j / 2} c'_j
// with c' the real fitted factors, and e^{i gamma t_j / 2} =
// e^{i omega / 2} (-1)^{floor(k0 / K)} (-1)^{[k0 mod K + j >= K]} e^{-i pi k_w / K}
// (k_w the wrapped grid index).  The FFT passes apply e^{-i pi k_w / K}; the
// sample kernels apply the rest: this per-sample phase (float64 angle) and a
// sign on taps that wrap past K.
template <int DIM>
__device__ __forceinline__ float2 mm_phase(const SampleGeom &geo, const float *om) {
    double ang = 0.0;
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) {
        const double u = __dmul_rn(double(om[ax]), geo.C[ax]);
        const double k0 = floor(u - 0.5 * geo.J) + 1.0;
        ang += 0.5 * double(om[ax]) + 3.141592653589793 * floor(k0 / double(geo.K[ax]));
    }
    double sn, cs;
    sincos(ang, &sn, &cs);
    return make_float2(float(cs), float(sn));
}

// First tap index j that wraps past K on axis `ax` (J or more: none).
__device__ __forceinline__ int mm_wrap_from(const SampleGeom &geo, int ax, float om) {
    const double u = __dmul_rn(double(om), geo.C[ax]);
    const double k0 = floor(u - 0.5 * geo.J) + 1.0;
    const int K = geo.K[ax];
    return K - wrap_first_tap(k0, K);
}

template <int NJ>
__device__ __forceinline__ void mm_sign_taps(float *w, int wrap_from) {
#pragma unroll
    for (int j = 0; j < NJ; ++j)
        if (j >= wrap_from) w[j] = -w[j];
}

// Per-tap polynomials of the kernel fit: NJ Horner chains in z over the
// coefficient rows (highest degree first, zero padded to a multiple of 2
// rows).  The table is the same for every lane, so it is read through the
// constant address space, which the compiler serves with scalar loads; a row
// pair is fetched at once instead of one dependent load per step.
typedef const __attribute__((address_space(4))) float const_float;

template <int NJ>
__device__ __forceinline__ void poly_rows(const float *rows, int jp, int nq, float z, float *w) {
    const_float *r = (const_float *)rows;
    float v[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) v[j] = 0.f;
    for (int q = 0; q < nq; q += 2) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
#pragma unroll
            for (int j = 0; j < NJ; ++j) v[j] = fmaf(v[j], z, r[(q + u) * jp + j]);
        }
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j) w[j] = v[j];
}

// w_j(f), j < J: the kernel weights of the window whose first tap is at
// fractional offset f.
template <int J>
__device__ __forceinline__ void window_weights(const SampleGeom &geo, const float *rows, int nq, float f, float *w) {
    poly_rows<J>(rows, geo.jp, nq, 2.0f * f - 1.0f, w);
}

// ---- the plan's window table (optional): one record per sorted sample
constexpr int table_taps_c(int J) { return J <= 6 ? 6 : J <= 8 ? 8 : 16; }
constexpr int table_f4(int DIM, int NJ) { return (2 + DIM * NJ + 3) / 4; }

// Window of sorted sample i on every axis: wrapped first taps and the NJ
// weights (zero past J), evaluated exactly as the table records them.
template <int NJ, int DIM>
__device__ __forceinline__ void eval_window(const SampleGeom &geo, const float *om, int *kw, float (*w)[NJ]) {
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) {
        const double u = __dmul_rn(double(om[ax]), geo.C[ax]);
        const double k0 = floor(u - 0.5 * geo.J) + 1.0;
        const float f = float(u - k0 - (0.5 * geo.J - 1.0));
        kw[ax] = wrap_first_tap(k0, geo.K[ax]);
        poly_rows<NJ>(geo.coef[ax], geo.jp, geo.nq[ax], 2.0f * f - 1.0f, w[ax]);
    }
}

// Unpacks a record already loaded as float4s.
template <int NJ, int DIM>
__device__ __forceinline__ void unpack_window(const float4 *r4, int *kw, float (*w)[NJ]) {
    float r[4 * table_f4(DIM, NJ)];
#pragma unroll
    for (int q = 0; q < table_f4(DIM, NJ); ++q) {
        r[4 * q] = r4[q].x;
        r[4 * q + 1] = r4[q].y;
        r[4 * q + 2] = r4[q].z;
        r[4 * q + 3] = r4[q].w;
    }
    const unsigned k01 = __float_as_uint(r[0]), k2 = __float_as_uint(r[1]);
    kw[0] = int(k01 & 0xffffu);
    if (DIM > 1) kw[1 < DIM ? 1 : 0] = int(k01 >> 16);
    if (DIM > 2) kw[2 < DIM ? 2 : 0] = int(k2 & 0xffffu);
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) {
#pragma unroll
        for (int j = 0; j < NJ; ++j) w[ax][j] = r[2 + ax * NJ + j];
    }
}

template <int NJ, int DIM>
__device__ __forceinline__ void load_window_record(const SampleGeom &geo, int64_t i, float4 *r4) {
    const float4 *src = reinterpret_cast<const float4 *>(geo.wtab + i * geo.wtab_stride);
#pragma unroll
    for (int q = 0; q < table_f4(DIM, NJ); ++q) r4[q] = src[q];
}

template <int NJ, int DIM>
__global__ __launch_bounds__(256) void k_weight_table(SampleGeom geo, const float *om_sorted, int64_t M, float *out) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= M) return;
    int kw[DIM];
    float w[DIM][NJ];
    eval_window<NJ, DIM>(geo, om_sorted + i * DIM, kw, w);
    float r[4 * table_f4(DIM, NJ)];
#pragma unroll
    for (int q = 0; q < 4 * table_f4(DIM, NJ); ++q) r[q] = 0.f;
    r[0] = __uint_as_float(unsigned(kw[0]) | (DIM > 1 ? unsigned(kw[1 < DIM ? 1 : 0]) << 16 : 0u));
    r[1] = __uint_as_float(DIM > 2 ? unsigned(kw[2 < DIM ? 2 : 0]) : 0u);
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) {
#pragma unroll
        for (int j = 0; j < NJ; ++j) r[2 + ax * NJ + j] = w[ax][j];
    }
    float4 *dst = reinterpret_cast<float4 *>(out + i * (4 * table_f4(DIM, NJ)));
#pragma unroll
    for (int q = 0; q < table_f4(DIM, NJ); ++q) dst[q] = make_float4(r[4 * q], r[4 * q + 1], r[4 * q + 2], r[4 * q + 3]);
}

// ------------------------------------------------------------ work distribution
// Work items (gather chunks, gridding tile chunks) are ordered by decreasing
// size on the host; workgroup b runs item b, and the hardware deals
// consecutive workgroups round-robin over the 8 XCDs, so the heavy items
// spread over the whole chip.

// ------------------------------------------------------------ V (gather)
// One workgroup per (bin, chunk), or per run of sparse tiles along the last
// axis: the tiles and their J-1 halo of the grid are staged in LDS once, then
// every sample of the item (window base inside the tiles) reads its J^d taps
// from LDS.
template <int J, int DIM>
__device__ __forceinline__ void interp_body(const InterpArgs &a, int64_t item) {
    extern __shared__ float2 reg[];
    const InterpItem it = a.items[item];
    int tc[DIM], base[DIM], E[DIM];
    {
        int t = it.bin;
#pragma unroll
        for (int ax = DIM - 1; ax >= 0; --ax) {
            tc[ax] = t % a.nt[ax];
            t /= a.nt[ax];
        }
    }
    // region: rows over the leading axes, each of P elements along the last
    // axis (its extent E made odd: the rows the lanes read then start in
    // different LDS banks)
    int rows = 1;
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) {
        base[ax] = tc[ax] * a.T[ax];
        // a run of it.tiles tiles along the last axis, plus the J - 1 halo
        E[ax] = (ax == DIM - 1 ? it.tiles : 1) * a.T[ax] + J - 1;
        if (ax < DIM - 1) rows *= E[ax];
    }
    const int P = E[DIM - 1] | 1;
    const int region = rows * P;
    constexpr int SPT = kInterpSamplesPerThread;
    float w[SPT][DIM][J];
    int off[SPT];
    bool valid[SPT];
    float2 ph[SPT];
    int dst[SPT];  // caller's index of the sample (loaded early, used by the final store)
#pragma unroll
    for (int k = 0; k < SPT; ++k) {
        const int s = threadIdx.x + k * 256;
        valid[k] = s < it.count;
        off[k] = 0;
        ph[k] = make_float2(1.f, 0.f);
        if (valid[k]) {
            const int64_t i = it.start + s;
            dst[k] = a.perm[i];
            int o = 0;
            if (a.geo.wtab) {
                // the window from the plan's table
                constexpr int NJ = table_taps_c(J);
                float4 r4[table_f4(DIM, NJ)];
                load_window_record<NJ, DIM>(a.geo, i, r4);
                int kw[DIM];
                float wt[DIM][NJ];
                unpack_window<NJ, DIM>(r4, kw, wt);
#pragma unroll
                for (int ax = 0; ax < DIM; ++ax) {
#pragma unroll
                    for (int j = 0; j < J; ++j) w[k][ax][j] = wt[ax][j];
                    o = o * (ax == DIM - 1 ? P : E[ax]) + (kw[ax] - base[ax]);
                }
            } else {
#pragma unroll
                for (int ax = 0; ax < DIM; ++ax) {
                    int kk[J];
                    const float f = window_pos<J>(a.geo, ax, a.om_sorted[i * DIM + ax], kk);
                    window_weights<J>(a.geo, a.geo.coef[ax], a.geo.nq[ax], f, w[k][ax]);
                    if (a.geo.minmax) mm_sign_taps<J>(w[k][ax], mm_wrap_from(a.geo, ax, a.om_sorted[i * DIM + ax]));
                    o = o * (ax == DIM - 1 ? P : E[ax]) + (kk[0] - base[ax]);
                }
            }
            off[k] = o;
            if (a.geo.minmax) ph[k] = mm_phase<DIM>(a.geo, a.om_sorted + i * DIM);
        }
    }
    // grid index of the first element of region row r (leading axes wrapped
    // at the grid's edge; the last axis is added by the caller)
    FastDiv byE1(DIM == 3 ? E[1] : 1);
    auto row_index = [&](int r) -> int64_t {
        if constexpr (DIM == 1) {
            return 0;
        } else if constexpr (DIM == 2) {
            int k0 = base[0] + r;
            if (k0 >= a.geo.K[0]) k0 -= a.geo.K[0];
            return int64_t(k0) * a.geo.K[1];
        } else {
            const int l0 = byE1.div(r);
            int k0 = base[0] + l0, k1 = base[1] + byE1.rem(r, l0);
            if (k0 >= a.geo.K[0]) k0 -= a.geo.K[0];
            if (k1 >= a.geo.K[1]) k1 -= a.geo.K[1];
            return (int64_t(k0) * a.geo.K[1] + k1) * a.geo.K[2];
        }
    };
    const int KL = a.geo.K[DIM - 1];
    const int H = (E[DIM - 1] + 1) >> 1;  // element pairs that cover a region row
    // pairs of the last axis in one 16-byte load: the grid's rows and the
    // region's first column must be even and the grid 16-byte aligned (a pair
    // then never straddles the wrap, K_last being even)
    const bool paired = (KL % 2 == 0) && (a.T[DIM - 1] % 2 == 0) && (a.grid_elems % 2 == 0) &&
                        (reinterpret_cast<uintptr_t>(a.G) % 16 == 0);
    // this thread's place in the row-major walk over the region's pairs: the
    // column stays fixed, the row advances by RP per round
    const int RP = H <= 256 ? 256 / H : 1;
    const int pr0 = H <= 256 ? int(threadIdx.x) / H : 0;
    const int pc = H <= 256 ? int(threadIdx.x) - pr0 * H : int(threadIdx.x);
    int kl = base[DIM - 1] + 2 * pc;  // grid column of the pair (< 2 K_last)
    if (kl >= KL) kl -= KL;
    for (int g = 0; g < a.grids; ++g) {
        const float2 *G = a.G + int64_t(g) * a.grid_elems;
        __syncthreads();
        constexpr int U = 8;  // loads in flight per thread
        if (paired && H <= 256) {
            // (2D regions are a few rows: 2 paired loads keep the registers,
            // and the occupancy, of the element path)
            constexpr int UP = DIM == 3 ? U : 2;
            // rows of the region, H lanes per row, RP rows per round: the
            // NR rounds go in batches of up to U whose loads are issued
            // together (rows past the region clamped to its last row, so
            // every load is in bounds, and not stored); idle lanes
            // (pr0 >= RP) skip
            const float4 *G4 = reinterpret_cast<const float4 *>(G);
            auto rows_batch = [&](int u0, auto nu) {
                constexpr int NU = decltype(nu)::value;
                float4 v[NU];
#pragma unroll
                for (int u = 0; u < NU; ++u)
                    v[u] = G4[(row_index(min(pr0 + (u0 + u) * RP, rows - 1)) + kl) >> 1];
#pragma unroll
                for (int u = 0; u < NU; ++u) {
                    const int r = pr0 + (u0 + u) * RP;
                    if (r < rows) {
                        float2 *dst = reg + r * P + 2 * pc;
                        dst[0] = make_float2(v[u].x, v[u].y);
                        if (2 * pc + 1 < P) dst[1] = make_float2(v[u].z, v[u].w);
                    }
                }
            };
            if (pr0 < RP) {
                const int NR = (rows + RP - 1) / RP;
                for (int u0 = 0; u0 < NR; u0 += UP) {
                    switch (min(UP, NR - u0)) {
                        case 1: rows_batch(u0, std::integral_constant<int, 1>()); break;
                        case 2: rows_batch(u0, std::integral_constant<int, 2>()); break;
                        case 3: rows_batch(u0, std::integral_constant<int, 3>()); break;
                        case 4: rows_batch(u0, std::integral_constant<int, 4>()); break;
                        case 5: rows_batch(u0, std::integral_constant<int, 5 <= UP ? 5 : 1>()); break;
                        case 6: rows_batch(u0, std::integral_constant<int, 6 <= UP ? 6 : 1>()); break;
                        case 7: rows_batch(u0, std::integral_constant<int, 7 <= UP ? 7 : 1>()); break;
                        default: rows_batch(u0, std::integral_constant<int, UP>()); break;
                    }
                }
            }
        } else {
            // element by element (odd tiles, unaligned grids, rows longer
            // than 512 elements), U elements per thread in flight
            FastDiv byP(P);
            for (int e0 = 0; e0 < region; e0 += U * 256) {
                float2 v[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int e = min(e0 + u * 256 + int(threadIdx.x), region - 1);
                    const int r = byP.div(e);
                    int k = base[DIM - 1] + byP.rem(e, r);
                    if (k >= KL) k -= KL;
                    v[u] = G[row_index(r) + k];
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int e = e0 + u * 256 + threadIdx.x;
                    if (e < region) reg[e] = v[u];
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < SPT; ++k) {
            if (!valid[k]) continue;
            float2 acc = make_float2(0.f, 0.f);
            const float2 *r0 = reg + off[k];
            if constexpr (DIM == 1) {
#pragma unroll
                for (int j = 0; j < J; ++j) acc = cadd(acc, cscale(r0[j], w[k][0][j]));
            } else if constexpr (DIM == 2) {
#pragma unroll
                for (int j0 = 0; j0 < J; ++j0) {
                    const float2 *row = r0 + j0 * P;
                    float2 rs = make_float2(0.f, 0.f);
#pragma unroll
                    for (int j1 = 0; j1 < J; ++j1) rs = cadd(rs, cscale(row[j1], w[k][1][j1]));
                    acc = cadd(acc, cscale(rs, w[k][0][j0]));
                }
            } else {
                for (int j0 = 0; j0 < J; ++j0) {
                    float2 ps = make_float2(0.f, 0.f);
#pragma unroll
                    for (int j1 = 0; j1 < J; ++j1) {
                        const float2 *row = r0 + (j0 * E[1] + j1) * P;
                        float2 rs = make_float2(0.f, 0.f);
#pragma unroll
                        for (int j2 = 0; j2 < J; ++j2) rs = cadd(rs, cscale(row[j2], w[k][2][j2]));
                        ps = cadd(ps, cscale(rs, w[k][1][j1]));
                    }
                    acc = cadd(acc, cscale(ps, w[k][0][j0]));
                }
            }
            if (a.geo.minmax) acc = cmul(acc, ph[k]);
            a.y[int64_t(g) * a.M + dst[k]] = acc;
        }
    }
}

template <int J, int DIM>
__global__ __launch_bounds__(256) void k_interp(InterpArgs a) {
    interp_body<J, DIM>(a, blockIdx.x);
}

template <int J, int DIM>
__global__ __launch_bounds__(256) void k_interp_multi(const InterpArgs *__restrict__ jobs,
                                                     const int4 *__restrict__ blocks) {
    const int4 b = blocks[blockIdx.x];
    interp_body<J, DIM>(jobs[b.x], b.y);
}

// Gather straight from the grid (L1/L2), one thread per sorted sample: used
// when the tile-plus-halo region does not fit the LDS budget.
template <int J, int DIM>
__device__ __forceinline__ void interp_direct_body(const InterpArgs &a, int64_t bx) {
    const int64_t i = bx * 256 + threadIdx.x;
    if (i >= a.M) return;
    float w[DIM][J];
    int kk[DIM][J];
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) {
        const float f = window_pos<J>(a.geo, ax, a.om_sorted[i * DIM + ax], kk[ax]);
        window_weights<J>(a.geo, a.geo.coef[ax], a.geo.nq[ax], f, w[ax]);
        if (a.geo.minmax) mm_sign_taps<J>(w[ax], mm_wrap_from(a.geo, ax, a.om_sorted[i * DIM + ax]));
    }
    const float2 ph = a.geo.minmax ? mm_phase<DIM>(a.geo, a.om_sorted + i * DIM) : make_float2(1.f, 0.f);
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
        if (a.geo.minmax) acc = cmul(acc, ph);
        a.y[int64_t(g) * a.M + m] = acc;
    }
}

template <int J, int DIM>
__global__ __launch_bounds__(256) void k_interp_direct(InterpArgs a) {
    interp_direct_body<J, DIM>(a, blockIdx.x);
}

template <int J, int DIM>
__global__ __launch_bounds__(256) void k_interp_direct_multi(const InterpArgs *__restrict__ jobs,
                                                            const int4 *__restrict__ blocks) {
    const int4 b = blocks[blockIdx.x];
    interp_direct_body<J, DIM>(jobs[b.x], b.y);
}

// ------------------------------------------------------------ V^H (output-driven gridding)
// One workgroup per (tile, chunk).  The samples that reach the tile are the
// tile's own bin plus, from each lower neighbour bin, only the sub-bins whose
// windows cross into this tile (tile_segments).
//
// No atomics: the tile's rows (leading coordinates) are cut into segments of
// LS cells along the last axis, one segment per lane, held in registers.
// Samples are staged in LDS in batches: window offsets along the leading
// axes, their per-axis weights, the value, and the last-axis weights already
// expanded into a zero-padded row of the tile (so the inner loop needs no
// tap index and no branch).  Every lane of a group then walks the group's
// batch and adds LS weighted values per sample.  Lane groups split the
// samples; their register tiles are summed through LDS at the end in group
// order, so the result does not depend on scheduling.
constexpr int kGridThreads = 256;

// Synchronise a lane group's LDS traffic: a single wavefront only needs its
// own LDS operations ordered (lockstep execution), larger groups need the
// workgroup barrier.
__device__ __forceinline__ void group_sync(int gsize) {
    if (gsize == 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// The sorted-sample segments that reach the work item's tile (its own bin and
// the crossing sub-bins of its lower neighbours, in tile_segments order), from
// the item's table made when the plan was built: segment starts into seg_lo,
// their offsets in the item's sample list (and the total) into seg_pre.  Needs
// nothing from the item record, so both loads are in flight together.  Every
// thread of the workgroup calls it; returns the number of segments.
__device__ __forceinline__ int grid_item_segments(const GridArgs &a, int64_t item, int *seg_lo, int *seg_pre) {
    constexpr int kSegRow = kMaxNeighbors + 1;
    if (threadIdx.x <= a.n_kinds) {
        const int2 e = a.item_segs[item * kSegRow + threadIdx.x];
        seg_lo[threadIdx.x] = e.x;
        seg_pre[threadIdx.x] = e.y;
    }
    __syncthreads();
    return a.n_kinds;
}

// Segment of item sample f (the last segment whose start is <= f) for a batch
// of consecutive samples fb .. fb + span - 1.  `cursor` is uniform over the
// batch's lanes and kept across the item's batches, which only move forward:
// it is advanced to the batch's first sample, then every segment start inside
// the batch adds one for the lanes at or past it.  The same segment as a scan
// from segment 0, without a divergent per-lane loop.
__device__ __forceinline__ int batch_segment(const int *seg_pre, int nseg, int &cursor, int fb, int span, int f) {
    while (cursor + 1 < nseg && seg_pre[cursor + 1] <= fb) ++cursor;
    int sg = cursor;
    for (int k = cursor + 1; k < nseg && seg_pre[k] < fb + span; ++k) sg += seg_pre[k] <= f ? 1 : 0;
    return sg;
}

template <int DIM, int LS, int JP>
__device__ __forceinline__ void grid_body(const GridArgs &a, int64_t item, int g) {
    extern __shared__ float4 stage_mem[];  // float4: 16-byte aligned rows for the vector reads
    float *stage = reinterpret_cast<float *>(stage_mem);
    __shared__ int seg_lo[kMaxNeighbors + 1];
    __shared__ int seg_pre[kMaxNeighbors + 1];
    const GridItem it = a.items[item];
    const int nseg = grid_item_segments(a, item, seg_lo, seg_pre);
    const int J = a.geo.J;
    const int L = a.T[DIM - 1];           // cells per tile row
    const int S = a.segs;                 // segments per row
    const int Lp = S * LS;                // padded row length
    const int lead = a.tile_cells / L;    // rows of the tile
    const int gsize = a.group_lanes;      // lanes per sample group (multiple of 64, >= lead * S)
    const int ngroups = kGridThreads / gsize;
    const int grp = threadIdx.x / gsize;
    const int lane = threadIdx.x - grp * gsize;
    const int B = gsize;                  // samples per batch and group
    const int BP = B + 1;
    // staged arrays of this group
    float *gbase = stage + grp * a.stage_floats;
    float *wrow = gbase;                              // [B][Lp] last-axis weights on the row
    float *sv = wrow + B * Lp;                        // [2][BP] value
    int *so = reinterpret_cast<int *>(sv + 2 * BP);   // [DIM-1][BP] leading first-tap offsets
    float *sw = sv + 2 * BP + (DIM - 1) * BP;         // [DIM-1][J][BP] leading weights

    int tc[DIM];
    {
        int t = it.tile;
#pragma unroll
        for (int ax = DIM - 1; ax >= 0; --ax) {
            tc[ax] = t % a.nt[ax];
            t /= a.nt[ax];
        }
    }
    const int total = seg_pre[nseg];
    const int f0 = it.chunk * a.chunk;
    const int n = min(total, f0 + a.chunk) - f0;
    int base[DIM];
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) base[ax] = tc[ax] * a.T[ax];
    // this lane's segment: row (leading coordinates) and first cell
    const int row = lane / S;
    const int cseg = (lane - row * S) * LS;
    int lc[DIM];
    {
        int r = row;
#pragma unroll
        for (int ax = DIM - 2; ax >= 0; --ax) {
            lc[ax] = r % a.T[ax];
            r /= a.T[ax];
        }
        lc[DIM - 1] = cseg;
    }
    const bool row_ok = row < lead;
    const float2 *y = a.y + int64_t(g) * a.M;
    float2 acc[LS];
#pragma unroll
    for (int c = 0; c < LS; ++c) acc[c] = make_float2(0.f, 0.f);

    // A group of one wavefront stages and consumes its own batches, so it
    // synchronises only with itself and runs ahead of the other groups.
    const int per_iter = B * ngroups;
    int cursor = 0;
    for (int b0 = 0; b0 < n; b0 += per_iter) {
        // ---- stage one batch per group: lane `lane` stages sample b0 + grp*B + lane
        const int s_idx = b0 + grp * B + lane;
        const int sg = batch_segment(seg_pre, nseg, cursor, f0 + b0 + grp * B, B, f0 + s_idx);
        if (s_idx < n) {
            const int f = f0 + s_idx;
            const int64_t i = seg_lo[sg] + (f - seg_pre[sg]);
            float wl_row[JP];  // last-axis weights, spread on the row below
            int o_last = 0;
#pragma unroll
            for (int ax = 0; ax < DIM; ++ax) {
                const double u = __dmul_rn(double(a.om_sorted[i * DIM + ax]), a.geo.C[ax]);
                // (min-max: taps wrapping past K carry a sign, see mm_phase)
                const double k0 = floor(u - 0.5 * J) + 1.0;
                const float fr = float(u - k0 - (0.5 * J - 1.0));
                const int K = a.geo.K[ax];
                const int kw = wrap_first_tap(k0, K);
                int o = kw - base[ax];
                if (a.nt[ax] > 1 && o >= a.T[ax]) o -= K;  // window wrapping in from the top
                const float z = 2.0f * fr - 1.0f;
                float wv[JP];
                poly_rows<JP>(a.geo.coef[ax], JP, a.geo.nq[ax], z, wv);
                if (a.geo.minmax) mm_sign_taps<JP>(wv, K - int(kw));
#pragma unroll
                for (int j = 0; j < JP; ++j) {
                    if (j < J) {
                        if (ax < DIM - 1)
                            sw[(ax * J + j) * BP + lane] = wv[j];
                        else
                            wl_row[j] = wv[j];
                    }
                }
                if (ax < DIM - 1) so[ax * BP + lane] = o;
                else o_last = o;
            }
            // the tile row of last-axis weights: cell c gets w[c - o] (wrapping
            // when the axis is one tile), built in registers and stored with
            // 16-byte writes
            const int Kl = a.geo.K[DIM - 1];
            const bool wrapl = a.nt[DIM - 1] == 1;
            float4 *wr4 = reinterpret_cast<float4 *>(wrow + lane * Lp);
            for (int c4 = 0; c4 < Lp; c4 += 4) {
                float r[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    int j = c4 + u - o_last;
                    if (wrapl && j < 0) j += Kl;
                    float v = 0.f;
#pragma unroll
                    for (int jj = 0; jj < JP; ++jj)
                        if (jj < J && j == jj) v = wl_row[jj];
                    r[u] = (c4 + u < L) ? v : 0.f;
                }
                wr4[c4 >> 2] = make_float4(r[0], r[1], r[2], r[3]);
            }
            float2 v = a.y_sorted ? y[i] : y[a.perm[i]];
            if (a.geo.minmax) v = cmulcj(mm_phase<DIM>(a.geo, a.om_sorted + i * DIM), v);
            sv[lane] = v.x;
            sv[BP + lane] = v.y;
        }
        group_sync(gsize);
        // ---- every lane of the group walks the group's batch
        const int nb = min(B, n - (b0 + grp * B));
#pragma unroll 2
        for (int s = 0; s < nb; ++s) {
            float wl = row_ok ? 1.f : 0.f;
#pragma unroll
            for (int ax = 0; ax < DIM - 1; ++ax) {
                int j = lc[ax] - so[ax * BP + s];
                if (a.nt[ax] == 1 && j < 0) j += a.geo.K[ax];
                const bool in = (j >= 0) && (j < J);
                const float w = sw[(ax * J + (in ? j : 0)) * BP + s];
                wl = in ? wl * w : 0.f;
            }
            const float vr = sv[s] * wl, vi = sv[BP + s] * wl;
            const float4 *wr4 = reinterpret_cast<const float4 *>(wrow + s * Lp + cseg);
#pragma unroll
            for (int q = 0; q < LS / 4; ++q) {
                const float4 w = wr4[q];
                acc[4 * q + 0].x = fmaf(w.x, vr, acc[4 * q + 0].x);
                acc[4 * q + 0].y = fmaf(w.x, vi, acc[4 * q + 0].y);
                acc[4 * q + 1].x = fmaf(w.y, vr, acc[4 * q + 1].x);
                acc[4 * q + 1].y = fmaf(w.y, vi, acc[4 * q + 1].y);
                acc[4 * q + 2].x = fmaf(w.z, vr, acc[4 * q + 2].x);
                acc[4 * q + 2].y = fmaf(w.z, vi, acc[4 * q + 2].y);
                acc[4 * q + 3].x = fmaf(w.w, vr, acc[4 * q + 3].x);
                acc[4 * q + 3].y = fmaf(w.w, vi, acc[4 * q + 3].y);
            }
        }
        group_sync(gsize);
    }
    // ---- combine the groups' register tiles (group order), write the tile
    float2 *red = reinterpret_cast<float2 *>(stage);  // [ngroups][lead][Lp], reuses the staging LDS
    const bool seg_ok = row_ok;
    if (ngroups > 1) {
        __syncthreads();  // every group is done with its staging area
        if (seg_ok) {
#pragma unroll
            for (int c = 0; c < LS; ++c) red[(grp * lead + row) * Lp + cseg + c] = acc[c];
        }
        __syncthreads();
    }
    const bool to_partial = it.nchunks > 1;
    float2 *dst = to_partial ? a.partials + (int64_t(g) * a.n_slots + it.slot + it.chunk) * a.tile_cells
                             : a.h + int64_t(g) * a.grid_elems;
    if (ngroups == 1) {
        if (seg_ok) {
            int64_t idx;
            if (to_partial) {
                idx = int64_t(row) * L + cseg;
            } else {
                idx = 0;
#pragma unroll
                for (int ax = 0; ax < DIM; ++ax) idx = idx * a.geo.K[ax] + base[ax] + lc[ax];
            }
#pragma unroll
            for (int c = 0; c < LS; ++c)
                if (cseg + c < L) dst[idx + c] = acc[c];
        }
    } else {
        for (int e = threadIdx.x; e < lead * L; e += kGridThreads) {
            const int r = e / L, c = e - r * L;
            float2 sum = red[r * Lp + c];
            for (int q = 1; q < ngroups; ++q) sum = cadd(sum, red[(q * lead + r) * Lp + c]);
            int64_t idx;
            if (to_partial) {
                idx = e;
            } else {
                int rr = r;
                int l[DIM];
                l[DIM - 1] = c;
#pragma unroll
                for (int ax = DIM - 2; ax >= 0; --ax) {
                    l[ax] = rr % a.T[ax];
                    rr /= a.T[ax];
                }
                idx = 0;
#pragma unroll
                for (int ax = 0; ax < DIM; ++ax) idx = idx * a.geo.K[ax] + base[ax] + l[ax];
            }
            dst[idx] = sum;
        }
    }
}

template <int DIM, int LS, int JP>
__global__ __launch_bounds__(kGridThreads) void k_grid(GridArgs a) {
    grid_body<DIM, LS, JP>(a, blockIdx.x, blockIdx.y);
}

template <int DIM, int LS, int JP>
__global__ __launch_bounds__(kGridThreads) void k_grid_multi(const GridArgs *__restrict__ jobs,
                                                            const int4 *__restrict__ blocks) {
    const int4 b = blocks[blockIdx.x];
    grid_body<DIM, LS, JP>(jobs[b.x], b.y, b.z);
}

// V^H on the matrix cores, for tiles of 16*MB rows (the leading axes) by 16
// cells (last axis).  Over a batch of samples s the tile is
//   H[r][c] = sum_s (v_s * wlead_s[r]) * wlast_s[c],
// a product of a rows x samples matrix and a samples x 16 matrix, i.e.
// 16x16x4 fp32 MFMAs with the samples as the reduction dimension (real and
// imaginary parts as two products sharing the wlast operand).  Each wave
// stages 64 samples in LDS: the values of the GP grids the workgroup grids
// (coils or batch entries share the trajectory, so the window weights are
// staged once for all of them) and, per axis, the sample's weights spread
// over the tile's T_a coordinates (zero outside the window, window wrapping
// resolved here), so in the walk lane (i + 16k) reads A[i][k] and B[k][i] of
// sample k at fixed offsets.  The four waves take different samples of the
// item and their tiles are summed in LDS in wave order (deterministic).
typedef float mfma_f4 __attribute__((ext_vector_type(4)));

template <int DIM, int NJ, int MB, int GP, bool TAB>
__device__ __forceinline__ void grid_mfma_body(const GridArgs &a, int64_t item, int gg) {
    extern __shared__ float mf_lds[];
    __shared__ int seg_lo[kMaxNeighbors + 1];
    __shared__ int seg_pre[kMaxNeighbors + 1];
    const GridItem it = a.items[item];
    const int nseg = grid_item_segments(a, item, seg_lo, seg_pre);
    const int J = a.geo.J;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wavefront
    const int lane = threadIdx.x & 63;
    const int g0 = gg * GP;                        // first grid of this workgroup
    const int ng = min(GP, a.grids - g0);          // grids it writes
    int tsum = 0;
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) tsum += a.T[ax];
    const int RS = (2 * GP + tsum) | 1;  // floats per staged sample: GP values, then T_a weights per axis (odd)
    float *rec = mf_lds + wave * 64 * RS;

    int tc[DIM];
    {
        int t = it.tile;
#pragma unroll
        for (int ax = DIM - 1; ax >= 0; --ax) {
            tc[ax] = t % a.nt[ax];
            t /= a.nt[ax];
        }
    }
    const int total = seg_pre[nseg];
    const int f0 = it.chunk * a.chunk;
    const int n = min(total, f0 + a.chunk) - f0;
    int base[DIM], off[DIM];
    {
        int o = 2 * GP;
#pragma unroll
        for (int ax = 0; ax < DIM; ++ax) {
            base[ax] = tc[ax] * a.T[ax];
            off[ax] = o;
            o += a.T[ax];
        }
    }

    // this lane's record offsets: A operand (leading weights of row
    // 16 blk + rl, per row block) and B operand (last-axis weight of column rl)
    const int rl = lane & 15;
    const int kq = lane >> 4;
    int aoff[MB][DIM - 1];
#pragma unroll
    for (int blk = 0; blk < MB; ++blk) {
        int r = blk * 16 + rl;
#pragma unroll
        for (int ax = DIM - 2; ax >= 0; --ax) {
            aoff[blk][ax] = off[ax] + r % a.T[ax];
            r /= a.T[ax];
        }
    }
    const int boff = off[DIM - 1] + rl;
    mfma_f4 acc_re[GP][MB], acc_im[GP][MB];
#pragma unroll
    for (int q = 0; q < GP; ++q) {
#pragma unroll
        for (int blk = 0; blk < MB; ++blk) {
            acc_re[q][blk] = mfma_f4{0.f, 0.f, 0.f, 0.f};
            acc_im[q][blk] = mfma_f4{0.f, 0.f, 0.f, 0.f};
        }
    }
    // The global reads of a batch (trajectory, sample values) are issued one
    // batch ahead, so they are in flight while the wave walks the current one.
    float pom[DIM];
    float4 prec[TAB ? table_f4(DIM, NJ) : 1];
    float2 pv[GP];
    bool pvalid = false;
    int cursor = 0;
    auto fetch = [&](int b) {
        const int s_idx = b + wave * 64 + lane;
        pvalid = s_idx < n;
        const int sg = batch_segment(seg_pre, nseg, cursor, f0 + b + wave * 64, 64, f0 + s_idx);
        if (pvalid) {
            const int f = f0 + s_idx;
            const int64_t i = seg_lo[sg] + (f - seg_pre[sg]);
            if constexpr (TAB) {
                load_window_record<NJ, DIM>(a.geo, i, prec);
            } else {
#pragma unroll
                for (int ax = 0; ax < DIM; ++ax) pom[ax] = a.om_sorted[i * DIM + ax];
            }
            const int64_t src = a.y_sorted ? i : int64_t(a.perm[i]);
#pragma unroll
            for (int q = 0; q < GP; ++q)
                pv[q] = q < ng ? a.y[int64_t(g0 + q) * a.M + src] : make_float2(0.f, 0.f);
        }
    };
    fetch(0);
    for (int b0 = 0; b0 < n; b0 += 256) {
        // ---- stage: lane = sample b0 + 64 * wave + lane of the item
        float *my = rec + lane * RS;
        {
            float2 ph = make_float2(1.f, 0.f);
            if constexpr (!TAB)
                if (pvalid && a.geo.minmax) ph = mm_phase<DIM>(a.geo, pom);
#pragma unroll
            for (int q = 0; q < GP; ++q) {
                const float2 v = pvalid ? (a.geo.minmax ? cmulcj(ph, pv[q]) : pv[q]) : make_float2(0.f, 0.f);
                my[2 * q] = v.x;
                my[2 * q + 1] = v.y;
            }
        }
        int kwa[DIM];
        float wva[DIM][NJ];
        if (pvalid) {
            if constexpr (TAB)
                unpack_window<NJ, DIM>(prec, kwa, wva);
            else
                eval_window<NJ, DIM>(a.geo, pom, kwa, wva);
        }
#pragma unroll
        for (int ax = 0; ax < DIM; ++ax) {
            float *E = my + off[ax];
            const int T = a.T[ax];
#pragma unroll 4
            for (int x = 0; x < T; ++x) E[x] = 0.f;
            if (pvalid) {
                const int K = a.geo.K[ax];
                const int kw = kwa[ax];
                const int o = kw - base[ax];  // first tap relative to the tile, in [-base, K - base)
                float *wv = wva[ax];
                if (a.geo.minmax) mm_sign_taps<NJ>(wv, K - kw);
#pragma unroll
                for (int j = 0; j < NJ; ++j) {
                    if (j < J) {
                        int x = o + j;
                        if (x >= K) x -= K;  // taps wrapping past the top of the axis
                        if (x >= 0 && x < T) E[x] = wv[j];
                    }
                }
            }
        }
        if (b0 + 256 < n) fetch(b0 + 256);
        group_sync(64);
        // ---- walk: 4 samples per step
        const int nb = min(64, n - (b0 + wave * 64));
#pragma unroll 2
        for (int st = 0; st * 4 < nb; ++st) {
            const float *sr = rec + (st * 4 + kq) * RS;
            float vx[GP], vy[GP];
#pragma unroll
            for (int q = 0; q < GP; ++q) {
                vx[q] = sr[2 * q];
                vy[q] = sr[2 * q + 1];
            }
            const float bw = sr[boff];
#pragma unroll
            for (int blk = 0; blk < MB; ++blk) {
                float wl = sr[aoff[blk][0]];
#pragma unroll
                for (int ax = 1; ax < DIM - 1; ++ax) wl *= sr[aoff[blk][ax]];
#pragma unroll
                for (int q = 0; q < GP; ++q) {
                    acc_re[q][blk] = __builtin_amdgcn_mfma_f32_16x16x4f32(vx[q] * wl, bw, acc_re[q][blk], 0, 0, 0);
                    acc_im[q][blk] = __builtin_amdgcn_mfma_f32_16x16x4f32(vy[q] * wl, bw, acc_im[q][blk], 0, 0, 0);
                }
            }
        }
        group_sync(64);
    }
    // ---- per grid: sum the waves' tiles in wave order and write the tile
    const int cells = MB * 256;
    float2 *red = reinterpret_cast<float2 *>(mf_lds);  // [4][cells], reuses the staging LDS
#pragma unroll
    for (int q = 0; q < GP; ++q) {
        __syncthreads();  // every wave is done with the staging area / the previous grid's sums
#pragma unroll
        for (int blk = 0; blk < MB; ++blk) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = blk * 16 + 4 * kq + r;  // D[row][col] sits in lane col + 16 (row / 4), register row % 4
                red[wave * cells + row * 16 + rl] = make_float2(acc_re[q][blk][r], acc_im[q][blk][r]);
            }
        }
        __syncthreads();
        if (q < ng) {
            const int g = g0 + q;
            const bool to_partial = it.nchunks > 1;
            float2 *dst = to_partial ? a.partials + (int64_t(g) * a.n_slots + it.slot + it.chunk) * a.tile_cells
                                     : a.h + int64_t(g) * a.grid_elems;
            for (int e = threadIdx.x; e < cells; e += 256) {
                float2 sum = red[e];
#pragma unroll
                for (int w = 1; w < 4; ++w) sum = cadd(sum, red[w * cells + e]);
                int64_t idx;
                if (to_partial) {
                    idx = e;
                } else {
                    int rr = e >> 4;
                    int l[DIM];
                    l[DIM - 1] = e & 15;
#pragma unroll
                    for (int ax = DIM - 2; ax >= 0; --ax) {
                        l[ax] = rr % a.T[ax];
                        rr /= a.T[ax];
                    }
                    idx = 0;
#pragma unroll
                    for (int ax = 0; ax < DIM; ++ax) idx = idx * a.geo.K[ax] + base[ax] + l[ax];
                }
                dst[idx] = sum;
            }
        }
    }
}

template <int DIM, int NJ, int MB, int GP, bool TAB>
__global__ __launch_bounds__(256) void k_grid_mfma(GridArgs a) {
    grid_mfma_body<DIM, NJ, MB, GP, TAB>(a, blockIdx.x, blockIdx.y);
}

template <int DIM, int NJ, int MB, int GP, bool TAB>
__global__ __launch_bounds__(256) void k_grid_mfma_multi(const GridArgs *__restrict__ jobs,
                                                        const int4 *__restrict__ blocks) {
    const int4 b = blocks[blockIdx.x];
    grid_mfma_body<DIM, NJ, MB, GP, TAB>(jobs[b.x], b.y, b.z);
}

// V^H on the matrix cores in 3D, by blocks.  The tile is T0 x T1 x 16 (T0,
// T1 in {8, 16}, at most 8 blocks); its leading axes are cut into 4 x 4
// blocks, and a block with the 16 cells of the last axis is one 16 x 16
// product over the samples:
//   H[(x0, x1)][x2] = sum_s (v_s w0_s[x0] w1_s[x1]) w2_s[x2]
// (v_mfma_f32_16x16x4_f32, samples as the reduction dimension, real and
// imaginary parts sharing the w2 operand).  Each wavefront stages its own 64
// samples of a batch (value and per-axis weights spread over the tile's
// coordinates, out-of-tile taps to a discard slot, and the set of blocks the
// window reaches) and walks them four at a time over the blocks in
// registers, running only the products of blocks that one of the four
// reaches.  Wavefronts synchronise only with themselves until the end, where
// their tiles are summed in wave order (the result does not depend on
// scheduling).  With NW = 1 a work item is one wavefront, which writes its
// blocks straight from registers (no summation across wavefronts).
template <int NJ, int T0, int T1, bool TAB, int NW>
__device__ __forceinline__ void grid_blk_body(const GridArgs &a, int64_t item, int g) {
    constexpr int T2 = 16;
    constexpr int NB1 = T1 / 4;
    constexpr int NBLK = (T0 / 4) * NB1;
    constexpr int TRASH = 2;  // discard slot of a record
    constexpr int ROW[3] = {3, 3 + T0, 3 + T0 + T1};
    constexpr int TAX[3] = {T0, T1, T2};
    constexpr int RS = 3 + T0 + T1 + T2;  // floats per record (odd)
    constexpr int CELLS = T0 * T1 * T2;
    static_assert(RS % 2 == 1 && NBLK >= 4 && NBLK <= 8, "tile shape");
    extern __shared__ float blk_lds[];
    __shared__ int seg_lo[kMaxNeighbors + 1];
    __shared__ int seg_pre[kMaxNeighbors + 1];
    const GridItem it = a.items[item];
    const int nseg = grid_item_segments(a, item, seg_lo, seg_pre);
    const int J = a.geo.J;
    const int wave = NW == 1 ? 0 : __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    float *rec = blk_lds + wave * 64 * (RS + 1);                 // [64][RS]
    unsigned *smask = reinterpret_cast<unsigned *>(rec + 64 * RS);  // [64]

    int tc[3];
    {
        int t = it.tile;
#pragma unroll
        for (int ax = 2; ax >= 0; --ax) {
            tc[ax] = t % a.nt[ax];
            t /= a.nt[ax];
        }
    }
    const int base[3] = {tc[0] * T0, tc[1] * T1, tc[2] * T2};
    const int total = seg_pre[nseg];
    const int f0 = it.chunk * a.chunk;
    const int n = min(total, f0 + a.chunk) - f0;

    // walk roles: lane rl + 16 kq reads row rl of sample kq's A operand and
    // column rl of its B operand; block q covers x0 in 4 (q / NB1) + [0, 4),
    // x1 in 4 (q % NB1) + [0, 4), its row rl is (x0, x1) = (+rl / 4, +rl % 4)
    const int rl = lane & 15;
    const int kq = lane >> 4;
    const float2 *y = a.y + int64_t(g) * a.M;
    mfma_f4 acc_re[NBLK], acc_im[NBLK];
#pragma unroll
    for (int q = 0; q < NBLK; ++q) {
        acc_re[q] = mfma_f4{0.f, 0.f, 0.f, 0.f};
        acc_im[q] = mfma_f4{0.f, 0.f, 0.f, 0.f};
    }
    // trajectory (or window record) and value of this lane's next sample,
    // loaded one batch ahead
    float pom[TAB ? 1 : 3];
    float4 prec[TAB ? table_f4(3, NJ) : 1];
    float2 pv = make_float2(0.f, 0.f);
    bool pvalid = false;
    int cursor = 0;
    auto fetch = [&](int b) {
        const int s_idx = b + wave * 64 + lane;
        pvalid = s_idx < n;
        const int sg = batch_segment(seg_pre, nseg, cursor, f0 + b + wave * 64, 64, f0 + s_idx);
        if (pvalid) {
            const int64_t i = seg_lo[sg] + (f0 + s_idx - seg_pre[sg]);
            if constexpr (TAB) {
                load_window_record<NJ, 3>(a.geo, i, prec);
            } else {
#pragma unroll
                for (int ax = 0; ax < 3; ++ax) pom[ax] = a.om_sorted[i * 3 + ax];
            }
            pv = a.y_sorted ? y[i] : y[a.perm[i]];
        }
    };
    fetch(0);
    for (int b0 = 0; b0 < n; b0 += 64 * NW) {
        {
            float4 *z = reinterpret_cast<float4 *>(rec);
            for (int e = lane; e < 16 * RS; e += 64) z[e] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
        group_sync(64);
        // ---- stage this lane's sample
        unsigned mk = 0;
        if (pvalid) {
            float *my = rec + lane * RS;
            if constexpr (!TAB)
                if (a.geo.minmax) pv = cmulcj(mm_phase<3>(a.geo, pom), pv);
            my[0] = pv.x;
            my[1] = pv.y;
            unsigned bm[2] = {0u, 0u};
            int kwa[3];
            float wta[TAB ? 3 : 1][NJ];
            if constexpr (TAB) unpack_window<NJ, 3>(prec, kwa, wta);
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                const int K = a.geo.K[ax];
                float wv[NJ];
                int kw;
                if constexpr (TAB) {
                    kw = kwa[ax];
#pragma unroll
                    for (int j = 0; j < NJ; ++j) wv[j] = wta[ax][j];
                } else {
                    const double u = __dmul_rn(double(pom[ax]), a.geo.C[ax]);
                    const double k0 = floor(u - 0.5 * J) + 1.0;
                    const float fr = float(u - k0 - (0.5 * J - 1.0));
                    kw = wrap_first_tap(k0, K);
                    poly_rows<NJ>(a.geo.coef[ax], a.geo.jp, a.geo.nq[ax], 2.0f * fr - 1.0f, wv);
                    if (a.geo.minmax) mm_sign_taps<NJ>(wv, K - kw);
                }
                if (a.nt[ax] > 1) {
                    // first tap relative to the tile, in [-(J-1), T): a window
                    // wrapping in from the top of the axis comes in negative
                    int o = kw - base[ax];
                    if (o >= TAX[ax]) o -= K;
                    // taps past J carry zero weights (zero coefficient rows)
                    // and land outside the window: harmless either way
#pragma unroll
                    for (int j = 0; j < NJ; ++j) {
                        const int x = o + j;
                        my[unsigned(x) < unsigned(TAX[ax]) ? ROW[ax] + x : TRASH] = wv[j];
                    }
                    if (ax < 2) {
                        // blocks of 4 cells the window's cells in the tile fall in
                        const int c0 = max(o, 0), c1 = min(o + J - 1, TAX[ax] - 1);
                        bm[ax] = c0 <= c1 ? ((2u << (c1 >> 2)) - 1u) & ~((1u << (c0 >> 2)) - 1u) : 0u;
                    }
                } else {
                    // the axis is one tile: taps wrap around inside it
#pragma unroll
                    for (int j = 0; j < NJ; ++j) {
                        int x = kw + j;
                        if (x >= K) x -= K;
                        const bool in = j < J;
                        my[in ? ROW[ax] + x : TRASH] = wv[j];
                        if (ax < 2) bm[ax] |= in ? 1u << (x >> 2) : 0u;
                    }
                }
            }
#pragma unroll
            for (int b = 0; b < T0 / 4; ++b)
                if ((bm[0] >> b) & 1u) mk |= bm[1] << (b * NB1);
        }
        smask[lane] = mk;
        if (b0 + 64 * NW < n) fetch(b0 + 64 * NW);
        group_sync(64);
        // ---- walk: lane l < 16 looks at samples 4l .. 4l + 3 (one product's
        // worth) and the blocks they reach.  Block by block, the wavefront
        // runs the products with work for that block, two at a time with all
        // their operand reads issued first (one accumulator per loop, so it
        // stays in its registers).
        unsigned gm = 0;
        if (lane < 16) {
            const uint4 m4 = reinterpret_cast<const uint4 *>(smask)[lane];
            gm = m4.x | m4.y | m4.z | m4.w;
        }
#pragma unroll
        for (int q = 0; q < NBLK; ++q) {
            const int a0 = ROW[0] + 4 * (q / NB1) + (rl >> 2);
            const int a1 = ROW[1] + 4 * (q % NB1) + (rl & 3);
            uint64_t act = __ballot((gm >> q) & 1u);
            while (act) {
                const int g0 = int(__builtin_ctzll(act));
                act &= act - 1;
                const bool two = act != 0;
                const int g1 = two ? int(__builtin_ctzll(act)) : g0;
                act &= act - 1;
                const float *s0 = rec + (4 * g0 + kq) * RS;
                const float *s1 = rec + (4 * g1 + kq) * RS;
                const float vx0 = s0[0], vy0 = s0[1], b0w = s0[ROW[2] + rl], l0 = s0[a0] * s0[a1];
                const float vx1 = s1[0], vy1 = s1[1], b1w = s1[ROW[2] + rl], l1 = two ? s1[a0] * s1[a1] : 0.f;
                acc_re[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(vx0 * l0, b0w, acc_re[q], 0, 0, 0);
                acc_im[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(vy0 * l0, b0w, acc_im[q], 0, 0, 0);
                acc_re[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(vx1 * l1, b1w, acc_re[q], 0, 0, 0);
                acc_im[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(vy1 * l1, b1w, acc_im[q], 0, 0, 0);
            }
        }
        group_sync(64);
    }
    // ---- write the tile.  D[i][j] of block q sits in lane j + 16 (i / 4),
    // register i % 4, block row i being (x0, x1) = (4 (q / NB1) + i / 4,
    // 4 (q % NB1) + i % 4).
    const bool to_partial = it.nchunks > 1;
    float2 *dst = to_partial ? a.partials + (int64_t(g) * a.n_slots + it.slot + it.chunk) * a.tile_cells
                             : a.h + int64_t(g) * a.grid_elems;
    const int64_t K1 = a.geo.K[1], K2 = a.geo.K[2];
    if constexpr (NW == 1) {
#pragma unroll
        for (int q = 0; q < NBLK; ++q) {
            const int x0 = 4 * (q / NB1) + kq;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int x1 = 4 * (q % NB1) + r;
                const int64_t idx = to_partial ? int64_t((x0 * T1 + x1) * T2 + rl)
                                               : (int64_t(base[0] + x0) * K1 + base[1] + x1) * K2 + base[2] + rl;
                dst[idx] = make_float2(acc_re[q][r], acc_im[q][r]);
            }
        }
        return;
    }
    // several wavefronts: their tiles are summed in wave order
    __syncthreads();  // every wave is done with its staging area
    float2 *red = reinterpret_cast<float2 *>(blk_lds);  // [4][CELLS], reuses the staging LDS
#pragma unroll
    for (int q = 0; q < NBLK; ++q) {
        const int x0 = 4 * (q / NB1) + kq;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int x1 = 4 * (q % NB1) + r;
            red[wave * CELLS + (x0 * T1 + x1) * T2 + rl] = make_float2(acc_re[q][r], acc_im[q][r]);
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < CELLS; e += 64 * NW) {
        float2 sum = red[e];
#pragma unroll
        for (int w = 1; w < NW; ++w) sum = cadd(sum, red[w * CELLS + e]);
        const int x2 = e % T2, x1 = (e / T2) % T1, x0 = e / (T1 * T2);
        const int64_t idx = to_partial ? int64_t(e) : (int64_t(base[0] + x0) * K1 + base[1] + x1) * K2 + base[2] + x2;
        dst[idx] = sum;
    }
}

template <int NJ, int T0, int T1, bool TAB, int NW>
__global__ __launch_bounds__(64 * NW) void k_grid_blk(GridArgs a) {
    grid_blk_body<NJ, T0, T1, TAB, NW>(a, blockIdx.x, blockIdx.y);
}

template <int NJ, int T0, int T1, bool TAB, int NW>
__global__ __launch_bounds__(64 * NW) void k_grid_blk_multi(const GridArgs *__restrict__ jobs,
                                                           const int4 *__restrict__ blocks) {
    const int4 b = blocks[blockIdx.x];
    grid_blk_body<NJ, T0, T1, TAB, NW>(jobs[b.x], b.y, b.z);
}

// Sums the partial tiles of every split tile; one workgroup per (tile,
// kReduceCellsPerWg cells, grid).  The kReduceLanes threads of a cell each
// sum every kReduceLanes-th partial tile in chunk order, and their sums are
// added in lane order (the order of the first inverse FFT pass that sums
// them itself), so the dependent chain of loads of the most crowded tiles is
// kReduceLanes times shorter.
__device__ __forceinline__ void reduce_partials_body(const ReduceArgs &a, int64_t hot, int cb, int g) {
    __shared__ float2 lane_sum[kReduceLanes][kReduceCellsPerWg];
    const HotTile ht = a.hot[hot];
    const int cl = int(threadIdx.x) % kReduceCellsPerWg;  // cell of the block
    const int ln = int(threadIdx.x) / kReduceCellsPerWg;  // its lane
    const int e = cb * kReduceCellsPerWg + cl;
    float2 acc = make_float2(0.f, 0.f);
    if (e < a.tile_cells) {
        const float2 *p = a.partials + (int64_t(g) * a.n_slots + ht.slot) * a.tile_cells + e;
        constexpr int R = 8;  // partial tiles in flight per round trip
        for (int c0 = ln; c0 < ht.nchunks; c0 += R * kReduceLanes) {
            float2 t[R];
#pragma unroll
            for (int j = 0; j < R; ++j)
                if (c0 + j * kReduceLanes < ht.nchunks) t[j] = p[int64_t(c0 + j * kReduceLanes) * a.tile_cells];
#pragma unroll
            for (int j = 0; j < R; ++j)
                if (c0 + j * kReduceLanes < ht.nchunks) acc = cadd(acc, t[j]);
        }
    }
    lane_sum[ln][cl] = acc;
    __syncthreads();
    if (ln != 0 || e >= a.tile_cells) return;
#pragma unroll
    for (int j = 1; j < kReduceLanes; ++j) acc = cadd(acc, lane_sum[j][cl]);
    int tc[kMaxDim];
    {
        int t = ht.tile;
        for (int ax = a.d - 1; ax >= 0; --ax) {
            tc[ax] = t % a.nt[ax];
            t /= a.nt[ax];
        }
    }
    int rem = e;
    int l[kMaxDim];
    for (int ax = a.d - 1; ax >= 0; --ax) {
        l[ax] = rem % a.T[ax];
        rem /= a.T[ax];
    }
    int64_t idx = 0;
    for (int ax = 0; ax < a.d; ++ax) idx = idx * a.K[ax] + tc[ax] * a.T[ax] + l[ax];
    a.h[int64_t(g) * a.grid_elems + idx] = acc;
}

__global__ __launch_bounds__(256) void k_reduce_partials(ReduceArgs a) {
    reduce_partials_body(a, blockIdx.x, blockIdx.y, blockIdx.z);
}

__global__ __launch_bounds__(256) void k_reduce_partials_multi(const ReduceArgs *__restrict__ jobs,
                                                             const int4 *__restrict__ blocks) {
    const int4 b = blocks[blockIdx.x];
    reduce_partials_body(jobs[b.x], b.y, b.z, b.w);
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
        window_weights<J>(a.geo, a.geo.coef[ax], a.geo.nq[ax], f, w[ax]);
        window_weights<J>(a.geo, a.geo.dcoef[ax], a.geo.nq_d[ax], f, dw[ax]);
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
// key = (tile of the first tap) * 2^d + crossing code, bit a set when the
// window leaves the tile through its upper face along axis a.
__global__ __launch_bounds__(256) void k_bin_keys(BinArgs a) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= a.M) return;
    int key = 0, code = 0;
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
                if (a.nt[ax] > 1 && int(kw) - tile * a.T[ax] + a.J - 1 >= a.T[ax]) code |= 1 << ax;
            }
        }
        key = key * a.nt[ax] + tile;
    }
    key = (key << a.d) | code;
    if (bad) atomicOr(a.flag, 1);
    a.keys[i] = key;
    atomicAdd(&a.counts[key], 1);
}

__global__ void k_iota(int *v, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) v[i] = int(i);
}

__device__ __forceinline__ void permute_samples_body(const float2 *y, const int *perm, int64_t M, int grids,
                                                     float2 *ys, int64_t bx) {
    const int64_t i = bx * 256 + threadIdx.x;
    if (i >= M) return;
    const int64_t m = perm[i];
    for (int g = 0; g < grids; ++g) ys[int64_t(g) * M + i] = y[int64_t(g) * M + m];
}

__global__ __launch_bounds__(256) void k_permute_samples(const float2 *y, const int *perm, int64_t M, int grids,
                                                         float2 *ys) {
    permute_samples_body(y, perm, M, grids, ys, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_permute_samples_multi(const PermuteJob *__restrict__ jobs,
                                                               const int4 *__restrict__ blocks) {
    const int4 b = blocks[blockIdx.x];
    const PermuteJob &j = jobs[b.x];
    permute_samples_body(j.y, j.perm, j.M, j.grids, j.ys, b.y);
}

__global__ void k_permute_points(const float *om, const int *perm, int64_t M, int d, float *out) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= M) return;
    const int64_t m = perm[i];
    for (int ax = 0; ax < d; ++ax) out[i * d + ax] = om[m * d + ax];
}

// ------------------------------------------------------------ density compensation
// One fixed-point step of the sampling-density weights (Pipe-Menon) with the
// kernel normalised to peak 1: the gridding ran on wc = w * inv_c and
// u = V V^H wc with the unnormalised kernel (peak c = prod_a I0(beta_a)), so
// |u| * inv_c is the normalised V V^H w;  w[m] <- w[m] / (|u[m]| * inv_c)
// (a zero or non-finite quotient keeps w[m]), and wc is refreshed for the
// next gridding.  The 1/c pre-scaling keeps the grid values near the
// weights' own scale (c^2d overflows float32 for d = 3 and J >= 8).
__global__ __launch_bounds__(256) void k_dc_update(float *w, const float2 *u, float2 *wc, int64_t M, float inv_c) {
    const int64_t m = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (m >= M) return;
    const float a = hypotf(u[m].x, u[m].y) * inv_c;
    float v = w[m];
    if (a > 0.f && isfinite(a)) v = v / a;
    w[m] = v;
    wc[m] = make_float2(v * inv_c, 0.f);
}

__global__ __launch_bounds__(256) void k_real_to_complex(const float *w, float2 *wc, int64_t M, float scale) {
    const int64_t m = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (m < M) wc[m] = make_float2(w[m] * scale, 0.f);
}

// ------------------------------------------------------------ TV split-Bregman pieces
// Image gradient grad_a x = x(.., i_a + 1, ..) - x(.., i_a, ..) with
// wrap-around, its transpose g(.., i_a - 1, ..) - g(.., i_a, ..), and the
// complex soft threshold shrink(z, t) = z / |z| * max(|z| - t, 0).  One
// thread per pixel; every axis of the pixel in registers.
struct TvGeom {
    int d;
    int64_t N[kMaxDim];
    int64_t stride[kMaxDim];
    int64_t n;
};

__device__ __forceinline__ float2 shrinkc(float2 z, float t) {
    const float a = hypotf(z.x, z.y);
    const float sc = a > t ? (a - t) / a : 0.f;
    return make_float2(z.x * sc, z.y * sc);
}

// index of the pixel one step along axis a (delta = +1 or -1), wrapped
__device__ __forceinline__ int64_t tv_step(const TvGeom &g, int64_t i, int a, int delta) {
    const int64_t c = (i / g.stride[a]) % g.N[a];
    int64_t c2 = c + delta;
    if (c2 < 0) c2 += g.N[a];
    if (c2 >= g.N[a]) c2 -= g.N[a];
    return i + (c2 - c) * g.stride[a];
}

__global__ __launch_bounds__(256) void k_tv_shrink(TvGeom g, const float2 *x, float2 *dd, float2 *bb, float t) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= g.n) return;
    const float2 xi = x[i];
    for (int a = 0; a < g.d; ++a) {
        const float2 xn = x[tv_step(g, i, a, +1)];
        const int64_t k = int64_t(a) * g.n + i;
        const float2 z = cadd(csub(xn, xi), bb[k]);
        const float2 dv = shrinkc(z, t);
        dd[k] = dv;
        bb[k] = csub(z, dv);
    }
}

__global__ __launch_bounds__(256) void k_tv_rhs(TvGeom g, float mu, const float2 *ahy, const float2 *df,
                                                const float2 *bf, float lam, const float2 *dd, const float2 *bb,
                                                float2 *rhs) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= g.n) return;
    float2 v = ahy[i];
    if (df) v = cadd(v, csub(df[i], bf[i]));
    float2 acc = cscale(v, mu);
    for (int a = 0; a < g.d; ++a) {
        const int64_t k = int64_t(a) * g.n;
        const int64_t ip = tv_step(g, i, a, -1);
        const float2 here = csub(dd[k + i], bb[k + i]);
        const float2 prev = csub(dd[k + ip], bb[k + ip]);
        acc = cadd(acc, cscale(csub(prev, here), lam));
    }
    rhs[i] = acc;
}

__global__ __launch_bounds__(256) void k_tv_normal(TvGeom g, float mu, const float2 *ahax, float lam, const float2 *x,
                                                   float2 *out) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= g.n) return;
    const float2 xi = x[i];
    float2 lap = make_float2(0.f, 0.f);
    for (int a = 0; a < g.d; ++a) {
        // grad^T grad along a: 2 x(i) - x(i - e_a) - x(i + e_a)
        const float2 xm = x[tv_step(g, i, a, -1)];
        const float2 xp = x[tv_step(g, i, a, +1)];
        lap = cadd(lap, csub(csub(cscale(xi, 2.f), xm), xp));
    }
    out[i] = cadd(cscale(ahax[i], mu), cscale(lap, lam));
}

__global__ __launch_bounds__(256) void k_bregman_shrink(int64_t n, const float2 *r, float2 *dv, float2 *bv, float t) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float2 z = cadd(r[i], bv[i]);
    const float2 dd = shrinkc(z, t);
    dv[i] = dd;
    bv[i] = csub(z, dd);
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
        if (a.items) {
            if (a.n_items == 0) return hipSuccess;
            launch_kernel((k_interp<J, DIM>), dim3(unsigned(a.n_items)), dim3(256), interp_lds(a), s, a);
        } else {
            const int64_t blocks = (a.M + 255) / 256;
            launch_kernel((k_interp_direct<J, DIM>), dim3(unsigned(blocks)), dim3(256), 0, s, a);
        }
        return hipGetLastError();
    }
};

template <int J, int DIM>
struct InterpMultiLaunch {
    static hipError_t go(const InterpArgs *jobs, const int4 *blocks, int64_t n, bool staged, size_t lds,
                         hipStream_t s) {
        if (n == 0) return hipSuccess;
        if (staged)
            launch_kernel((k_interp_multi<J, DIM>), dim3(unsigned(n)), dim3(256), lds, s, jobs, blocks);
        else
            launch_kernel((k_interp_direct_multi<J, DIM>), dim3(unsigned(n)), dim3(256), 0, s, jobs, blocks);
        return hipGetLastError();
    }
};

template <int J, int DIM>
struct GradLaunch {
    static hipError_t go(const GradArgs &a, hipStream_t s) {
        if (a.M == 0) return hipSuccess;
        const int64_t blocks = (a.M + 255) / 256;
        launch_kernel((k_grad<J, DIM>), dim3(unsigned(blocks)), dim3(256), 0, s, a);
        return hipGetLastError();
    }
};

// FFT tile sizes: a tile holds up to THREADS * kEPT elements.  The host takes
// the largest tile that still leaves about target_groups workgroups (small
// transforms spread over the whole chip), then the smallest block that holds
// it.

template <template <int> class L, class A>
hipError_t fft_dispatch(int threads, const A &a, hipStream_t s, int p0, int64_t p1, size_t lds, unsigned blocks) {
    switch (threads) {
        case 64: return L<64>::go(a, s, p0, p1, lds, blocks);
        case 128: return L<128>::go(a, s, p0, p1, lds, blocks);
        case 256: return L<256>::go(a, s, p0, p1, lds, blocks);
        default: return L<512>::go(a, s, p0, p1, lds, blocks);
    }
}

int threads_for(int elems) {
    int t = 64;
    while (t < 512 && t * kEPT < elems) t *= 2;
    return t;
}

template <int T>
struct FirstGo {
    static hipError_t go(const FirstPassArgs &a, hipStream_t s, int lpw, int64_t, size_t lds, unsigned blocks) {
        launch_kernel(k_first_pass<T>, dim3(blocks), dim3(T), lds, s, a, lpw);
        return hipGetLastError();
    }
};

template <int T>
struct StridedGoF {
    static hipError_t go(const StridedPassArgs &a, hipStream_t s, int W, int64_t ntc, size_t lds, unsigned blocks) {
        launch_kernel((k_strided_pass<T, false, false>), dim3(blocks), dim3(T), lds, s, a, W, ntc);
        return hipGetLastError();
    }
};

template <int T>
struct StridedGoI {
    static hipError_t go(const StridedPassArgs &a, hipStream_t s, int W, int64_t ntc, size_t lds, unsigned blocks) {
        if (a.split_of_tile)
            launch_kernel((k_strided_pass<T, true, true>), dim3(blocks), dim3(T), lds, s, a, W, ntc);
        else
            launch_kernel((k_strided_pass<T, true, false>), dim3(blocks), dim3(T), lds, s, a, W, ntc);
        return hipGetLastError();
    }
};

}  // namespace

// ------------------------------------------------------------ launchers
FftLaunch first_pass_launch(const FirstPassArgs &a, int threads) {
    FftLaunch L{64, 0, 0, 1, 0};
    const int64_t total = int64_t(a.B) * a.C * a.rows;
    if (total == 0) return L;
    const int cap = kFftTileElems / a.K;  // lines that fit the largest tile
    int lpw = int(std::min<int64_t>(std::max<int64_t>(1, total / a.target_groups), std::min(cap, kMaxLinesPerWg)));
    lpw = std::max(1, lpw);
    if (threads > 0)  // a given workgroup size: as many lines as its tile holds
        lpw = int(std::max<int64_t>(1, std::min<int64_t>({total, kMaxLinesPerWg, threads * kEPT / a.K})));
    L.threads = threads > 0 ? threads : threads_for(lpw * a.K);
    L.blocks = (total + lpw - 1) / lpw;
    L.lds = size_t(lpw + 1) * a.K * sizeof(float2);
    L.p0 = lpw;
    return L;
}

hipError_t launch_first_pass(const FirstPassArgs &a, hipStream_t s) {
    const FftLaunch L = first_pass_launch(a);
    if (L.blocks == 0) return hipSuccess;
    return fft_dispatch<FirstGo>(L.threads, a, s, L.p0, 0, L.lds, unsigned(L.blocks));
}

FftLaunch strided_pass_launch(const StridedPassArgs &a, int threads) {
    FftLaunch L{64, 0, 0, 1, 0};
    const int64_t columns = a.grids * a.outer * a.inner;
    if (columns == 0) return L;
    const int cap = std::max(1, threads > 0 ? threads * kEPT / a.K : kFftTileElems / a.K);
    // columns per tile: at least 4 adjacent (32-byte rows), fewer only for narrow
    // arrays; with a given workgroup size, as many as its tile holds
    int64_t W = threads > 0 ? cap : std::max<int64_t>(4, columns / a.target_groups);
    W = std::min<int64_t>(W, cap);
    W = std::min<int64_t>(W, a.inner);
    W = std::max<int64_t>(W, 1);
    const int64_t ntc = (a.inner + W - 1) / W;
    L.blocks = ntc * a.outer * a.grids;
    L.threads = threads > 0 ? threads : threads_for(int(W) * a.K);
    L.lds = size_t(W + 1) * a.K * sizeof(float2);
    L.p0 = int(W);
    L.p1 = ntc;
    return L;
}

hipError_t launch_strided_pass(const StridedPassArgs &a, hipStream_t s) {
    const FftLaunch L = strided_pass_launch(a);
    if (L.blocks == 0) return hipSuccess;
    if (a.inverse) return fft_dispatch<StridedGoI>(L.threads, a, s, L.p0, L.p1, L.lds, unsigned(L.blocks));
    return fft_dispatch<StridedGoF>(L.threads, a, s, L.p0, L.p1, L.lds, unsigned(L.blocks));
}

namespace {
template <int T>
struct LastGo {
    static hipError_t go(const LastPassArgs &a, hipStream_t s, int rpw, int64_t cpr, size_t lds, unsigned blocks) {
        launch_kernel(k_last_pass<T>, dim3(blocks), dim3(T), lds, s, a, rpw, int(cpr));
        return hipGetLastError();
    }
};
}  // namespace

FftLaunch last_pass_launch(const LastPassArgs &a, int threads) {
    FftLaunch L{64, 0, 0, 1, 1};
    const int64_t total_rows = int64_t(a.B) * a.rows;
    if (total_rows == 0) return L;
    const int tile = threads > 0 ? threads * kEPT : kFftTileElems;
    int rows_per_wg, coils_per_round;
    if (a.C * a.K <= tile) {
        coils_per_round = a.C;
        const int cap = std::min(tile / (a.C * a.K), kMaxLinesPerWg);
        rows_per_wg = threads > 0 ? cap
                                  : int(std::min<int64_t>(std::max<int64_t>(1, total_rows / a.target_groups), cap));
    } else {
        rows_per_wg = 1;
        coils_per_round = std::max(1, tile / a.K);
    }
    if (int64_t(rows_per_wg) > a.rows) rows_per_wg = int(a.rows);
    rows_per_wg = std::max(1, rows_per_wg);
    L.threads = threads > 0 ? threads : threads_for(rows_per_wg * coils_per_round * a.K);
    const int64_t nrt = (a.rows + rows_per_wg - 1) / rows_per_wg;
    L.blocks = nrt * a.B;
    const bool one_round = coils_per_round >= a.C;
    L.lds = (size_t(a.K) + size_t(rows_per_wg) * coils_per_round * a.K +
             (one_round ? 0 : size_t(rows_per_wg) * a.N)) * sizeof(float2);
    L.p0 = rows_per_wg;
    L.p1 = coils_per_round;
    return L;
}

hipError_t launch_last_pass(const LastPassArgs &a, hipStream_t s) {
    const FftLaunch L = last_pass_launch(a);
    if (L.blocks == 0) return hipSuccess;
    return fft_dispatch<LastGo>(L.threads, a, s, L.p0, L.p1, L.lds, unsigned(L.blocks));
}

// ---- many problems per launch
namespace {
template <int T>
struct FirstMulti {
    static void go(const FirstJob *j, const int4 *b, int64_t n, size_t lds, hipStream_t s) {
        launch_kernel(k_first_pass_multi<T>, dim3(unsigned(n)), dim3(T), lds, s, j, b);
    }
};
template <int T>
struct LastMulti {
    static void go(const LastJob *j, const int4 *b, int64_t n, size_t lds, hipStream_t s) {
        launch_kernel(k_last_pass_multi<T>, dim3(unsigned(n)), dim3(T), lds, s, j, b);
    }
};
template <bool INV, bool SPLIT>
struct StridedMultiF {
    template <int T>
    struct K {
        static void go(const StridedJob *j, const int4 *b, int64_t n, size_t lds, hipStream_t s) {
            launch_kernel((k_strided_pass_multi<T, INV, SPLIT>), dim3(unsigned(n)), dim3(T), lds, s, j, b);
        }
    };
};

template <template <int> class L, class Job>
hipError_t threads_go(int threads, const Job *j, const int4 *b, int64_t n, size_t lds, hipStream_t s) {
    if (n == 0) return hipSuccess;
    switch (threads) {
        case 64: L<64>::go(j, b, n, lds, s); break;
        case 128: L<128>::go(j, b, n, lds, s); break;
        case 256: L<256>::go(j, b, n, lds, s); break;
        case 512: L<512>::go(j, b, n, lds, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
}  // namespace

hipError_t launch_first_pass_multi(const FirstJob *jobs, const int4 *blocks, int64_t nblocks, int threads,
                                   size_t lds, hipStream_t s) {
    return threads_go<FirstMulti>(threads, jobs, blocks, nblocks, lds, s);
}

hipError_t launch_strided_pass_multi(const StridedJob *jobs, const int4 *blocks, int64_t nblocks, int threads,
                                     bool inverse, bool split, size_t lds, hipStream_t s) {
    if (!inverse) return threads_go<StridedMultiF<false, false>::K>(threads, jobs, blocks, nblocks, lds, s);
    if (split) return threads_go<StridedMultiF<true, true>::K>(threads, jobs, blocks, nblocks, lds, s);
    return threads_go<StridedMultiF<true, false>::K>(threads, jobs, blocks, nblocks, lds, s);
}

hipError_t launch_last_pass_multi(const LastJob *jobs, const int4 *blocks, int64_t nblocks, int threads, size_t lds,
                                  hipStream_t s) {
    return threads_go<LastMulti>(threads, jobs, blocks, nblocks, lds, s);
}

size_t interp_lds(const InterpArgs &a) {
    if (!a.items) return 0;
    return size_t(interp_region_elems(a.geo.d, a.T, a.geo.J, a.merge)) * sizeof(float2);
}

hipError_t launch_interp(const InterpArgs &a, hipStream_t s) {
    return dispatch_jd<InterpLaunch>(a.geo.J, a.geo.d, a, s);
}

hipError_t launch_interp_multi(const InterpArgs *jobs, const int4 *blocks, int64_t nblocks, int J, int d,
                               bool staged, size_t lds, hipStream_t s) {
    return dispatch_jd<InterpMultiLaunch>(J, d, jobs, blocks, nblocks, staged, lds, s);
}

template <int DIM, int LS>
hipError_t launch_grid_t(const GridArgs &a, hipStream_t s) {
    const size_t lds = grid_lds(a);
    const dim3 grid(unsigned(a.n_items), unsigned(a.grids));
    if (a.geo.jp == 8)
        launch_kernel((k_grid<DIM, LS, 8>), grid, dim3(kGridThreads), lds, s, a);
    else if (a.geo.jp == 16)
        launch_kernel((k_grid<DIM, LS, 16>), grid, dim3(kGridThreads), lds, s, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <int DIM>
hipError_t launch_grid_d(const GridArgs &a, hipStream_t s) {
    switch (a.seg_len) {
        case 4: return launch_grid_t<DIM, 4>(a, s);
        case 8: return launch_grid_t<DIM, 8>(a, s);
        case 16: return launch_grid_t<DIM, 16>(a, s);
        default: return hipErrorInvalidValue;
    }
}

// The window-table form of the sample kernels exists for windows of up to 8
// taps (table_taps 6 or 8); wider windows evaluate the kernel on the fly even
// when the plan holds a table.
inline bool use_table(const SampleGeom &g) { return g.wtab != nullptr && table_taps(g.J) <= 8; }

template <int DIM, int NJ, int MB, bool TAB>
hipError_t launch_grid_mfma_t(const GridArgs &a, hipStream_t s) {
    const size_t lds = grid_lds(a);
    const int gp = a.grids_per_wg;
    const dim3 grid(unsigned(a.n_items), unsigned((a.grids + gp - 1) / gp));
    switch (gp) {
        case 1: launch_kernel((k_grid_mfma<DIM, NJ, MB, 1, TAB>), grid, dim3(256), lds, s, a); break;
        case 2: launch_kernel((k_grid_mfma<DIM, NJ, MB, 2, TAB>), grid, dim3(256), lds, s, a); break;
        case 4:
            if constexpr (MB <= 2) {
                launch_kernel((k_grid_mfma<DIM, NJ, MB, 4, TAB>), grid, dim3(256), lds, s, a);
                break;
            }
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int DIM, int NJ, int MB>
hipError_t launch_grid_mfma_m(const GridArgs &a, hipStream_t s) {
    if constexpr (NJ <= 8)
        if (use_table(a.geo)) return launch_grid_mfma_t<DIM, NJ, MB, true>(a, s);
    return launch_grid_mfma_t<DIM, NJ, MB, false>(a, s);
}

template <int DIM, int NJ>
hipError_t launch_grid_mfma_j(const GridArgs &a, hipStream_t s) {
    switch (a.tile_cells) {
        case 256: return launch_grid_mfma_m<DIM, NJ, 1>(a, s);
        case 512: return launch_grid_mfma_m<DIM, NJ, 2>(a, s);
        case 1024: return launch_grid_mfma_m<DIM, NJ, 4>(a, s);
        default: return hipErrorInvalidValue;
    }
}

template <int DIM>
hipError_t launch_grid_mfma_d(const GridArgs &a, hipStream_t s) {
    if (a.T[DIM - 1] != 16) return hipErrorInvalidValue;
    // taps evaluated per sample: J rounded up to 6, 8 or 16
    if (a.geo.J <= 6) return launch_grid_mfma_j<DIM, 6>(a, s);
    if (a.geo.J <= 8) return launch_grid_mfma_j<DIM, 8>(a, s);
    return launch_grid_mfma_j<DIM, 16>(a, s);
}

template <int NJ, int T0, int T1, bool TAB, int NW, bool MULTI>
void launch_grid_blk_i(const GridArgs &a, const GridArgs *jobs, const int4 *blocks, int64_t nblocks, size_t lds,
                       hipStream_t s) {
    if (MULTI)
        launch_kernel((k_grid_blk_multi<NJ, T0, T1, TAB, NW>), dim3(unsigned(nblocks)), dim3(64 * NW), lds, s, jobs,
                      blocks);
    else
        launch_kernel((k_grid_blk<NJ, T0, T1, TAB, NW>), dim3(unsigned(a.n_items), unsigned(a.grids)), dim3(64 * NW),
                      lds, s, a);
}

template <int NJ, int T0, int T1, bool MULTI>
hipError_t launch_grid_blk_t(const GridArgs &a, const GridArgs *jobs, const int4 *blocks, int64_t nblocks,
                             size_t lds, hipStream_t s) {
    const bool tab = NJ <= 8 && use_table(a.geo);
    if (a.grid_waves == 1) {
        if (tab)
            launch_grid_blk_i<NJ, T0, T1, true, 1, MULTI>(a, jobs, blocks, nblocks, lds, s);
        else
            launch_grid_blk_i<NJ, T0, T1, false, 1, MULTI>(a, jobs, blocks, nblocks, lds, s);
    } else {
        if (tab)
            launch_grid_blk_i<NJ, T0, T1, true, 4, MULTI>(a, jobs, blocks, nblocks, lds, s);
        else
            launch_grid_blk_i<NJ, T0, T1, false, 4, MULTI>(a, jobs, blocks, nblocks, lds, s);
    }
    return hipGetLastError();
}

template <int NJ, bool MULTI>
hipError_t launch_grid_blk_j(const GridArgs &a, const GridArgs *jobs, const int4 *blocks, int64_t nblocks,
                             size_t lds, hipStream_t s) {
    if (a.T[0] == 8 && a.T[1] == 8) return launch_grid_blk_t<NJ, 8, 8, MULTI>(a, jobs, blocks, nblocks, lds, s);
    if (a.T[0] == 8 && a.T[1] == 16) return launch_grid_blk_t<NJ, 8, 16, MULTI>(a, jobs, blocks, nblocks, lds, s);
    if (a.T[0] == 16 && a.T[1] == 8) return launch_grid_blk_t<NJ, 16, 8, MULTI>(a, jobs, blocks, nblocks, lds, s);
    return hipErrorInvalidValue;
}

template <bool MULTI>
hipError_t launch_grid_blk(const GridArgs &a, const GridArgs *jobs, const int4 *blocks, int64_t nblocks,
                           size_t lds, hipStream_t s) {
    if (a.geo.d != 3 || a.T[2] != 16) return hipErrorInvalidValue;
    if (a.geo.J <= 6) return launch_grid_blk_j<6, MULTI>(a, jobs, blocks, nblocks, lds, s);
    if (a.geo.J <= 8) return launch_grid_blk_j<8, MULTI>(a, jobs, blocks, nblocks, lds, s);
    return launch_grid_blk_j<16, MULTI>(a, jobs, blocks, nblocks, lds, s);
}

hipError_t launch_grid(const GridArgs &a, hipStream_t s) {
    if (a.n_items == 0) return hipSuccess;
    if (a.blk) return launch_grid_blk<false>(a, nullptr, nullptr, 0, grid_lds(a), s);
    if (a.mfma) {
        switch (a.geo.d) {
            case 2: return launch_grid_mfma_d<2>(a, s);
            case 3: return launch_grid_mfma_d<3>(a, s);
            default: return hipErrorInvalidValue;
        }
    }
    switch (a.geo.d) {
        case 1: return launch_grid_d<1>(a, s);
        case 2: return launch_grid_d<2>(a, s);
        case 3: return launch_grid_d<3>(a, s);
        default: return hipErrorInvalidValue;
    }
}

// Kernel instance of a gridding launch: matrix cores (d, taps rounded to
// 6/8/16, row blocks) or vector ALUs (d, segment length, coefficient row
// width), as launch_grid picks it; -1 if there is none.
int grid_variant(const GridArgs &a) {
    if (a.blk) {
        if (a.geo.d != 3 || a.T[2] != 16 || (a.T[0] != 8 && a.T[0] != 16) || (a.T[1] != 8 && a.T[1] != 16) ||
            a.T[0] * a.T[1] > 128)
            return -1;
        const int nj = a.geo.J <= 6 ? 0 : a.geo.J <= 8 ? 1 : 2;
        if (a.grid_waves != 1 && a.grid_waves != 4) return -1;
        return 3000 + 100 * a.grid_waves + 10 * nj + (a.T[0] == 16 ? 2 : 0) + (a.T[1] == 16 ? 1 : 0);
    }
    if (a.mfma) {
        if (a.geo.d < 2 || a.T[a.geo.d - 1] != 16) return -1;
        const int nj = a.geo.J <= 6 ? 6 : a.geo.J <= 8 ? 8 : 16;
        const int mb = a.tile_cells / 256;
        if (a.tile_cells % 256 || (mb != 1 && mb != 2 && mb != 4)) return -1;
        const int gp = a.grids_per_wg;
        if ((gp != 1 && gp != 2 && gp != 4) || gp * mb > 8) return -1;
        return 10000 * gp + 1000 + 100 * a.geo.d + 10 * (nj == 6 ? 0 : nj == 8 ? 1 : 2) + mb;
    }
    if (a.seg_len != 4 && a.seg_len != 8 && a.seg_len != 16) return -1;
    if (a.geo.jp != 8 && a.geo.jp != 16) return -1;
    return 2000 + 100 * a.geo.d + a.seg_len * 2 + (a.geo.jp == 16 ? 1 : 0);
}

size_t grid_lds(const GridArgs &a) {
    if (a.blk) {
        const size_t staged = size_t(64) * a.grid_waves * (3 + a.T[0] + a.T[1] + a.T[2] + 1) * sizeof(float);
        return a.grid_waves == 1 ? staged : std::max(staged, size_t(a.grid_waves) * a.tile_cells * sizeof(float2));
    }
    if (a.mfma) {
        int tsum = 0;
        for (int ax = 0; ax < a.geo.d; ++ax) tsum += a.T[ax];
        const size_t rs = size_t((2 * a.grids_per_wg + tsum) | 1);
        return std::max(size_t(4) * 64 * rs, size_t(4) * 2 * a.tile_cells) * sizeof(float);
    }
    return size_t(kGridThreads / a.group_lanes) * a.stage_floats * sizeof(float);
}

namespace {
template <int DIM, int NJ, int MB, bool TAB>
hipError_t grid_mfma_multi_t(const GridArgs *jobs, const int4 *blocks, int64_t n, int gp, size_t lds, hipStream_t s) {
    const dim3 grid = dim3(unsigned(n));
    switch (gp) {
        case 1: launch_kernel((k_grid_mfma_multi<DIM, NJ, MB, 1, TAB>), grid, dim3(256), lds, s, jobs, blocks); break;
        case 2: launch_kernel((k_grid_mfma_multi<DIM, NJ, MB, 2, TAB>), grid, dim3(256), lds, s, jobs, blocks); break;
        case 4:
            if constexpr (MB <= 2) {
                launch_kernel((k_grid_mfma_multi<DIM, NJ, MB, 4, TAB>), grid, dim3(256), lds, s, jobs, blocks);
                break;
            }
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int DIM, int NJ, int MB>
hipError_t grid_mfma_multi_m(const GridArgs *jobs, const int4 *blocks, int64_t n, int gp, bool tab, size_t lds,
                             hipStream_t s) {
    if constexpr (NJ <= 8)
        if (tab) return grid_mfma_multi_t<DIM, NJ, MB, true>(jobs, blocks, n, gp, lds, s);
    return grid_mfma_multi_t<DIM, NJ, MB, false>(jobs, blocks, n, gp, lds, s);
}

template <int DIM, int NJ>
hipError_t grid_mfma_multi_j(const GridArgs *jobs, const int4 *blocks, int64_t n, int mb, int gp, bool tab,
                             size_t lds, hipStream_t s) {
    switch (mb) {
        case 1: return grid_mfma_multi_m<DIM, NJ, 1>(jobs, blocks, n, gp, tab, lds, s);
        case 2: return grid_mfma_multi_m<DIM, NJ, 2>(jobs, blocks, n, gp, tab, lds, s);
        case 4: return grid_mfma_multi_m<DIM, NJ, 4>(jobs, blocks, n, gp, tab, lds, s);
        default: return hipErrorInvalidValue;
    }
}

template <int DIM>
hipError_t grid_mfma_multi_d(const GridArgs *jobs, const int4 *blocks, int64_t n, const GridArgs &p, size_t lds,
                             hipStream_t s) {
    const int mb = p.tile_cells / 256;
    const bool tab = use_table(p.geo);
    if (p.geo.J <= 6) return grid_mfma_multi_j<DIM, 6>(jobs, blocks, n, mb, p.grids_per_wg, tab, lds, s);
    if (p.geo.J <= 8) return grid_mfma_multi_j<DIM, 8>(jobs, blocks, n, mb, p.grids_per_wg, tab, lds, s);
    return grid_mfma_multi_j<DIM, 16>(jobs, blocks, n, mb, p.grids_per_wg, tab, lds, s);
}

template <int DIM, int LS>
hipError_t grid_valu_multi_t(const GridArgs *jobs, const int4 *blocks, int64_t n, int jp, size_t lds, hipStream_t s) {
    if (jp == 8)
        launch_kernel((k_grid_multi<DIM, LS, 8>), dim3(unsigned(n)), dim3(kGridThreads), lds, s, jobs, blocks);
    else if (jp == 16)
        launch_kernel((k_grid_multi<DIM, LS, 16>), dim3(unsigned(n)), dim3(kGridThreads), lds, s, jobs, blocks);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <int DIM>
hipError_t grid_valu_multi_d(const GridArgs *jobs, const int4 *blocks, int64_t n, const GridArgs &p, size_t lds,
                             hipStream_t s) {
    switch (p.seg_len) {
        case 4: return grid_valu_multi_t<DIM, 4>(jobs, blocks, n, p.geo.jp, lds, s);
        case 8: return grid_valu_multi_t<DIM, 8>(jobs, blocks, n, p.geo.jp, lds, s);
        case 16: return grid_valu_multi_t<DIM, 16>(jobs, blocks, n, p.geo.jp, lds, s);
        default: return hipErrorInvalidValue;
    }
}
}  // namespace

hipError_t launch_grid_multi(const GridArgs *jobs, const int4 *blocks, int64_t nblocks, const GridArgs &proto,
                             size_t lds, hipStream_t s) {
    if (nblocks == 0) return hipSuccess;
    if (grid_variant(proto) < 0) return hipErrorInvalidValue;
    if (proto.blk) return launch_grid_blk<true>(proto, jobs, blocks, nblocks, lds, s);
    if (proto.mfma) {
        switch (proto.geo.d) {
            case 2: return grid_mfma_multi_d<2>(jobs, blocks, nblocks, proto, lds, s);
            case 3: return grid_mfma_multi_d<3>(jobs, blocks, nblocks, proto, lds, s);
            default: return hipErrorInvalidValue;
        }
    }
    switch (proto.geo.d) {
        case 1: return grid_valu_multi_d<1>(jobs, blocks, nblocks, proto, lds, s);
        case 2: return grid_valu_multi_d<2>(jobs, blocks, nblocks, proto, lds, s);
        case 3: return grid_valu_multi_d<3>(jobs, blocks, nblocks, proto, lds, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_reduce_partials_multi(const ReduceArgs *jobs, const int4 *blocks, int64_t nblocks, hipStream_t s) {
    if (nblocks == 0) return hipSuccess;
    launch_kernel(k_reduce_partials_multi, dim3(unsigned(nblocks)), dim3(256), 0, s, jobs, blocks);
    return hipGetLastError();
}

hipError_t launch_permute_samples_multi(const PermuteJob *jobs, const int4 *blocks, int64_t nblocks, hipStream_t s) {
    if (nblocks == 0) return hipSuccess;
    launch_kernel(k_permute_samples_multi, dim3(unsigned(nblocks)), dim3(256), 0, s, jobs, blocks);
    return hipGetLastError();
}

hipError_t launch_reduce_partials(const ReduceArgs &a, hipStream_t s) {
    if (a.n_hot == 0) return hipSuccess;
    launch_kernel(k_reduce_partials,
                  dim3(unsigned(a.n_hot), unsigned((a.tile_cells + kReduceCellsPerWg - 1) / kReduceCellsPerWg),
                       unsigned(a.grids)),
                  dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_grad(const GradArgs &a, hipStream_t s) {
    return dispatch_jd<GradLaunch>(a.geo.J, a.geo.d, a, s);
}

hipError_t launch_bin_keys(const BinArgs &a, hipStream_t s) {
    if (a.M == 0) return hipSuccess;
    const int64_t blocks = (a.M + 255) / 256;
    launch_kernel(k_bin_keys, dim3(unsigned(blocks)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_dc_update(float *w, const float2 *u, float2 *wc, int64_t M, float inv_c, hipStream_t s) {
    if (M == 0) return hipSuccess;
    launch_kernel(k_dc_update, dim3(unsigned((M + 255) / 256)), dim3(256), 0, s, w, u, wc, M, inv_c);
    return hipGetLastError();
}

template <int NJ>
hipError_t launch_weight_table_j(const SampleGeom &g, const float *om_sorted, int64_t M, float *out, hipStream_t s) {
    const dim3 grid(unsigned((M + 255) / 256));
    switch (g.d) {
        case 1: launch_kernel((k_weight_table<NJ, 1>), grid, dim3(256), 0, s, g, om_sorted, M, out); break;
        case 2: launch_kernel((k_weight_table<NJ, 2>), grid, dim3(256), 0, s, g, om_sorted, M, out); break;
        case 3: launch_kernel((k_weight_table<NJ, 3>), grid, dim3(256), 0, s, g, om_sorted, M, out); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_weight_table(const SampleGeom &g, const float *om_sorted, int64_t M, float *out, hipStream_t s) {
    if (M == 0) return hipSuccess;
    if (g.wtab_stride != table_stride(g.d, g.J)) return hipErrorInvalidValue;
    switch (table_taps(g.J)) {
        case 6: return launch_weight_table_j<6>(g, om_sorted, M, out, s);
        case 8: return launch_weight_table_j<8>(g, om_sorted, M, out, s);
        default: return launch_weight_table_j<16>(g, om_sorted, M, out, s);
    }
}

hipError_t launch_real_to_complex(const float *w, float2 *wc, int64_t M, float scale, hipStream_t s) {
    if (M == 0) return hipSuccess;
    launch_kernel(k_real_to_complex, dim3(unsigned((M + 255) / 256)), dim3(256), 0, s, w, wc, M, scale);
    return hipGetLastError();
}

// ---- fixed device scratch of the allocation-free density compensation
// The two complex sample buffers of the iteration (the weights handed to the
// gridding, and V V^H of them), kDcScratchMaxM samples each, as one static
// device array: every GPU the library runs on holds its own copy from the
// first use until the process ends.  Host code never passes the array's name
// to a kernel (on the host it is only a stand-in for the symbol); it uses the
// device address that hipGetSymbolAddress returns, looked up once per device
// with that device current.
static __device__ __align__(256) float2 scratch[2 * kDcScratchMaxM];

hipError_t dc_scratch(float2 **wc, float2 **u) {
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *wc = static_cast<float2 *>(addr[dev]);
    *u = *wc + kDcScratchMaxM;
    return hipSuccess;
}

static TvGeom tv_geom(int d, const int64_t *N) {
    TvGeom g{};
    g.d = d;
    int64_t st = 1;
    for (int a = d - 1; a >= 0; --a) {
        g.N[a] = N[a];
        g.stride[a] = st;
        st *= N[a];
    }
    g.n = st;
    return g;
}

hipError_t launch_tv_shrink(int d, const int64_t *N, const float2 *x, float2 *dd, float2 *bb, float t, hipStream_t s) {
    const TvGeom g = tv_geom(d, N);
    if (g.n == 0) return hipSuccess;
    launch_kernel(k_tv_shrink, dim3(unsigned((g.n + 255) / 256)), dim3(256), 0, s, g, x, dd, bb, t);
    return hipGetLastError();
}

hipError_t launch_tv_rhs(int d, const int64_t *N, float mu, const float2 *ahy, const float2 *df, const float2 *bf,
                         float lam, const float2 *dd, const float2 *bb, float2 *rhs, hipStream_t s) {
    const TvGeom g = tv_geom(d, N);
    if (g.n == 0) return hipSuccess;
    launch_kernel(k_tv_rhs, dim3(unsigned((g.n + 255) / 256)), dim3(256), 0, s, g, mu, ahy, df, bf, lam, dd, bb,
                       rhs);
    return hipGetLastError();
}

hipError_t launch_tv_normal(int d, const int64_t *N, float mu, const float2 *ahax, float lam, const float2 *x,
                            float2 *out, hipStream_t s) {
    const TvGeom g = tv_geom(d, N);
    if (g.n == 0) return hipSuccess;
    launch_kernel(k_tv_normal, dim3(unsigned((g.n + 255) / 256)), dim3(256), 0, s, g, mu, ahax, lam, x, out);
    return hipGetLastError();
}

hipError_t launch_bregman_shrink(int64_t n, const float2 *r, float2 *dv, float2 *bv, float t, hipStream_t s) {
    if (n == 0) return hipSuccess;
    launch_kernel(k_bregman_shrink, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, n, r, dv, bv, t);
    return hipGetLastError();
}

hipError_t launch_iota(int *v, int64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    launch_kernel(k_iota, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, v, n);
    return hipGetLastError();
}

hipError_t launch_permute_samples(const float2 *y, const int *perm, int64_t M, int grids, float2 *ys,
                                  hipStream_t s) {
    if (M == 0 || grids == 0) return hipSuccess;
    launch_kernel(k_permute_samples, dim3(unsigned((M + 255) / 256)), dim3(256), 0, s, y, perm, M, grids, ys);
    return hipGetLastError();
}

hipError_t launch_permute_points(const float *om, const int *perm, int64_t M, int d, float *om_sorted,
                                 hipStream_t s) {
    if (M == 0) return hipSuccess;
    launch_kernel(k_permute_points, dim3(unsigned((M + 255) / 256)), dim3(256), 0, s, om, perm, M, d,
                       om_sorted);
    return hipGetLastError();
}

hipError_t sort_pairs_temp_bytes(int64_t n, int key_bits, size_t *bytes) {
    *bytes = 0;
    if (n == 0) return hipSuccess;
    return hipcub::DeviceRadixSort::SortPairs(nullptr, *bytes, static_cast<const int *>(nullptr),
                                              static_cast<int *>(nullptr), static_cast<const int *>(nullptr),
                                              static_cast<int *>(nullptr), int(n), 0, key_bits);
}

hipError_t sort_pairs(const int *keys_in, int *keys_out, const int *vals_in, int *vals_out, int64_t n,
                      int key_bits, void *temp, size_t temp_bytes, hipStream_t s) {
    if (n == 0) return hipSuccess;
    size_t need = 0;
    hipError_t e = sort_pairs_temp_bytes(n, key_bits, &need);
    if (e != hipSuccess) return e;
    if (need > temp_bytes || !temp) return hipErrorInvalidValue;
    return hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, keys_in, keys_out, vals_in, vals_out, int(n), 0,
                                              key_bits, s);
}

}  // namespace nufft
