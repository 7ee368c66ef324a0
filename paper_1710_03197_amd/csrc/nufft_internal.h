// Internal declarations shared by the runtime (plan, C ABI) and the HIP
// kernels of libnufft_mi355x.  Not installed; the public interface is
// include/nufft_mi355x.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace nufft {

constexpr int kMaxDim = 3;
constexpr int kMaxJ = 16;
constexpr int kMaxPasses = 16;     // radix passes per axis (K <= 4096)
constexpr int kMaxNeighbors = 27;  // bins whose windows can reach one tile
constexpr int kFftTileElems = 4096;  // complex elements of the largest FFT workgroup tile (512 threads x 8)
constexpr int kMaxLinesPerWg = 64;   // lines (contiguous-axis passes) per FFT workgroup
constexpr int kMaxPolyDeg = 23;
constexpr int kInterpSamplesPerThread = 2;  // gather work item = 512 samples
constexpr int kLdsBudget = 64 * 1024;      // bytes of LDS a gather or gridding tile may use
constexpr int kInterpLdsBudget = 64 * 1024;  // bytes of LDS a gather item covering several tiles may use

// Radix schedule of one FFT axis (Stockham, product of r[] == K).
// Per pass p (Ns = r[0] ... r[p-1] the length of the sub-transforms done so
// far): span = K / (Ns r[p]), and the division magics ceil(2^32 / D) of
// D = Ns and D = K / r[p] (0 for D = 1) the passes use instead of integer
// divisions.
struct RadixPlan {
    int n;
    int r[kMaxPasses];
    int span[kMaxPasses];
    unsigned m_ns[kMaxPasses];
    unsigned m_nbl[kMaxPasses];
};

// Kaiser-Bessel kernel of one axis (unnormalised, phi(0) = I0(beta)) as per-tap
// polynomials in z = 2f - 1, f in [0, 1) the offset of the first tap:
// w_j(z) = sum_k c[j][k] z^k (k <= deg), and the same for d phi / d t.
struct AxisKernel {
    double beta;
    int deg;       // polynomial degree of w_j
    int deg_d;     // polynomial degree of the derivative fit
    std::vector<float> coef;   // [J][deg+1]
    std::vector<float> dcoef;  // [J][deg_d+1]
};

// ---- host-side mathematics (kb_host.cpp)
double kb_beta(int J, double sigma);
double kb_i0(double z);
double kb_phi(double t, int J, double beta);
double kb_dphi(double t, int J, double beta);
double kb_ft(double xi, int J, double beta);       // continuous Fourier transform
// Fit the kernel and its derivative per tap; returns false if no degree
// up to kMaxPolyDeg reaches the target accuracy.
bool kb_fit(int J, double beta, AxisKernel *out);
// Evaluate the fitted polynomials exactly as the GPU does (float32 Horner).
void kb_eval_fit(const AxisKernel &k, int J, float f, float *w, float *dw);
// Device layout of per-tap coefficients [J][deg+1]: rows r = 0..nq-1 of jp
// floats, row r holding the degree nq-1-r coefficient of every tap (zero for
// degrees above deg and taps j >= J), nq = deg+1 rounded up to a multiple of
// 2.  Horner from v = 0 over the rows gives the same float32 result as over
// the unpadded coefficients (the leading zero row keeps v at 0).
std::vector<float> coef_rows(const std::vector<float> &coef, int J, int deg, int jp, int *nq);
// Row width for J taps: 8 for J <= 8, else 16.
inline int coef_row_width(int J) { return J <= 8 ? 8 : 16; }
// Min-max interpolator of one axis (real factor c' of the coefficients per
// tap; see kb_host.cpp), its scaling table 1 / Phi((i - N/2 + 1/2)/K), and
// the grid phase e^{-i pi k / K}, k in [0, K).
bool minmax_fit(int N, int K, int J, double beta, AxisKernel *out);
std::vector<float> minmax_scaling(int N, int K, int J, double beta);
std::vector<float2> half_phase(int K);
// Scaling table s(i) = 1 / Phi((i - N/2)/K), i in [0, N) (float32).
std::vector<float> kb_scaling(int N, int K, int J, double beta);
// Twiddles e^{-2 pi i e / K}, e in [0, K), computed in float64.
std::vector<float2> twiddles(int K);
// Stockham radix schedule; false if K has a prime factor above 5.  schedule
// 0: radices 8, 4, 2, 3, 5 taken greedily in that order (the default); 1: 4,
// 8, 2, 3, 5; 2: 3, 5, 8, 4, 2; 3: schedule 0 with its passes reversed.
bool radix_plan(int K, RadixPlan *rp, int schedule = 0);

// ---- device kernel launchers (kernels.hip).  All asynchronous on `s`.

// Forward pass along the contiguous last axis: pad N -> K, scaling, coil
// multiply; x [B][rows][N] -> out [B*C][rows][K].
struct FirstPassArgs {
    const float2 *x;
    float2 *out;
    const float2 *tw;
    RadixPlan rp;
    const float2 *coils;  // [C][rows*N] or nullptr
    int C;                // grids per image (1 without coils)
    int B;                // images
    int K, N;             // last axis
    int64_t rows;         // prod_{a<d-1} N_a
    int d;
    int Nax[kMaxDim];
    const float *scale[kMaxDim];
    const float2 *mult;  // d = 1 Toeplitz product: the output line times mult[q] (nullptr: none)
    int target_groups;  // workgroups the launch aims for
    const float2 *phase;  // min-max grid phase e^{-i pi k / K} of this pass's axis (nullptr: none)
};
hipError_t launch_first_pass(const FirstPassArgs &a, hipStream_t s);

// Pass along a strided axis: [G][outer][Lin][inner] -> [G][outer][Lout][inner],
// Lin < K means zero padded input rows, Lout < K a cropped output.
struct HotTile;
struct StridedPassArgs {
    const float2 *in;
    float2 *out;
    const float2 *tw;
    RadixPlan rp;
    int K, Lin, Lout;
    int64_t outer, inner;
    int64_t grids;
    bool inverse;
    const float2 *mult;  // inverse pass: the input times mult (same layout, shared by all grids)
    int target_groups;
    // First inverse pass of the adjoint only (split_of_tile != nullptr): cells of
    // split gridding tiles are read as the sum of their partial tiles.
    const int2 *split_of_tile;  // [tiles] (first partial slot, chunks); chunks 0: not split
    const float2 *partials;     // [grids][n_slots][tile_cells]
    int64_t n_slots;
    int tile_cells;
    int d;
    int Kax[kMaxDim];
    int T[kMaxDim];
    int nt[kMaxDim];
    const float2 *phase;  // min-max grid phase e^{-i pi k / K} of this pass's axis (nullptr: none)
};
hipError_t launch_strided_pass(const StridedPassArgs &a, hipStream_t s);

// Inverse pass along the contiguous last axis with crop K -> N, scaling and
// coil combination: in [B*C][rows][K] -> x [B][rows][N].
struct LastPassArgs {
    const float2 *in;
    float2 *x;
    const float2 *tw;
    RadixPlan rp;
    const float2 *coils;
    int C, B;
    int K, N;
    int64_t rows;
    int d;
    int Nax[kMaxDim];
    const float *scale[kMaxDim];
    int target_groups;
    const float2 *phase;  // min-max grid phase e^{-i pi k / K} of this pass's axis (nullptr: none)
};
hipError_t launch_last_pass(const LastPassArgs &a, hipStream_t s);

// Geometry shared by the sample kernels.
struct SampleGeom {
    int d;
    int J;
    int K[kMaxDim];
    double C[kMaxDim];   // K_a / (2 pi)
    int jp;               // coefficient row width (coef_row_width(J))
    int nq[kMaxDim];      // coefficient rows of the kernel fit (multiple of 2)
    int nq_d[kMaxDim];    // coefficient rows of the derivative fit
    const float *coef[kMaxDim];   // [nq][jp], highest degree first (coef_rows)
    const float *dcoef[kMaxDim];  // [nq_d][jp]
    int minmax;           // min-max interpolator: real factors c' in coef, plus
                          // the per-sample phase e^{i sum omega/2} and tap signs
    // Optional table of every sorted sample's window, made with the plan
    // (nullptr: the sample kernels evaluate it on the fly).  Record of
    // wtab_stride floats per sample: the wrapped first taps as 16-bit fields
    // (k0 | k1 << 16, then k2), then table_taps(J) weights per axis (zero
    // past J), zero padded to a multiple of 4 floats.
    const float *wtab;
    int wtab_stride;
};
inline int table_taps(int J) { return J <= 6 ? 6 : J <= 8 ? 8 : 16; }
inline int table_stride(int d, int J) { return (2 + d * table_taps(J) + 3) & ~3; }
hipError_t launch_weight_table(const SampleGeom &g, const float *om_sorted, int64_t M, float *out, hipStream_t s);

// Interpolation V: y[g][perm[i]] = sum_taps w * G[g][..] for sorted sample i.
// With items, one workgroup per (bin, chunk) stages the tile plus halo in LDS;
// without (items == nullptr), one thread per sample reads the grid directly.
struct InterpItem {
    int bin;    // first tile
    int start;  // first sorted sample
    int count;  // <= 256 * kInterpSamplesPerThread
    int tiles;  // tiles along the last axis the item covers (their samples are contiguous)
};
struct InterpArgs {
    SampleGeom geo;
    const float *om_sorted;  // [M][d]
    const int *perm;         // sorted -> caller order
    int64_t M;
    const float2 *G;
    int64_t grid_elems;
    int grids;
    float2 *y;               // [grids][M]
    const InterpItem *items;
    int64_t n_items;
    int T[kMaxDim];
    int nt[kMaxDim];
    int merge;  // most tiles one item covers (sizes the LDS region)
};
hipError_t launch_interp(const InterpArgs &a, hipStream_t s);
// Elements of a gather item's LDS region: the tiles (merge of them along the
// last axis) plus the J - 1 halo, the last axis made odd.
inline int64_t interp_region_elems(int d, const int *T, int J, int merge) {
    int64_t n = 1;
    for (int ax = 0; ax < d - 1; ++ax) n *= T[ax] + J - 1;
    return n * ((int64_t(merge) * T[d - 1] + J - 1) | 1);
}

// Gridding V^H, output driven: one work item per (tile, chunk); tiles that
// need more than one chunk write partial tiles that reduce_partials sums.
struct GridItem {
    int tile;
    int chunk;
    int nchunks;
    int slot;  // first partial slot of the tile (nchunks > 1)
};
struct HotTile {
    int tile;
    int slot;
    int nchunks;
    int pad;
};
struct GridArgs {
    SampleGeom geo;
    const float *om_sorted;
    const int *perm;
    const int *sub_start;  // [nbins * 2^d + 1] offsets of the (bin, crossing code) sub-bins
    int64_t M;
    int T[kMaxDim];
    int nt[kMaxDim];
    int R[kMaxDim];
    int tile_cells;
    int seg_len;       // LS: cells of a tile row one lane accumulates (4, 8 or 16)
    int segs;          // segments per tile row, ceil(T_last / LS)
    int group_lanes;   // lanes per sample group: 64, 128 or 256 >= rows * segs, rows = tile_cells / T_last
    int stage_floats;  // LDS floats per group (staged batch, or the group's register tile at the end)
    int chunk;  // samples per work item
    const GridItem *items;
    int64_t n_items;
    const float2 *y;      // [grids][M]: sorted sample order when y_sorted (k_permute_samples
                          // wrote it), else the caller's order, read through perm
    int y_sorted;
    int grids;
    float2 *h;            // [grids][K^d]
    int n_kinds;          // segment kinds: bits 0..2 = neighbour offset e per axis,
    int kinds[kMaxNeighbors];  // bits 8..15 = crossing code, 255 = the whole bin
    int64_t grid_elems;
    float2 *partials;     // [grids][n_slots][tile_cells]
    int64_t n_slots;
    const int2 *item_segs;  // [n_items][kMaxNeighbors + 1]: per segment of the item's tile (first
                            // sorted sample, offset in the item's list), then (0, total)
    int mfma;             // matrix-core gridding (d >= 2, T_last = 16, 16, 32 or 64 rows)
    int rec_stride;       // its LDS floats per staged sample: 2 + sum of T_a, made odd
    int blk;              // 3D matrix-core gridding by 4 x 4 blocks (T_2 = 16, T_0 and T_1 in {8, 16})
    int grids_per_wg;     // row-tile matrix-core gridding: grids one workgroup grids together (1, 2, 4)
    int grid_waves;       // block gridding: wavefronts per work item (1 or 4)
};
// Grids per workgroup of the row-tile matrix-core gridding: the window weights
// are staged once for all of them (coils and batch entries share the
// trajectory); four at most, at most eight accumulator blocks per lane, and
// the staged records (2 floats per grid + the tile's edge lengths tsum, odd)
// of four wavefronts within 64 KiB.
inline int grid_grids_per_wg(int grids, int tile_cells, int tsum) {
    const int mb = tile_cells / 256;
    auto fits = [&](int gp) { return gp * mb <= 8 && 4 * 64 * ((2 * gp + tsum) | 1) * 4 <= 64 * 1024; };
    if (grids >= 3 && fits(4)) return 4;
    if (grids >= 2 && fits(2)) return 2;
    return 1;
}

// Events a timed stage hands to its kernel launch: the launch has the runtime
// stamp them at the kernel's own start and end (hipExtLaunchKernel), so the
// per-kernel timings leave out dispatch and event-record latency.  Set by the
// plan's timing wrapper around one stage (one kernel), null otherwise; per
// host thread.
struct LaunchEvents {
    hipEvent_t start, stop;
    bool used;
};
extern thread_local LaunchEvents *g_launch_events;
hipError_t launch_grid(const GridArgs &a, hipStream_t s);
// ys[g][i] = y[g][perm[i]]: samples into the plan's sorted order.
hipError_t launch_permute_samples(const float2 *y, const int *perm, int64_t M, int grids, float2 *ys,
                                  hipStream_t s);

// The segment kinds of tile_segments in the same order, as a table the
// gridding kernel expands with one lane per segment.
inline int segment_kinds(int d, const int *R, int *kinds) {
    const int ncode = 1 << d;
    int n = 0;
    int e[kMaxDim] = {0, 0, 0};
    while (true) {
        int emask = 0;
        for (int a = 0; a < d; ++a) emask |= e[a] << a;
        if (emask == 0) {
            kinds[n++] = 255 << 8;
        } else {
            for (int c = 0; c < ncode; ++c)
                if ((c & emask) == emask) kinds[n++] = emask | (c << 8);
        }
        int a = d - 1;
        while (a >= 0) {
            if (++e[a] < R[a]) break;
            e[a] = 0;
            --a;
        }
        if (a < 0) break;
    }
    return n;
}

// Sorted-sample segments [lo, hi) whose windows reach tile tc: the whole own
// bin, and from each lower neighbour bin (tc - e, e in {0,1}^d, e_a < R_a)
// only the sub-bins whose crossing code contains e.  Shared by the plan (to
// size work items) and the gridding kernel.  Returns the number of segments:
// at most sum_e 2^(d - |e|) = 3^d - 2^d + 1, i.e. 2 in 1D, 6 in 2D, 20 in 3D.
__host__ __device__ inline int tile_segments(int d, const int *tc, const int *nt, const int *R,
                                             const int *sub_start, int *lo, int *hi) {
    const int ncode = 1 << d;
    int n = 0;
    int e[kMaxDim] = {0, 0, 0};
    while (true) {
        int bin = 0, emask = 0;
        for (int a = 0; a < d; ++a) {
            int b = tc[a] - e[a];
            if (b < 0) b += nt[a];
            bin = bin * nt[a] + b;
            emask |= e[a] << a;
        }
        const int base = bin * ncode;
        if (emask == 0) {
            lo[n] = sub_start[base];
            hi[n] = sub_start[base + ncode];
            ++n;
        } else {
            for (int c = 0; c < ncode; ++c) {
                if ((c & emask) != emask) continue;
                lo[n] = sub_start[base + c];
                hi[n] = sub_start[base + c + 1];
                ++n;
            }
        }
        int a = d - 1;
        while (a >= 0) {
            if (++e[a] < R[a]) break;
            e[a] = 0;
            --a;
        }
        if (a < 0) break;
    }
    return n;
}

struct ReduceArgs {
    const HotTile *hot;
    int64_t n_hot;
    int d;
    int K[kMaxDim];
    int T[kMaxDim];
    int nt[kMaxDim];
    int tile_cells;
    const float2 *partials;
    int64_t n_slots;
    float2 *h;
    int64_t grid_elems;
    int grids;
};
hipError_t launch_reduce_partials(const ReduceArgs &a, hipStream_t s);
// Split-tile reduction: tile cells per workgroup, and threads (interleaved
// partial sums, added in lane order) per cell: 256 threads.
constexpr int kReduceCellsPerWg = 64;
constexpr int kReduceLanes = 4;

// Trajectory gradient: gom[perm[i]][a] = sum_g Re(conj(gy[g][perm[i]]) * dy/domega_a).
struct GradArgs {
    SampleGeom geo;
    const float *om_sorted;
    const int *perm;
    int64_t M;
    const float2 *G;
    int64_t grid_elems;
    int grids;
    const float2 *gy;  // [grids][M]
    float *gom;        // [M][d]
};
hipError_t launch_grad(const GradArgs &a, hipStream_t s);

// Plan-time binning.
struct BinArgs {
    const float *om;
    int64_t M;
    int d;
    int K[kMaxDim];
    double C[kMaxDim];
    int J;
    int T[kMaxDim];
    int nt[kMaxDim];
    int *keys;
    int *counts;
    int *flag;  // set to 1 on a non-finite coordinate
};
hipError_t launch_bin_keys(const BinArgs &a, hipStream_t s);
hipError_t launch_iota(int *v, int64_t n, hipStream_t s);
// ---- many problems in one launch per stage.  Each stage kernel has a form
// that reads its arguments from a device array of per-problem jobs and runs,
// as workgroup b, block blocks[b] = (problem, block x, block y, block z) of
// that problem's own launch; problems whose launches use the same kernel
// instance share one launch.
struct FftLaunch {
    int threads;     // workgroup size
    int64_t blocks;  // workgroups of the problem's launch
    size_t lds;      // dynamic LDS bytes
    int p0;          // first pass: lines per workgroup; strided: columns W; last: rows per workgroup
    int64_t p1;      // strided: column tiles per row block; last: coils per round
};
// threads > 0: the launch of a given workgroup size (64..512, large enough for
// one line of K), lines or columns per workgroup as many as its tile holds.
FftLaunch first_pass_launch(const FirstPassArgs &a, int threads = 0);
FftLaunch strided_pass_launch(const StridedPassArgs &a, int threads = 0);
FftLaunch last_pass_launch(const LastPassArgs &a, int threads = 0);
struct FirstJob {
    FirstPassArgs a;
    int lpw;
};
struct StridedJob {
    StridedPassArgs a;
    int W;
    int64_t ntc;
};
struct LastJob {
    LastPassArgs a;
    int rpw;
    int cpr;
};
struct PermuteJob {
    const float2 *y;
    const int *perm;
    int64_t M;
    int grids;
    float2 *ys;
};
hipError_t launch_first_pass_multi(const FirstJob *jobs, const int4 *blocks, int64_t nblocks, int threads,
                                   size_t lds, hipStream_t s);
hipError_t launch_strided_pass_multi(const StridedJob *jobs, const int4 *blocks, int64_t nblocks, int threads,
                                     bool inverse, bool split, size_t lds, hipStream_t s);
hipError_t launch_last_pass_multi(const LastJob *jobs, const int4 *blocks, int64_t nblocks, int threads, size_t lds,
                                  hipStream_t s);
// LDS of a staged gather launch (0 for the direct form).
size_t interp_lds(const InterpArgs &a);
hipError_t launch_interp_multi(const InterpArgs *jobs, const int4 *blocks, int64_t nblocks, int J, int d,
                               bool staged, size_t lds, hipStream_t s);
// The gridding kernel instance a launch uses (problems with the same value
// share a launch) and its LDS bytes.
int grid_variant(const GridArgs &a);
size_t grid_lds(const GridArgs &a);
hipError_t launch_grid_multi(const GridArgs *jobs, const int4 *blocks, int64_t nblocks, const GridArgs &proto,
                             size_t lds, hipStream_t s);
hipError_t launch_reduce_partials_multi(const ReduceArgs *jobs, const int4 *blocks, int64_t nblocks, hipStream_t s);
hipError_t launch_permute_samples_multi(const PermuteJob *jobs, const int4 *blocks, int64_t nblocks, hipStream_t s);

hipError_t launch_tv_shrink(int d, const int64_t *N, const float2 *x, float2 *dd, float2 *bb, float t, hipStream_t s);
hipError_t launch_tv_rhs(int d, const int64_t *N, float mu, const float2 *ahy, const float2 *df, const float2 *bf,
                         float lam, const float2 *dd, const float2 *bb, float2 *rhs, hipStream_t s);
hipError_t launch_tv_normal(int d, const int64_t *N, float mu, const float2 *ahax, float lam, const float2 *x,
                            float2 *out, hipStream_t s);
hipError_t launch_bregman_shrink(int64_t n, const float2 *r, float2 *dv, float2 *bv, float t, hipStream_t s);
hipError_t launch_dc_update(float *w, const float2 *u, float2 *wc, int64_t M, float inv_c, hipStream_t s);
hipError_t launch_real_to_complex(const float *w, float2 *wc, int64_t M, float scale, hipStream_t s);
// The allocation-free density compensation's buffers: wc and u, kDcScratchMaxM
// complex samples each, in a static device array of the current device.
constexpr int64_t kDcScratchMaxM = int64_t(1) << 21;
constexpr int kMaxDevices = 64;
hipError_t dc_scratch(float2 **wc, float2 **u);
hipError_t launch_permute_points(const float *om, const int *perm, int64_t M, int d, float *om_sorted,
                                 hipStream_t s);
// Stable sort of (key, value) pairs with hipCUB in caller-owned temporary
// storage of temp_bytes (sort_pairs_temp_bytes gives the size for n pairs of
// key_bits-bit keys).  Asynchronous on s; allocates nothing.
hipError_t sort_pairs_temp_bytes(int64_t n, int key_bits, size_t *bytes);
hipError_t sort_pairs(const int *keys_in, int *keys_out, const int *vals_in, int *vals_out, int64_t n,
                      int key_bits, void *temp, size_t temp_bytes, hipStream_t s);

}  // namespace nufft
