/*
 * nufft_mi355x: the NUFFT pair A = V F S and A^H = S^H F^H V^H on one MI355X
 * (gfx950) GPU.
 *
 * The operator follows the paper (PyNUFFT, arXiv 1710.03197):
 *   Section 2.1, Eq. A = VFS: scaling S, oversampled FFT F (zero padding from
 *     N to K per axis), interpolation V onto M non-Cartesian samples;
 *   Section 2.1 "Adjoint PyNUFFT", Eq. A^H = S^H F^H V^H: gridding V^H, inverse
 *     oversampled FFT with crop, rescaling;
 *   Section 2.1, batch mode ("serial or parallel processing");
 *   Section 2.2 "Multi-coil regularized image reconstruction": coil maps c_i
 *     multiply before A and, conjugated, after A^H.
 *
 * Conventions.  Arrays are C order (last axis fastest).  Image index i_a in
 * [0, N_a) stands for n_a = i_a - N_a/2.  The forward kernel is e^{-i omega.n}
 * (y_m ~ sum_n x_n e^{-i omega_m . n}); FFTs are unnormalised both ways, so the
 * adjoint is the exact conjugate transpose of the forward (no 1/K^d factor).
 * The interpolator is a separable Kaiser-Bessel kernel of J taps per axis with
 * Beatty's shape beta_a = pi sqrt((J/s_a)^2 (s_a - 1/2)^2 - 0.8), s_a = K_a/N_a;
 * the scaling is the reciprocal of its continuous Fourier transform.  The
 * window of sample m on axis a is the J integers in (u - J/2, u + J/2],
 * u = omega_{m,a} * (K_a / (2 pi)) evaluated as one float64 multiply; taps wrap
 * modulo K_a, so any finite omega is accepted (periodic).
 *
 * Data types: images and samples are complex64 (interleaved float re, im);
 * trajectories are float32 [M][d] in radians.  Arithmetic is float32 with
 * float32 accumulation; window positions are float64.
 *
 * Memory: every pointer argument named *_dev is device memory that the caller
 * owns; the library never frees or retains it beyond the call (nufft_plan and
 * nufft_set_points copy the trajectory).  A plan owns its workspace.
 *
 * Streams: `stream` is a hipStream_t (NULL = the default stream).  Transform
 * calls are asynchronous on that stream and allocate nothing once the plan's
 * workspace is large enough for the batch (see nufft_reserve), so they may be
 * captured into a hipGraph.  Plan creation and nufft_set_points synchronise.
 *
 * Concurrency: a plan owns one workspace, so at most one call per plan may be
 * in flight; distinct plans are independent.
 *
 * Errors: every entry point returns a nufft_status (0 = success, negative =
 * failure) and never throws or aborts.  nufft_last_error() returns a
 * thread-local description of the most recent failure on the calling thread.
 */
#ifndef NUFFT_MI355X_H
#define NUFFT_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NUFFT_OK = 0,
    NUFFT_ERR_INVALID_ARG = -1, /* a size, pointer or count is out of range */
    NUFFT_ERR_NO_DEVICE = -2,   /* no HIP device is visible */
    NUFFT_ERR_OOM = -3,         /* a device allocation failed */
    NUFFT_ERR_HIP = -4,         /* a HIP runtime call or kernel launch failed */
    NUFFT_ERR_BAD_PLAN = -5,    /* NULL, destroyed or foreign plan handle */
    NUFFT_ERR_NONFINITE = -6,   /* a trajectory coordinate is NaN or infinite */
    NUFFT_ERR_UNSUPPORTED = -7  /* valid request the library does not handle */
} nufft_status;

typedef struct nufft_plan_s *nufft_plan_t;

/* Create a plan for the d-dimensional pair (Section 2.1, Eq. A = VFS).
 *   d      : 1, 2 or 3.
 *   N[d]   : image size per axis, even, >= 2.
 *   K[d]   : oversampled grid size per axis, even, K_a >= N_a, K_a <= 4096,
 *            and K_a has no prime factor above 5 (mixed-radix 2/3/4/5/8 FFT).
 *   J      : taps per axis, 2 <= J <= 16 and J <= K_a.
 *   M      : number of samples, 0 <= M < 2^31.
 *   om_dev : device float32 [M][d], radians; copied into the plan.  May be
 *            NULL when M == 0.
 *   stream : stream used for the plan-time kernels; the call synchronises it.
 *   out    : receives the handle.
 * Errors: INVALID_ARG, NO_DEVICE, OOM, HIP, NONFINITE (no plan is returned). */
int nufft_plan(int d, const int64_t *N, const int64_t *K, int J, int64_t M,
               const float *om_dev, void *stream, nufft_plan_t *out);

/* Tuning knobs of a plan; 0 in any field keeps the built-in default.  Any
 * choice gives the same operator (to float32 rounding); only speed changes.
 *   tile[a]       grid tile edge on axis a for binning, gathering and
 *                 gridding (rounded to a divisor of K_a that is >= J - 1)
 *   grid_chunk    samples per gridding work item (>= 64)
 *   fft_groups    workgroups the FFT passes aim to launch (sets lines or
 *                 columns per workgroup)
 *   interp_direct 1: the interpolation reads taps straight from the grid
 *                 (through the caches) instead of staging tile + halo in LDS
 *   presort       1: the gridding reads the samples after one permute into
 *                 the plan's sorted order; 2: through the permutation;
 *                 0: the default (1 for d = 3, 2 otherwise)
 *   fuse_reduce   1: the partial tiles of split gridding tiles are summed by
 *                 the first inverse FFT pass; 2: by a kernel of their own;
 *                 0: the default (1 for d = 2, 2 otherwise; always 2 for d = 1)
 *   grid_mfma     1: gridding on the matrix cores (d = 3 with tile[2] =
 *                 16, tile[0], tile[1] in {8, 16} and tile[0] tile[1] <=
 *                 128: by 4 x 4 blocks of
 *                 the leading axes; otherwise by row tiles, which need
 *                 tile[d-1] = 16, 16, 32 or 64 cells over the leading axes
 *                 and sum(tile) <= 61, else NUFFT_ERR_UNSUPPORTED);
 *                 2: on the vector ALUs; 3: matrix cores by row tiles
 *                 also where the block form applies; 0: matrix cores
 *                 where the tile allows it (d >= 2)
 *   interpolator  0: Kaiser-Bessel (the workloads' kernel); 1: min-max (the
 *                 paper's default, Section 2.1 "Interpolation", after Fessler
 *                 and Sutton): per sample and axis the J coefficients that
 *                 minimise the worst-case interpolation error over unit-norm
 *                 images for the scaling factors 1/Phi((n + 1/2)/K), Phi the
 *                 Kaiser-Bessel transform (the same J and beta).  With
 *                 min-max, nufft_grad_points and nufft_density_compensation
 *                 return NUFFT_ERR_UNSUPPORTED.
 *   weight_table  1: the plan stores every sample's interpolation window
 *                 (first taps and the J weights per axis, made with the
 *                 binning: M * 4 * (2 + d * J') bytes rounded up to 16 per
 *                 sample, J' = J rounded up to 6, 8 or 16), and the
 *                 gridding and the staged interpolation read it instead of
 *                 evaluating the kernel per sample (the paper's precomputed
 *                 interpolator, Section 2.1 "Interpolation"); Kaiser-Bessel
 *                 only (with min-max: NUFFT_ERR_UNSUPPORTED); 0: evaluate on
 *                 the fly
 *   fft_radix     radix schedule of the Stockham FFT passes on every axis
 *                 (Section 2.1 "Oversampled FFT"): 0: radices 8, 4, 2, 3, 5
 *                 taken greedily in that order; 1: 4, 8, 2, 3, 5; 2: 3, 5,
 *                 8, 4, 2; 3: schedule 0's passes in reverse order
 *   grid_waves    wavefronts per work item of the gridding by 4 x 4 blocks:
 *                 4 (the default, 0 asks for it) sum their partial tiles
 *                 in a fixed order at the end; 1: one wavefront per item,
 *                 which writes its tile from registers (pair it with a
 *                 smaller grid_chunk); ignored by the other gridding kernels
 *   reserved      must be 0
 *   interp_merge  most grid tiles along the last axis that one interpolation
 *                 work item covers when their samples are few (>= 1; the
 *                 region it stages must fit 64 KiB of LDS, wider runs are
 *                 cut to what fits); 0: the default (1 for d <= 2, 2 for d = 3)
 * Other values give NUFFT_ERR_INVALID_ARG.
 * Used by the autotuner (paper_1710_03197_amd/autotune.py). */
typedef struct {
    int tile[3];
    int grid_chunk;
    int fft_groups;
    int interp_direct;
    int presort;
    int fuse_reduce;
    int grid_mfma;
    int interpolator;
    int interp_merge;
    int weight_table;
    int fft_radix;
    int grid_waves;
    int reserved[2];
} nufft_options_t;

/* nufft_plan with tuning options (opt may be NULL = defaults). */
int nufft_plan_ex(int d, const int64_t *N, const int64_t *K, int J, int64_t M, const float *om_dev,
                  const nufft_options_t *opt, void *stream, nufft_plan_t *out);

/* Replace the trajectory (same M) and re-bin it; synchronises `stream` (and
 * the stream of the plan's previous call).  On NONFINITE the plan keeps its
 * previous trajectory.  The binning scratch is owned by the plan, and the
 * work-item tables are rewritten in place when the new ones fit, so a re-bin
 * allocates device memory only when the new trajectory needs larger tables.
 * The plan's tables change: a hipGraph captured from this plan's transforms
 * before the call must not be replayed after it (capture again). */
int nufft_set_points(nufft_plan_t plan, const float *om_dev, void *stream);

/* Coil mode (Section 2.2, multi-coil): with C >= 1 maps c_dev = complex64
 * [C][N^d] (copied into the plan), the forward maps one image x to C sample
 * vectors y_i = A (c_i * x), stored [C][M], and the adjoint maps [C][M] to one
 * image sum_i conj(c_i) * A^H y_i.  C = 0 (c_dev NULL) returns to single mode.
 * Synchronous. */
int nufft_set_coils(nufft_plan_t plan, int C, const void *c_dev);

/* Grow the plan's workspace for batches of up to B images (B * C grids).  The
 * batched calls grow it on demand; calling this first keeps them
 * allocation-free. */
int nufft_reserve(nufft_plan_t plan, int B);

/* y = A x (Section 2.1, Eq. A = VFS).  x_dev complex64 [N^d]; y_dev complex64
 * [M] ([C][M] in coil mode), in the caller's sample order.  x and y must not
 * overlap.  Asynchronous on `stream`. */
int nufft_forward(nufft_plan_t plan, const void *x_dev, void *y_dev, void *stream);

/* x = A^H y (Section 2.1, Eq. A^H = S^H F^H V^H): x_n ~ sum_m y_m e^{+i omega_m.n}.
 * y_dev complex64 [M] ([C][M] in coil mode); x_dev complex64 [N^d]. */
int nufft_adjoint(nufft_plan_t plan, const void *y_dev, void *x_dev, void *stream);

/* B independent transforms sharing the trajectory (Section 2.1, batch mode):
 * x [B][N^d] -> y [B][M] ([B][C][M] in coil mode), and back. */
int nufft_forward_batched(nufft_plan_t plan, int B, const void *x_dev, void *y_dev, void *stream);
int nufft_adjoint_batched(nufft_plan_t plan, int B, const void *y_dev, void *x_dev, void *stream);

/* Trajectory gradient of a real loss L through y = A(omega) x (torch
 * convention): given gy_dev = dL/dRe y + i dL/dIm y, complex64 [M] ([C][M] in
 * coil mode), writes gom_dev float32 [M][d] with
 *   gom[m][a] = sum_i Re( conj(gy_i[m]) * dy_i[m]/domega_{m,a} ),
 * the derivative taken through the interpolation weights (derivative of the
 * Kaiser-Bessel kernel) of the same approximate operator.  x_dev is the image
 * the forward was applied to.  Uses the plan's workspace for F S (c_i x). */
int nufft_grad_points(nufft_plan_t plan, const void *x_dev, const void *gy_dev,
                      float *gom_dev, void *stream);

/* The trajectory gradient summed over a batch of B images sharing the
 * trajectory (Section 2.1, batch mode): x_dev complex64 [B][N^d], gy_dev
 * complex64 [B][M] ([B][C][M] in coil mode), gom_dev float32 [M][d] =
 * sum_b of the single-image gradient.  The workspace grows to B * C grids on
 * the first call with a larger batch (see nufft_reserve). */
int nufft_grad_points_batched(nufft_plan_t plan, int B, const void *x_dev, const void *gy_dev,
                              float *gom_dev, void *stream);

/* Stage entry points, for stage-wise checks.  The K^d grid is complex64 in C
 * order (no batching, no coils):
 *   nufft_stage_fs   : G = F S x   (scaling, zero padding, oversampled FFT)
 *   nufft_stage_v    : y = V G     (interpolation only)
 *   nufft_stage_vh   : h = V^H y   (gridding only; h is fully overwritten)
 *   nufft_stage_shfh : x = S^H F^H h (inverse FFT, crop, rescaling) */
int nufft_stage_fs(nufft_plan_t plan, const void *x_dev, void *G_dev, void *stream);
int nufft_stage_v(nufft_plan_t plan, const void *G_dev, void *y_dev, void *stream);
int nufft_stage_vh(nufft_plan_t plan, const void *y_dev, void *h_dev, void *stream);
int nufft_stage_shfh(nufft_plan_t plan, const void *h_dev, void *x_dev, void *stream);

/* Plan facts: beta per axis, the kernel's polynomial degree, tile shape,
 * number of bins / scatter work items, workspace bytes.  Any pointer may be
 * NULL.  Host only. */
int nufft_plan_info(nufft_plan_t plan, double *beta3, int *poly_degree, int *tile3,
                    int64_t *n_bins, int64_t *n_items, int64_t *workspace_bytes);

/* Kernel weights the GPU evaluates, computed on the host from the same
 * plan-time polynomial fit (float32 coefficients, float32 Horner): for
 * fractional offsets f[i] in [0, 1) writes w[i*J + j] = phi(f + J/2 - 1 - j),
 * phi(t) = I0(beta sqrt(1 - (2t/J)^2)) with beta from (J, sigma), and
 * dw[i*J + j] = phi'(f + J/2 - 1 - j) (dw may be NULL).  Needs no device. */
int nufft_kernel_weights_host(int J, double sigma, int64_t n, const double *f, double *w, double *dw);

/* Per-kernel timing: with enable = 1 the plan records a pair of HIP events on
 * the launch stream around every kernel it launches (not for graph capture);
 * enable = 0 stops.  Either call discards the records collected so far.
 * nufft_timing_read reports, for kernel index k in [0, nufft_timing_kernels()),
 * its name (static storage), the number of launches recorded and their summed
 * duration in milliseconds; it waits for the recorded events. */
int nufft_timing_enable(nufft_plan_t plan, int enable);
int nufft_timing_kernels(void);
int nufft_timing_read(nufft_plan_t plan, int kernel, const char **name, int64_t *launches, double *total_ms);

/* ---- Many uneven problems in one launch (Section 2.1 batch mode, Section 2.2
 * coils): P independent transforms with their own sizes, trajectories and
 * coil maps, all with the same d and J. */
typedef struct {
    int d;              /* 1, 2 or 3 (the same for every problem) */
    int64_t N[3];       /* image size (first d used) */
    int64_t K[3];       /* grid size (first d used) */
    int J;              /* taps per axis (the same for every problem) */
    int64_t M;          /* samples */
    const float *om;    /* device float32 [M][d], copied */
    int C;              /* coils, 0 = none */
    const void *coils;  /* device complex64 [C][N^d] or NULL, copied */
    const nufft_options_t *opt;  /* this problem's plan options, NULL = defaults */
} nufft_problem_t;

typedef struct nufft_multi_s *nufft_multi_t;

/* Plan P problems (1 <= P <= 256); synchronous.  Errors as nufft_plan, plus
 * UNSUPPORTED when d or J differ between problems. */
int nufft_multi_plan(int P, const nufft_problem_t *probs, void *stream, nufft_multi_t *out);

/* x[p] complex64 [N_p^d] -> y[p] complex64 [M_p] ([C_p][M_p] with coils) for
 * every p, and back.  x and y are host arrays of P device pointers.  Every
 * stage (FFT pass, gather, gridding, partial sums) runs as ONE kernel launch
 * over the work blocks of all problems and coils -- problems whose stage uses
 * a different kernel instance (e.g. another FFT workgroup size) get a launch
 * of their own -- so the number of launches does not grow with P; each
 * workgroup reads its problem's arguments from a device table.  The first
 * call with a given set of pointers builds those tables (synchronous
 * uploads) and captures the launches into a HIP graph; later calls with the
 * same pointers replay it with one graph launch (the last 4 pointer sets per
 * direction are kept).  Asynchronous on `stream` after the first call; a
 * first call with new pointers must not happen inside a stream capture. */
int nufft_multi_forward(nufft_multi_t m, const void *const *x_dev, void *const *y_dev, void *stream);
int nufft_multi_adjoint(nufft_multi_t m, const void *const *y_dev, void *const *x_dev, void *stream);

/* Kernel launches that one call of each direction makes (in its graph), for
 * the most recently used pointer set; -1 for a direction not called yet.
 * Either pointer may be NULL.  Host only. */
int nufft_multi_info(nufft_multi_t m, int64_t *launches_fwd, int64_t *launches_adj);

/* Synchronises and frees the sub-plans and cached graphs; a NULL or foreign
 * handle returns BAD_PLAN. */
int nufft_multi_destroy(nufft_multi_t m);

/* ---- Toeplitz normal operator (Section 2.1, "Self-adjoint NUFFT"; Table 1)
 *
 * out = A^H W A x applied without the interpolator: with the point-spread
 * function p[Delta] = sum_m w_m e^{+i omega_m . Delta}, Delta in [-N, N)^d,
 *   out[n] = sum_{n'} p[n - n'] x[n'],
 * computed as crop(F^-1(P . F(pad(x)))) on the 2N grid, P the FFT of p
 * divided by prod(2N).  Each application costs two zero-padded FFTs of size
 * 2N and a product (fused into the first inverse pass), against a forward +
 * adjoint pair through the interpolator.
 *
 * nufft_toeplitz_plan builds P from `plan`'s trajectory: one adjoint NUFFT
 * with image 2N on grid 2K (same J and oversampling) of the weights, then one
 * FFT.  w_dev: device float [M] real sample weights in the caller's sample
 * order (density compensation), NULL for w = 1.  Synchronous on `stream`;
 * needs 2N_a 2-3-5 smooth and <= 4096 and 2K_a <= 4096 (NUFFT_ERR_UNSUPPORTED),
 * finite weights (NUFFT_ERR_NONFINITE).  The operator keeps a reference to
 * `plan`: destroy the operator first; calls after the plan is gone return
 * NUFFT_ERR_BAD_PLAN.
 *
 * nufft_toeplitz_apply: x_dev complex64 [B][N^d] -> out_dev complex64
 * [B][N^d], asynchronous on `stream`.  In coil mode (the plan's coils at the
 * time of the call) out = sum_i conj(c_i) . T(c_i . x), i.e. A_c^H W A_c with
 * A_c the coil-mode forward.  x and out must not overlap.  The workspace
 * grows on the first call with a larger B * C (that call allocates).
 */
typedef struct nufft_toeplitz_s *nufft_toeplitz_t;
int nufft_toeplitz_plan(nufft_plan_t plan, const float *w_dev, void *stream, nufft_toeplitz_t *out);
int nufft_toeplitz_apply(nufft_toeplitz_t t, int B, const void *x_dev, void *out_dev, void *stream);
int nufft_toeplitz_destroy(nufft_toeplitz_t t);

/* Sampling-density compensation weights (Section 2.2, "Density compensation
 * and gridding", Eq. of the stable iterations, after Pipe and Menon):
 *   w <- w / (V V^H w)   (elementwise), `iters` times,
 * with V the plan's interpolator (the gather of Eq. A = VFS) with the
 * Kaiser-Bessel kernel normalised to peak 1, and V^H its gridding.  The paper
 * writes A A^H; Pipe and Menon's iteration divides by the gridding kernel's
 * convolution at the samples, which V V^H is: real and positive for
 * positive w, so the iteration stays real and stable (with the whole A the
 * quotient is complex and oscillates on undersampled radial trajectories).
 * A zero or non-finite (V V^H w)_m leaves w_m unchanged.  Coils
 * are ignored (the weights belong to the trajectory).  w_dev: device float
 * [M] in the caller's sample order, the starting weights on entry (e.g. all
 * 1) and the result on return.  The gridding reconstruction is then
 * x = A^H (y . w).  Allocates temporary buffers; synchronous on `stream`. */
int nufft_density_compensation(nufft_plan_t plan, int iters, float *w_dev, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * iteration and kernels as nufft_density_compensation, with its two complex
 * [M] sample buffers taken from a static device array of the library instead
 * of hipMalloc.  Calls no hipMalloc/hipFree and no allocating library
 * routine; asynchronous on `stream` (no synchronisation).  Limits and errors:
 * M <= 2^21 samples (the array holds 2 x 2^21 complex64 = 32 MiB per GPU,
 * kept from the first call on that GPU until the process ends), else
 * NUFFT_ERR_INVALID_ARG; the plan's own workspace (made by nufft_plan and
 * nufft_set_points) must exist, else NUFFT_ERR_INVALID_ARG.  Every call on
 * one GPU shares that GPU's array: calls that overlap in time on one GPU
 * (other streams, other threads, other plans) race and give wrong weights;
 * serialise them.  The array keeps the last call's contents; nothing in it
 * needs to start at zero. */
int nufft_density_compensation_noalloc(nufft_plan_t plan, int iters, float *w_dev, void *stream);

/* ---- L1TV split-Bregman pieces (Section 2.2, "Iterative NUFFT": the image
 * gradient, Eq. TV, and the L1TV-OLS / L1TV-LAD iterations).  Image-domain
 * kernels, independent of any plan; every array is device complex64 in C
 * order, images [N^d], gradient-shaped arrays [d][N^d] (axis-major).
 *   grad_a x = x(.., i_a + 1, ..) - x(.., i_a, ..)   (wrap-around)
 *   grad_a^T g = g(.., i_a - 1, ..) - g(.., i_a, ..)
 *   shrink(z, t) = z / |z| * max(|z| - t, 0)
 * All are asynchronous on `stream`; the in/out arrays must not overlap
 * except as stated; NUFFT_ERR_INVALID_ARG on bad sizes, NULL pointers or a
 * negative / non-finite threshold. */
/* For every axis a and pixel: z = grad_a x + b_a; d_a = shrink(z, t);
 * b_a = z - d_a (d_dev, b_dev: [d][N^d], updated in place). */
int nufft_tv_shrink(int d, const int64_t *N, const void *x_dev, void *d_dev, void *b_dev, float t, void *stream);
/* rhs = mu (ahy + df - bf) + lam sum_a grad_a^T (d_a - b_a); df and bf
 * (the LAD data-term split) both NULL for L1TV-OLS. */
int nufft_tv_rhs(int d, const int64_t *N, float mu, const void *ahy_dev, const void *df_dev, const void *bf_dev,
                 float lam, const void *d_dev, const void *b_dev, void *rhs_dev, void *stream);
/* out = mu ahax + lam sum_a grad_a^T grad_a x, ahax = A^H A x computed by the
 * caller (pair or Toeplitz operator): the system matrix K of the inner
 * iterations applied to x. */
int nufft_tv_normal(int d, const int64_t *N, float mu, const void *ahax_dev, float lam, const void *x_dev,
                    void *out_dev, void *stream);
/* n complex values: z = r + b; d = shrink(z, t); b = z - d (d, b in place). */
int nufft_bregman_shrink(int64_t n, const void *r_dev, void *d_dev, void *b_dev, float t, void *stream);

/* Synchronise the plan's last stream and free everything.  A NULL, destroyed
 * or foreign handle returns BAD_PLAN and is not touched. */
int nufft_destroy(nufft_plan_t plan);

const char *nufft_status_string(int status);
const char *nufft_last_error(void);

/* Number of visible HIP devices (0 when none); needs no plan. */
int nufft_device_count(void);

#ifdef __cplusplus
}
#endif

#endif /* NUFFT_MI355X_H */
