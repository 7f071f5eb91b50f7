/*
 * tm.h - C ABI of the MI355X (gfx950) library for reference-less
 * transmission-matrix (TM) retrieval with Fourier-structured probing.
 *
 * Method: Zhong et al., "Efficient reference-less transmission matrix
 * retrieval for a multimode fiber using fast Fourier transform",
 * arXiv 2302.13524. Each TM row t_p (length N = n1*n2 input modes) is
 * recovered from its K*N intensities I_p = |A t_p|^2 where
 *   A = [F diag(psi_1); ...; F diag(psi_K)]                (Sec. 2.2, Eq. probingmatrix)
 * F is the unnormalised 2-D DFT (kernel exp(-2 pi j k i / n)) of the
 * row-major n1 x n2 mode grid (index i = i1*n2 + i2), psi_m are K
 * unit-modulus random-phase masks shared by all rows. A is never stored:
 * A x is K masked 2-D FFTs, A^H y is K inverse FFTs (unnormalised,
 * F^H = N * inverse) multiplied by conj(psi_m) and summed.
 *
 * Conventions for every entry point
 *  - Ownership: every array argument is a caller-owned DEVICE pointer
 *    (hipMalloc / torch), unless the comment says host. The library never
 *    frees or keeps caller pointers after the call returns; it allocates
 *    only its own workspace inside the context (twiddle tables, solver
 *    history), which tm_destroy releases.
 *  - Streams: `stream` is a hipStream_t (NULL = default stream). Calls are
 *    stream-ordered and asynchronous unless the comment says otherwise.
 *  - Layout: row-major, contiguous. Complex values are interleaved
 *    (re, im) float pairs (tm_c32) or double pairs (tm_c64).
 *    Intensities are [P][K][n1][n2] (mask-major per row).
 *  - Errors: functions return TM_OK (0) or a negative code; argument
 *    checks run on the host before any device work is queued, so an error
 *    return means nothing was launched. tm_last_error() gives a message.
 *  - Threads: one context must not be used by two host threads at once.
 *  - Supported grids: n1, n2 powers of two, 16 <= N <= 8192, each of
 *    n1, n2 <= 128, or 1-D grids (n1 = 1) with N <= 8192;
 *    tm_grid_supported() tells.
 */
#ifndef TM_H
#define TM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tm_ctx tm_ctx;

typedef struct { float re, im; } tm_c32;
typedef struct { double re, im; } tm_c64;

enum {
  TM_OK = 0,
  TM_EINVAL = -1,        /* bad argument (null pointer, size, enum value)  */
  TM_EUNSUPPORTED = -2,  /* grid not in the compiled FFT plan set          */
  TM_EHIP = -3,          /* a HIP runtime call failed (message kept)       */
  TM_ENOMEM = -4         /* workspace allocation failed                    */
};

/* Problem size: N = n1*n2 modes, K masks, P rows. */
typedef struct {
  int32_t n1, n2, K, P;
} tm_dims;

/* Intensity storage type. */
enum { TM_F32 = 0, TM_BF16 = 1, TM_U16 = 2 /* camera images only */ };

/* ---- context ----------------------------------------------------------- */

/* Create a context bound to HIP device `device`. *ctx receives the handle. */
int tm_create(tm_ctx **ctx, int device);
/* Destroy a context and free its workspace (synchronises its device). */
int tm_destroy(tm_ctx *ctx);
/* Message for the last error on this context (never NULL). ctx may be NULL
 * for errors from tm_create. */
const char *tm_last_error(const tm_ctx *ctx);
/* 1 if the (n1, n2) grid has compiled FFT kernels, else 0. */
int tm_grid_supported(int32_t n1, int32_t n2);

/* ---- probing operator (Sec. 2.2, Eq. probingmatrix) --------------------- */

enum { TM_FIELD = 0, TM_INTENSITY = 1 };

/* Forward model y = A t for every row.
 *   masks [K][N] tm_c32 unit-modulus mask fields e^{j psi_m}
 *   t     [P][N] tm_c32 TM rows
 *   out_kind TM_FIELD:     out is tm_c32 y[P][K][N]
 *            TM_INTENSITY: out is I[P][K][N] = |y|^2 of type out_dtype
 *                          (TM_F32 float or TM_BF16 bfloat16 bits, RNE)
 * (Eq. forwardmodel applied per pixel as Eq. optTMsmall2.) */
int tm_forward(tm_ctx *ctx, tm_dims d, const tm_c32 *masks, const tm_c32 *t,
               int out_kind, int out_dtype, void *out, void *stream);

/* Adjoint x = A^H y = sum_m conj(psi_m) * F^H y_m for every row
 * (the inverse FFTs the paper uses for Q^H, Sec. 2.2).
 *   y [P][K][N] tm_c32, x [P][N] tm_c32 (overwritten). */
int tm_adjoint(tm_ctx *ctx, tm_dims d, const tm_c32 *masks, const tm_c32 *y,
               tm_c32 *x, void *stream);

/* Packed gradient of f(t) = ||I - |A t|^2||^2 (Eq. derivative, App. A):
 *   grad = -4 A^H ( (A t) (I - |A t|^2) ),  packed as d/dRe + j d/dIm.
 *   I [P][K][N] (I_dtype), grad [P][N] tm_c32, f [P] float (may be NULL):
 *   f_p = sum (I - |A t|^2)^2 with compensated FP32 summation. */
int tm_gradient(tm_ctx *ctx, tm_dims d, const tm_c32 *masks, const void *I, int I_dtype,
                const tm_c32 *t, tm_c32 *grad, float *f, void *stream);

/* Packed gradient of the amplitude cost f_a(t) = || sqrt(I) - |A t| ||^2
 * (the Poisson-noise cost of the Discussion):
 *   grad = -2 A^H ( (sqrt(I) - |A t|) (A t)/|A t| ), (A t)/|A t| := 1 where A t = 0,
 *   f [P] float (may be NULL): f_a per row. Same layouts as tm_gradient. */
int tm_amp_gradient(tm_ctx *ctx, tm_dims d, const tm_c32 *masks, const void *I, int I_dtype,
                    const tm_c32 *t, tm_c32 *grad, float *f, void *stream);

/* FP64 acceptance residual per row:
 *   rho_p = ||I_p - |A t_p|^2||^2 / ||I_p||^2
 * evaluated with FP64 FFTs and FP64 sums from the FP32 inputs.
 *   rho [P] double. */
int tm_residual_f64(tm_ctx *ctx, tm_dims d, const tm_c32 *masks, const void *I, int I_dtype,
                    const tm_c32 *t, double *rho, void *stream);

/* ---- retrieval (Sec. 2.2, Alg. 1) --------------------------------------- */

/* TM_METHOD_LBFGS_AMP: L-BFGS on the amplitude cost sum (sqrt(I) - |A t|)^2,
 * the Poisson-noise form the Discussion names: gradient
 * -2 A^H((sqrt(I) - |y|) y/|y|), line search over the trial steps 1/8 .. 16
 * (the smallest cost wins if below the cost at t, else no step and the row's
 * history is dropped), direction -g/(2KN) with no history. */
/* TM_METHOD_ER_CYCLIC: error reduction with one mask's projection at a time
 * (a solver chosen here, not the paper's): a sweep (one of `iters`) takes
 * m = 1..K in order, y = F(psi_m t), t <- conj(psi_m) F^H(sqrt(I_m) y/|y|)/N,
 * the nearest point of that mask's measurement set; plain TM_METHOD_ER
 * averages the K projections instead. Same cost per sweep as one ER
 * iteration; er_momentum must be 0. The reported f and amp_res are the
 * last sweep's sums, each mask's term at the iterate its projection starts
 * from. */
enum { TM_METHOD_ER = 0, TM_METHOD_LBFGS = 1, TM_METHOD_LBFGS_AMP = 2, TM_METHOD_ER_CYCLIC = 3 };
enum {
  TM_START_GIVEN = 0,     /* use t as passed in                                  */
  TM_START_BACKPROP = 1,  /* t = A^H sqrt(I) / (K N)          (Eq. backpropagation) */
  TM_START_SPECTRAL = 2,  /* truncated spectral start seeded with the t passed in  */
  TM_START_LANCZOS = 3,   /* the same eigenvector by spectral_iters (1..64) Lanczos
                             steps on A^H diag(w) A from the t passed in: Ritz vector
                             of the largest Ritz value (tridiagonal eigenproblem in
                             FP64), scaled to ||t||^2 = sum(I)/(K N); workspace
                             spectral_iters P N complex floats                       */
  TM_START_LEARNED = 4    /* TM_START_LANCZOS with the learned weights w = T(I/mean(I_p))
                             of the table set by tm_set_weight_table instead of the
                             truncation (not in the paper; see the learned start below) */
};

typedef struct {
  int32_t method;          /* TM_METHOD_ER (projection), _ER_CYCLIC, TM_METHOD_LBFGS (Alg. 1) or _AMP */
  int32_t iters;           /* solver iterations (the paper's maxiter), >= 0              */
  int32_t lbfgs_m;         /* L-BFGS memory, 1..16 (default 5)                           */
  int32_t I_dtype;         /* TM_F32 or TM_BF16                                          */
  int32_t start;           /* TM_START_*                                                 */
  int32_t spectral_iters;  /* power-iteration (or Lanczos) steps of the spectral start     */
  float spectral_tau;      /* weight truncation w = min(I/mean(I_p), tau), e.g. 3        */
  float spectral_momentum; /* heavy-ball factor c in [0, 1): beta = (c lambda)^2/4       */
  float er_momentum;       /* ER only: Nesterov factor b in [0, 1): t <- ER(t + b (t - t_prev)); 0 = plain ER */
  float spectral_lower;    /* lower end l of the rest of the spectrum, as a fraction of lambda,
                              in [-1, c]: step x <- (M - s) x - beta x_prev with
                              s = (c + l) lambda / 2, beta = ((c - l) lambda / 2)^2 / 4;
                              l = -c is the unshifted heavy-ball step, l = 0 uses that
                              A^H diag(w) A is positive semidefinite                      */
} tm_retrieve_opts;

/* Per-row results written to device memory. */
typedef struct {
  double rho;      /* FP64 acceptance residual of the returned row              */
  float f;         /* intensity loss sum (I - |A t|^2)^2 at the last evaluation  */
  float amp_res;   /* amplitude residual sum (sqrt(I) - |A t|)^2 (ER only)       */
  int32_t iters;   /* iterations run                                           */
  int32_t flags;   /* bit 0: rho > 1e-2 (row not accepted); bit 1: non-finite   */
} tm_row_stats;

/* Retrieve every row. t is in/out: the start (or the spectral seed) on
 * entry, the result on exit. stats [P] may be NULL. Asynchronous. */
int tm_retrieve(tm_ctx *ctx, tm_dims d, const tm_c32 *masks, const void *I,
                tm_c32 *t, const tm_retrieve_opts *opts, tm_row_stats *stats,
                void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * tm_retrieve restricted to error reduction (TM_METHOD_ER without momentum,
 * or TM_METHOD_ER_CYCLIC) from a TM_START_GIVEN or TM_START_BACKPROP start,
 * with the same arguments, kernels and results. Its per-row sums live in a
 * static device array of the library (about 1.6 MiB per device, held until
 * the process ends) instead of context workspace, so the call runs no
 * hipMalloc, hipFree or other allocating routine and records no events.
 * Every call on one device shares that array: calls that overlap on one GPU
 * (other streams, other host threads, other contexts) race and must be
 * ordered by the caller. Errors: P > TM_NOALLOC_MAX_ROWS -> TM_EINVAL; another
 * method, start or a nonzero er_momentum -> TM_EUNSUPPORTED (nothing launched). */
#define TM_NOALLOC_MAX_ROWS 32768
int tm_retrieve_noalloc(tm_ctx *ctx, tm_dims d, const tm_c32 *masks, const void *I,
                        tm_c32 *t, const tm_retrieve_opts *opts, tm_row_stats *stats,
                        void *stream);

/* ---- uneven batches of TMs ----------------------------------------------- */

/* One retrieval problem of a batch. d.n1 x d.n2 must be one of the grids
 * compiled for batches (32x32, 64x32, 64x64, 128x64); each problem has its
 * own masks [K][N], intensities I [P][K][N] (type opts->I_dtype), in/out
 * rows t [P][N] and optional stats [P]. */
typedef struct {
  tm_dims d;
  const tm_c32 *masks;
  const void *I;
  tm_c32 *t;
  tm_row_stats *stats;
} tm_problem;

typedef struct tm_batch tm_batch;

/* Plan the retrieval of n problems with the same options (method ER or
 * ER_CYCLIC; start GIVEN, BACKPROP, SPECTRAL or LANCZOS). Every iteration is one persistent
 * launch whose work items are (problem, row tile): 1 row of 8192 modes, 2 of
 * 4096, 4 of 2048 or 8 of 1024, each run with its grid's FFT specialisation
 * and the digit order chosen by tm_set_variant. With use_graph = 1 the whole
 * sequence (start, iterations, FP64 residuals, stats) is captured once into a
 * HIP graph. The plan keeps the problem pointers: tm_batch_run reuses them.
 * Allocates its workspace here (not in tm_batch_run). */
int tm_batch_create(tm_ctx *ctx, int32_t n, const tm_problem *probs, const tm_retrieve_opts *opts,
                    int32_t use_graph, tm_batch **out);
/* Run the planned sequence on `stream` (asynchronous). */
int tm_batch_run(tm_batch *b, void *stream);
/* Release the plan (synchronises the device). */
int tm_batch_destroy(tm_batch *b);

/* ---- autotuning ------------------------------------------------------------ */

/* Average device time (microseconds) of one error-reduction launch over P
 * rows of an n1 x n2 grid with K masks, FFT digit-order variant `variant`
 * (0: larger radices first, 1: smaller first), on synthetic data in library
 * workspace. */
int tm_tune_time(tm_ctx *ctx, int32_t n1, int32_t n2, int32_t K, int32_t P, int32_t I_dtype,
                 int32_t variant, int32_t reps, double *us);
/* Use digit-order variant `variant` for the grid n1 x n2 in this context. */
int tm_set_variant(tm_ctx *ctx, int32_t n1, int32_t n2, int32_t variant);

/* Launch configurations of the fused row kernels (the 2-D FFTs of Sec. 2.2,
 * Eq. probingmatrix): cfg in 0..7, bit 0 the digit-order variant (as
 * tm_set_variant), bit 1 eight values per thread instead of sixteen, bit 2
 * twice the rows per workgroup. Bits 1 and 2 change the error-reduction steps
 * (averaged and cyclic), the spectral and Lanczos steps of the start, the
 * gradient kernels of the L-BFGS solvers (Alg. 1 and its amplitude-cost form)
 * and the amplitude cost's line search; every other kernel keeps the default
 * plan of the same digit order. The batch
 * (tm_batch_create) takes bit 0 only, so its rows equal single-problem runs in
 * configurations 0 and 1.
 * They are compiled for the 32x32, 64x32, 64x64 and 128x64 grids (twice the
 * rows only where a workgroup stays at 512 threads or fewer).
 *
 * tm_config_info: 1 if configuration cfg is compiled for the grid, with its
 * threads per workgroup, rows per workgroup and values per thread (each
 * pointer may be NULL); 0 otherwise. No device work. */
int tm_config_info(int32_t n1, int32_t n2, int32_t cfg, int32_t *wg, int32_t *rows_per_wg,
                   int32_t *values_per_thread);
/* Use configuration cfg for the grid n1 x n2 in this context (TM_EUNSUPPORTED
 * if it is not compiled for the grid). */
int tm_set_config(tm_ctx *ctx, int32_t n1, int32_t n2, int32_t cfg);
/* Average device time (microseconds) of one Lanczos-step launch (us[0]) and
 * one cyclic error-reduction launch (us[1]) over P rows of an n1 x n2 grid
 * with K masks in configuration cfg, on synthetic data in library workspace
 * (synchronous, on the null stream). us: host array of 2 doubles. */
int tm_tune_config(tm_ctx *ctx, int32_t n1, int32_t n2, int32_t K, int32_t P, int32_t I_dtype, int32_t cfg,
                   int32_t reps, double *us);

/* ---- phase-offset correction (Sec. 2.3) -------------------------------- */

typedef struct {
  int32_t P;            /* rows (pixels) with a retrieved TM row                   */
  int32_t N;            /* modes per row                                           */
  int32_t Nd;           /* defocus images                                          */
  int32_t nf1, nf2;     /* field grid; images are (2 nf1) x (2 nf2)                */
} tm_defocus_dims;

typedef struct {
  double lambda;   /* wavelength                                   */
  double ps_field; /* field-grid pixel size (same length unit)     */
  double NA;       /* numerical aperture of the pupil              */
  double z;        /* defocus distance z_d                         */
} tm_optics;

typedef struct {
  int32_t iters;       /* L-BFGS iterations over phi (upper bound)                  */
  int32_t m;           /* L-BFGS memory (1..16)                                     */
  double ftol;         /* stop after an accepted iteration that lowers g by at most
                          ftol * g (>= 0; 0 runs all iters)                         */
} tm_phase_opts;

/* Solve the per-row phase offsets phi of TM_true = diag(e^{j phi}) TM_est
 * (Eq. phaseoffset) from defocus intensities by L-BFGS on
 *   g(phi) = sum_n || I_n - | K2^H P diag(h) K1 diag(c_n) e^{j phi} |^2 ||^2
 * (Eq. forwarddefocusImage, Eq. optphase, gradient Eq. phasederive), FP64.
 *   pix    [P] int32 raster index of each row's pixel in the nf1 x nf2 grid
 *   tm_est [P][N] tm_c32, theta [Nd][N] tm_c32 unit-modulus inputs e^{j theta_n}
 *   I_d    [Nd][2nf1][2nf2] float defocus images
 *   phi    [P] double: start on entry (zeros in the paper), result on exit
 *   g_out  host double* (may be NULL): final objective value.
 * Synchronous with respect to the host (the line search runs on the
 * device; the host reads its state between batches of iterations); work
 * is queued on `stream`. Errors: TM_EINVAL for bad sizes, optics or
 * options, and for a pix entry outside the grid or shared by two rows
 * (checked on the device, reported when the call returns, phi unchanged). */
int tm_phase_offset_correct(tm_ctx *ctx, const tm_defocus_dims *dd, const int32_t *pix,
                            const tm_c32 *tm_est, const tm_c32 *theta, const float *I_d,
                            const tm_optics *optics, double *phi, const tm_phase_opts *opts,
                            double *g_out, void *stream);

/* The same solve (Eq. phaseoffset, Eq. optphase, Eq. phasederive), stream-
 * ordered: queues the start, `evals` iterations of the device-side L-BFGS
 * (each decides the pending trial, moves or changes the step, and evaluates
 * the next trial; once the solve has ended an iteration returns at once) and
 * the result, then returns without waiting, so that a caller can overlap the
 * solve with work on another stream. A solve of opts->iters iterations needs
 * as many iterations here as the evaluations tm_phase_last_counts reports for
 * it (the start point's included).
 *   evals  iterations to queue, 1 .. 40 * opts->iters + 2 (ignored when
 *          opts->iters == 0); with fewer than the solve needs, each of them
 *          evaluates a trial (rec[2] = evals + 1) and rec[3] stays 0
 *   rec    device double[7], written when the queued work runs:
 *          [0] objective g, [1] accepted iterations, [2] evaluations,
 *          [3] 1 if the solve ended within `evals` or the pixel check
 *          failed (0: phi holds the iterate reached), [4] pixel check (0: pix valid; bit 0: an entry
 *          outside the grid, bit 1: a pixel shared by two rows, phi then
 *          unchanged), [5], [6] the offending rows.
 * Other arguments as tm_phase_offset_correct. Allocates its workspace on
 * the first call of a size, as that call does; tm_phase_last_counts keeps
 * reporting the last synchronous call. The solve's state lives in the
 * context's workspace: calls on one context must be queued on one stream
 * (solves meant to overlap each other need a context each). Errors: TM_EINVAL for bad sizes,
 * optics or options, evals out of range or rec NULL, returned at once; pix
 * errors only through rec[4]. */
int tm_phase_offset_correct_async(tm_ctx *ctx, const tm_defocus_dims *dd, const int32_t *pix,
                                  const tm_c32 *tm_est, const tm_c32 *theta, const float *I_d,
                                  const tm_optics *optics, double *phi, const tm_phase_opts *opts,
                                  int32_t evals, double *rec, void *stream);

/* Counts of the last tm_phase_offset_correct call on ctx (0 before any):
 * accepted L-BFGS iterations and objective evaluations, the start point's
 * included. The first direction is -sqrt(P) g/||g|| (a = 1 moves the
 * offsets by 1 rad RMS). The line search (Sec. 2.3 leaves it open) tries a = 1 first,
 * doubles a while the trial satisfies Armijo (c1 = 1e-4) but the slope there
 * is still below 0.9 times the slope at phi (at most 20 times) and takes the
 * best such trial; with no acceptable trial it halves a (at most 40 times).
 *   iterations, evaluations: host int32_t* (not NULL).
 * Returns TM_EINVAL on a null argument. */
int tm_phase_last_counts(tm_ctx *ctx, int32_t *iterations, int32_t *evaluations);

/* Evaluation path of the defocus model in tm_phase_objective and
 * tm_phase_offset_correct. h (Eq. angularspectrum) vanishes outside the
 * pupil, so the model only involves the spectrum bins of the pupil's
 * bounding box. enable = 1 (the default): when that box is at most 16 x 16
 * bins, the transforms are pruned to it (one pass builds the box spectrum
 * and its image-axis-2 transform, one pass over the image rows forms a_n,
 * the residual and the adjoint's first axis, one pass maps back to the
 * pixels); otherwise, and with enable = 0, every transform is a full FFT
 * over the field and image grids. Both compute the same objective and
 * gradient up to rounding. */
int tm_phase_set_band(tm_ctx *ctx, int32_t enable);

/* Objective and gradient of the phase-offset problem at phi (FP64):
 *   g_dev [1] double, grad [P] double (both device). */
int tm_phase_objective(tm_ctx *ctx, const tm_defocus_dims *dd, const int32_t *pix,
                       const tm_c32 *tm_est, const tm_c32 *theta, const float *I_d,
                       const tm_optics *optics, const double *phi, double *g_dev,
                       double *grad, void *stream);

/* Defocus images of the forward model (Eq. forwarddefocusImage) for the
 * rows tm [P][N] with offsets phi [P] (double):
 *   I_out [Nd][2nf1][2nf2] float = | K2^H P diag(h) K1 diag(tm e^{j theta_n}) e^{j phi} |^2
 * (used to synthesise defocus data). Same argument rules as
 * tm_phase_objective. */
int tm_defocus_forward(tm_ctx *ctx, const tm_defocus_dims *dd, const int32_t *pix,
                       const tm_c32 *tm, const tm_c32 *theta, const tm_optics *optics,
                       const double *phi, float *I_out, void *stream);

/* ---- learned start (not in the paper; its start is Eq. backpropagation) --- */

/* Network x = I_p / mean(I_p) (n_in = K N features) -> Linear(n_in, hidden)
 * -> GELU -> Linear(hidden, hidden) -> GELU -> Linear(hidden, n_out = 2N),
 * read as u = o[:N] + j o[N:]; the start row is u rescaled to
 * ||t||^2 = sum(I_p) / (K N) (Parseval for A^H A = K N I). GEMMs run on
 * MFMA with BF16 operands and FP32 accumulation. */
typedef struct {
  int32_t n_in, hidden, n_out;
} tm_mlp_dims;

/* Parameters (all device pointers, caller-owned). W[l] is FP32
 * [fan_in][fan_out] row-major; Wh[l] its BF16 copy, written by the library
 * (tm_mlp_sync_bf16, tm_mlp_train_step); b[l] FP32 biases; mW/vW/mb/vb the
 * Adam moments (FP32, same shapes; training only, zero-initialised by the
 * caller). */
typedef struct {
  float *W[3];
  uint16_t *Wh[3];
  float *b[3];
  float *mW[3], *vW[3], *mb[3], *vb[3];
} tm_mlp_params;

/* Write the BF16 weight copies Wh from the FP32 masters W. */
int tm_mlp_sync_bf16(tm_ctx *ctx, const tm_mlp_dims *md, const tm_mlp_params *p, void *stream);

/* Learned start rows t0 [P][N] from intensities I [P][K][N] (float),
 * n_in = K N and n_out = 2 N. */
int tm_mlp_start(tm_ctx *ctx, const tm_mlp_dims *md, const tm_mlp_params *p, int32_t K, int32_t N,
                 const float *I, int32_t P, tm_c32 *t0, void *stream);

/* Gradients of the mean phase-invariant loss over a batch of B rows
 * (I [B][K][N] float, targets t [B][N]); dW[l], db[l] FP32 device buffers
 * shaped like W[l], b[l]; loss [B] per-row loss (device, may be NULL). */
int tm_mlp_gradients(tm_ctx *ctx, const tm_mlp_dims *md, const tm_mlp_params *p, int32_t K, int32_t N,
                     const float *I, const tm_c32 *t, int32_t B, float *const dW[3], float *const db[3],
                     float *loss, void *stream);

/* One training step: gradients as above, then Adam (beta1 0.9, beta2 0.999,
 * eps 1e-8, bias-corrected with step number `step` >= 1) on the FP32
 * masters, and the BF16 copies refreshed. */
int tm_mlp_train_step(tm_ctx *ctx, const tm_mlp_dims *md, const tm_mlp_params *p, int32_t K, int32_t N,
                      const float *I, const tm_c32 *t, int32_t B, float lr, int32_t step, float *loss,
                      void *stream);

/* C [M][N] (float) = op(A) op(B) with BF16 A and B: A is [M][K] (ta = 0) or
 * [K][M] (ta = 1), B is [K][N] (tb = 0) or [N][K] (tb = 1). The MFMA tile
 * used by the network. */
int tm_gemm_bf16(tm_ctx *ctx, int32_t M, int32_t N, int32_t K, const uint16_t *A, int32_t ta,
                 const uint16_t *B, int32_t tb, float *C, void *stream);

/* ---- learned weighting of the spectral start (not in the paper) -------------
 * The spectral start takes the top eigenvector of A^H diag(w) A. Its plain
 * form truncates, w = min(x, tau), x = I / mean(I_p); the learned form uses
 * w = T(x), a function a small network proposes: per point of a uniform
 * table x_b = b xmax / (nt - 1), b < nt, the network maps TM_WNET_FEATURES
 * fixed functions of x_b (the same ones in the library and its tests)
 * through Linear(64, hidden) -> GELU -> Linear(hidden, hidden) -> GELU ->
 * Linear(hidden, 1) to T(x_b) (BF16 MFMA GEMMs, FP32 accumulation; the
 * tm_mlp_dims / tm_mlp_params layout above with n_in = 64, n_out = 1).
 * Weights between the points are linear interpolations; x beyond xmax reads
 * T(xmax). It is trained on (intensity, row) pairs of the forward model:
 * the loss is minus the mean fidelity |t^H u_k|^2 / (||t||^2 ||u_k||^2)
 * after k normalised power steps u <- M u / ||M u|| from seeds v0, and its
 * gradient goes back through the k steps to the table and the network. */
#define TM_WNET_FEATURES 64
#define TM_WTAB_MAX 4096

/* The table of the network: tab [nt][2] float (device) = (T(x_b), T(x_{b+1}) - T(x_b)),
 * the last slope 0. 2 <= nt <= TM_WTAB_MAX, xmax > 0. */
int tm_wnet_table(tm_ctx *ctx, const tm_mlp_dims *md, const tm_mlp_params *p, int32_t nt, float xmax,
                  float *tab, void *stream);

/* Warm start of the network: one Adam step on the mean squared difference
 * between T(x_b) and the plain truncation min(x_b, tau) over the table
 * points. loss [1] device float (may be NULL). */
int tm_wnet_pretrain_step(tm_ctx *ctx, const tm_mlp_dims *md, const tm_mlp_params *p, int32_t nt, float xmax,
                          float tau, float lr, int32_t step, float *loss, void *stream);

/* Training loss of a table and its gradient: d.P rows with true rows t [P][N],
 * intensities I [P][K][N] (I_dtype), seeds v0 [P][N]; `steps` (1..256) power
 * steps with the weights of tab [nt][2]; dtab [nt] float receives d loss / d T(x_b)
 * (overwritten), loss [1] float the loss (both device). */
int tm_wtab_power_grad(tm_ctx *ctx, tm_dims d, const tm_c32 *masks, const void *I, int32_t I_dtype,
                       const tm_c32 *t, const tm_c32 *v0, int32_t steps, const float *tab, int32_t nt, float xmax,
                       float *dtab, float *loss, void *stream);

/* One training step of the network: its table, the loss and table gradient
 * as tm_wtab_power_grad, backward through the network, Adam (as
 * tm_mlp_train_step) and the BF16 copies refreshed. loss [1] device (may be NULL). */
int tm_wnet_train_step(tm_ctx *ctx, const tm_mlp_dims *md, const tm_mlp_params *p, tm_dims d,
                       const tm_c32 *masks, const void *I, int32_t I_dtype, const tm_c32 *t, const tm_c32 *v0,
                       int32_t steps, int32_t nt, float xmax, float lr, int32_t step, float *loss, void *stream);

/* Copy a table [nt][2] into the context for TM_START_LEARNED (stream-ordered). */
int tm_set_weight_table(tm_ctx *ctx, const float *tab, int32_t nt, float xmax, void *stream);

/* Retrieval from the learned start with the plain start as fallback: tm_retrieve
 * with opts->start = TM_START_LEARNED; then every row whose FP64 acceptance
 * residual exceeds rho_fallback is retrieved again from the plain truncated
 * Lanczos start (opts->spectral_tau, seeded with that row's t as passed in),
 * and keeps whichever result has the lower residual. *n_fallback (host)
 * receives the number of rows redone. Synchronises the stream once (to read
 * that count). stats [P] may be NULL. */
int tm_retrieve_learned(tm_ctx *ctx, tm_dims d, const tm_c32 *masks, const void *I, tm_c32 *t,
                        const tm_retrieve_opts *opts, double rho_fallback, tm_row_stats *stats,
                        int32_t *n_fallback, void *stream);

/* ---- instrumentation ------------------------------------------------------ */

/* Enable (1) or disable (0) per-launch HIP-event timing of the fused row
 * kernels issued by this context; enabling clears the accumulated times. */
int tm_profile_enable(tm_ctx *ctx, int enable);
/* Accumulated device time (milliseconds) and launch count of the fused row
 * kernel of kind `mode` (0 forward field, 1 forward intensity, 2 adjoint,
 * 3 error reduction, 4 gradient, 5 spectral step, 6 line-search sums,
 * 7 FP64 residual, 8 back-propagation, 9 amplitude gradient, 10 amplitude
 * line sums, 11 filter, 12 cyclic error reduction, 13 Lanczos step, 14
 * Lanczos step with learned weights, 15/16 weight-network training), or of the
 * L-BFGS direction's coefficients (20: its dot-product pass and small solve
 * together; d itself is formed by the line-search kernel) and step (21), since
 * enabling; mode < 24. Synchronises the context's device. */
int tm_profile_query(tm_ctx *ctx, int mode, double *ms, int64_t *launches);

/* ---------------------------------------------------------------------------
 * Preprocessing of the measured image stack (Sec. 2.2, the paragraph after
 * Algorithm 1): the images are half-sampled (the 1-based odd rows and
 * columns, i.e. 0-based even: an (H/2) x (W/2) grid, raster index
 * q = y (W/2) + x), a binary fiber mask keeps the pixels holding frac
 * (0.999 in the paper) of the total intensity, and each kept pixel becomes
 * one row of K N intensities (one per image, in image order = the row order
 * of A).
 *   stack  [n_img][H][W] device, TM_U16 (camera counts) or TM_F32, H and W even
 */

/* energy [(H/2)(W/2)] double (device): intensity of each kept pixel summed
 * over all images, FP64 (exact for TM_U16 stacks). */
int tm_pre_energy(tm_ctx *ctx, const void *stack, int32_t stack_dtype, int64_t n_img, int32_t H, int32_t W,
                  double *energy, void *stream);

/* The smallest set of pixels, taken by decreasing energy (ties by increasing
 * raster index), whose summed energy first reaches frac (0 < frac <= 1) of
 * the total; an all-zero energy gives the empty set. pix [npix] int32
 * (device) receives the set in increasing raster order, *P_out (host) its
 * size. npix <= 8192 (the sort runs in one workgroup's LDS); energies must be
 * non-negative. Synchronous with respect to the host. */
int tm_pre_fiber_mask(tm_ctx *ctx, const double *energy, int32_t npix, double frac, int32_t *pix,
                      int32_t *P_out, void *stream);

/* out [P][n_img] (device, TM_F32 or TM_BF16 with round-to-nearest-even):
 * out[p][i] = stack[i][2 y_p][2 x_p] with pix[p] = y_p (W/2) + x_p, i.e. the
 * rows tm_retrieve takes as I [P][K][n1][n2] when n_img = K n1 n2. pix
 * entries are checked on the host (outside the grid: TM_EINVAL). */
int tm_pre_gather(tm_ctx *ctx, const void *stack, int32_t stack_dtype, int64_t n_img, int32_t H, int32_t W,
                  const int32_t *pix, int32_t P, void *out, int32_t out_dtype, void *stream);

/* ---------------------------------------------------------------------------
 * Validation by foci (Sec. 3): the phase of the conjugate of each row of
 * tm_est, u_p = exp(-j arg tm_est[p]) (1 where tm_est is 0), is displayed on
 * the modulator; the focus image is |sum_n tm_true[q][n] u_p[n]|^2 over the
 * rows q of tm_true (one complex FP32 GEMM, tm_cgemm_f32), and its power
 * ratio is the power in the (2w+1) x (2w+1) grid window around the brightest
 * pixel (first in raster order on ties; the window is clipped at the grid
 * border) over the image's total power (w = 3: the paper's 7 x 7 window).
 *   tm_est [Pf][N] tm_c32 (the patterns), tm_true [G][N] tm_c32 (the system,
 *   one row per image pixel), pix [G] int32 distinct raster indices of those
 *   pixels on a g1 x g2 grid (checked on the host); pr [Pf] float, peak [Pf]
 *   int32 raster index of each image's peak (-1 and PR 0 for an image with no
 *   power). Workspace Pf N + Pf G complex floats. */
int tm_foci_power_ratio(tm_ctx *ctx, int32_t Pf, int32_t G, int32_t N, const tm_c32 *tm_true, const int32_t *pix,
                        const tm_c32 *tm_est, int32_t g1, int32_t g2, int32_t w, float *pr, int32_t *peak,
                        void *stream);

/* Comparator without FFTs (Sec. 2.2, Table time): the gradient of
 * f(t) = ||I - |Q t|^2||^2 for an explicit dense probing matrix Q [M][N]
 * (e.g. random phases), grad = -4 Q^H((Q t)(I - |Q t|^2)), as two complex
 * FP32 GEMMs (tm_cgemm_f32, Theta(M N) per row) around a fused pointwise kernel.
 *   Q [M][N] tm_c32, I [P][M] float, t [P][N] tm_c32, grad [P][N] tm_c32,
 *   f [P] float (may be NULL). Workspace P M complex floats. */
/* Complex FP32 GEMM on the matrix cores (the products of the foci and of the
 * dense comparator): C = A op(B), op(B) = B^T when trans_b (B stored [N][K])
 * and B otherwise (stored [K][N]); conj(C) when conj_c. Row-major complex64
 * device arrays with leading dimensions (in complex elements) lda >= K,
 * ldb >= K (trans_b) or >= N, ldc >= N; C must not overlap A or B. FP32
 * products and sums (32 x 32 x 2 FP32 MFMAs over K, one per real and one per
 * imaginary part). TM_EINVAL on bad sizes or null pointers; M or N = 0 does
 * nothing. */
int tm_cgemm_f32(tm_ctx *ctx, int32_t M, int32_t N, int32_t K, const tm_c32 *A, int64_t lda, const tm_c32 *B,
                 int64_t ldb, int32_t trans_b, tm_c32 *C, int64_t ldc, int32_t conj_c, void *stream);

int tm_dense_gradient(tm_ctx *ctx, int32_t M, int32_t N, int32_t P, const tm_c32 *Q, const float *I,
                      const tm_c32 *t, tm_c32 *grad, float *f, void *stream);

/* Propagated TM (Sec. 4, 3-D foci): every column of tm [P][N], laid out on
 * the g1 x g2 output grid at the pixels pix [P] (zero elsewhere), propagated
 * by optics->z with the angular-spectrum kernel of Eq. angularspectrum
 * (pupil NA, wavelength lambda, grid pixel ps_field):
 *   out [g1 g2][N] tm_c32 = ifft2(h_z .* fft2(column)) for every column,
 * i.e. the TM at the plane z for every grid pixel. (g1, g2) must be a
 * compiled FFT grid (tm_grid_supported); the 2-D FFTs run in the fused row
 * kernel, one column per row group. Workspace N g1 g2 complex floats. */
int tm_propagate_tm(tm_ctx *ctx, int32_t P, int32_t N, const tm_c32 *tm, const int32_t *pix, int32_t g1, int32_t g2,
                    const tm_optics *optics, tm_c32 *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* TM_H */
