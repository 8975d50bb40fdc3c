/*
 * foe.h -- C ABI of the MI355X (gfx950) FoE + iPiano despeckling library.
 *
 * The library minimises the FoE-regularised speckle energies of
 * Chen, Feng, Ranftl, Qiao and Pock, "A higher-order MRF based variational
 * model for multiplicative noise reduction":
 *
 *   E(u, f) = E_FoE(u) + D(u, f),  E_FoE(u) = sum_i theta_i sum_p rho((k_i * u)_p),
 *   rho(x) = log(1 + x^2)                                   (Sec. II-A, eq. (FOEmodel))
 *
 * with iPiano, u+ = (I + a dG)^{-1}(u - a grad F(u) + b (u - u_prev))
 * (Sec. II-C, eq. (fplusg)), for three data terms:
 *   FOE_MODEL_COMBINED  eq. (newmodel), w = log u:
 *                       G(w) = sum_p lam1/2 (2w + f^2 e^{-2w}) + lam2/2 (e^{2w} - 2 f^2 w)
 *   FOE_MODEL_LOG       eq. (original): COMBINED with lam2 = 0
 *   FOE_MODEL_IDIV      eq. (variant), in u: G(u) = lam1/2 sum_p (u^2 - 2 f^2 log u)
 * grad_w F = sum_i theta_i W K_i^T rho'(K_i e^w), W = diag(e^w) for the log models and
 * grad_u F = sum_i theta_i K_i^T rho'(K_i u) for IDIV (Sec. II-C).  The prox of the log
 * models is solved by Newton's method (Sec. II-C, eq. (subproblem)); IDIV uses the
 * closed form printed in Sec. II-C.
 *
 * Conventions
 *   - Images are row-major float32 planes of height x width, pitch = width, in
 *     device memory (d_ prefix) owned by the caller.  Host arrays have no prefix.
 *   - K_i is a true 2-D convolution with a 7x7 filter (centre tap (3,3)) of the image
 *     extended by 3 pixels with the boundary map (SYMMETRIC = half-sample reflection,
 *     ZERO, PERIODIC); K_i^T is its exact adjoint.
 *   - Every call returns a foe_status; nothing throws across the ABI; out-parameters
 *     are left untouched on error.  foe_last_error() describes the last failure of
 *     the calling thread.
 *   - Work is enqueued on the solver's HIP stream.  Calls that return host values
 *     (solve, eval_energy, step) synchronise that stream before returning.
 *   - A solver allocates all of its device scratch in foe_create; no other call
 *     allocates.  A solver must not be used from two host threads at once.
 */
#ifndef FOE_H
#define FOE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FOE_ABI_VERSION 2
#define FOE_MAX_FILTERS 64
#define FOE_KSIZE 7
#define FOE_STATS_COLS 8

typedef enum foe_status {
  FOE_OK = 0,
  FOE_EINVAL = 1,       /* invalid argument or parameter (checked on the host) */
  FOE_ENOMEM = 2,       /* device allocation failed */
  FOE_EDEVICE = 3,      /* HIP runtime error */
  FOE_ELINESEARCH = 4,  /* backtracking exceeded max_backtracks; state = last accepted iterate */
  FOE_ENONFINITE = 5,   /* a reduction produced NaN/Inf */
  FOE_EINPUT = 6        /* f (or the init image) has a non-finite or non-positive pixel */
} foe_status;

typedef enum foe_model { FOE_MODEL_COMBINED = 0, FOE_MODEL_LOG = 1, FOE_MODEL_IDIV = 2 } foe_model;
typedef enum foe_boundary { FOE_BC_SYMMETRIC = 0, FOE_BC_ZERO = 1, FOE_BC_PERIODIC = 2 } foe_boundary;
typedef enum foe_step_mode { FOE_STEP_BACKTRACK = 0, FOE_STEP_FIXED = 1 } foe_step_mode;
typedef enum foe_precision { FOE_PREC_FP32 = 0, FOE_PREC_BF16 = 1 } foe_precision;
typedef enum foe_engine {
  FOE_ENGINE_AUTO = 0,
  FOE_ENGINE_VALU = 1,
  FOE_ENGINE_MFMA = 2,
  FOE_ENGINE_MFMA_SPLIT = 3
} foe_engine;
typedef enum foe_fusion { FOE_FUSED = 0, FOE_UNFUSED = 1 } foe_fusion;
typedef enum foe_prox { FOE_PROX_NEWTON = 0, FOE_PROX_LAMBERTW = 1 } foe_prox;

/* Solver parameters.  foe_default_params() fills every field. */
typedef struct foe_params {
  int32_t height, width;   /* >= 4 each */
  int32_t num_filters;     /* 1 .. FOE_MAX_FILTERS (the paper uses 48, Fig. 1) */
  int32_t ksize;           /* must be 7 */
  int32_t model;           /* foe_model */
  int32_t boundary;        /* foe_boundary */
  int32_t precision;       /* foe_precision: FP32 = both filter-bank contractions at FP32 accuracy; BF16 =
                              the adjoint contraction of grad F (Sec. II-C) with z and the adjoint taps
                              rounded to BF16, FP32 accumulation (the forward, F and the line search
                              keep FP32 accuracy) */
  int32_t step_mode;       /* foe_step_mode */
  int32_t looks;           /* L >= 1; selects the default (lam1, lam2) of Sec. III-B */
  int32_t max_iters;       /* iterations of foe_solve, >= 0; also the stats capacity */
  int32_t max_backtracks;  /* rejected trials allowed per iteration, >= 0 */
  int32_t newton_iters;    /* log-model prox: at most this many Newton iterations per pixel (each
                              pixel stops when converged), 1 .. 100 */
  int32_t engine;          /* foe_engine, for FP32 precision: VALU = direct convolution; MFMA = implicit
                              GEMM on FP32 matrix cores (v_mfma_f32_16x16x4f32); MFMA_SPLIT = the same
                              GEMM on FP16 matrix cores (v_mfma_f32_16x16x32_f16), each FP32 operand
                              split into an FP16 head and a scaled FP16 tail (about 22 significant bits,
                              exact products, FP32 accumulation; u scaled per tile by a power of two;
                              every |tap| < 16384, else EINVAL; a tap is carried to an absolute 2^-36,
                              so a filter whose largest |tap| is below 2^-10 loses relative accuracy);
                              AUTO = MFMA_SPLIT when every |tap| < 16384 and every nonzero filter has a
                              largest |tap| of at least 2^-10, else MFMA.  BF16 precision runs its own kernel (the split-FP16
                              forward and the adjoint bank on BF16 matrix cores): engine must be AUTO
                              and every |tap| < 16384, else EINVAL. */
  int32_t fusion;          /* foe_fusion: FUSED keeps the 48 z planes on chip; UNFUSED writes them to
                              HBM between a forward and an adjoint launch (num_filters * pixels
                              extra floats of device memory; same results up to summation order) */
  int32_t prox_method;     /* foe_prox: NEWTON solves eq. (subproblem) by safeguarded Newton (every log
                              model); LAMBERTW evaluates its closed form through the principal branch of
                              Lambert's W, the direct solver Sec. II-C mentions (LOG model only, else EINVAL) */
  double lambda1, lambda2; /* < 0 => the paper's value for `looks` (log models only) */
  double beta;             /* inertia b in [0, 1) */
  double alpha_fixed;      /* step a of FOE_STEP_FIXED, > 0 */
  double L0;               /* initial Lipschitz estimate of the backtracking mode, > 0 */
  double eta_up;           /* L <- eta_up L on a rejected trial, > 1 */
  double eta_down;         /* L <- eta_down L at the start of each iteration, in (0, 1] */
} foe_params;

/* Per-call summary. */
typedef struct foe_summary {
  int32_t iters_done;      /* accepted iterations of this call */
  int32_t total_trials;    /* trials of this call (accepted + rejected) */
  double H, F, G;          /* energies at the final iterate */
  double L, alpha;         /* last accepted Lipschitz estimate and step */
} foe_summary;

typedef struct foe_solver foe_solver;

/* Fill p with defaults: 48 filters, 7x7, COMBINED, SYMMETRIC, FP32, backtracking,
 * looks = 1, max_iters = 300, max_backtracks = 40, newton_iters = 30, lambdas from looks,
 * beta = 0.8, L0 = 1, eta_up = 2, eta_down = 1.  height/width are set to 0 (caller sets them). */
void foe_default_params(foe_params* p);

/* Create a solver.  filters_host: [num_filters][7][7] float32 row-major (k_i[a][b]);
 * weights_host: [num_filters] theta_i >= 0, finite.  Both are copied.  hip_stream may be
 * NULL (the null stream).  Allocates 8 planes of height*width floats plus O(tiles) scratch.
 * Errors: EINVAL (parameters), ENOMEM, EDEVICE. */
foe_status foe_create(const foe_params* p, const float* filters_host, const float* weights_host, void* hip_stream,
                      foe_solver** out);

foe_status foe_destroy(foe_solver* s);

/* Run max_iters iPiano iterations on the observed amplitude d_f (> 0, finite).
 * d_init (nullable): initial amplitude u^0 > 0; NULL => u^0 = f.  The iteration starts at
 * x^0 = x^{-1} = log u^0 (log models) or u^0 (IDIV).  d_u_out receives the amplitude
 * u = e^{x^N} (log models) or x^N.  sum_host (nullable) receives the summary; stats_host
 * (nullable, [max_iters][8] doubles) receives per accepted iteration
 *   {F(x+), G(x+), L, alpha, trials, <grad F(x), d>, |d|^2, |x - x_prev|^2}, d = x+ - x.
 * A trial whose energies are not finite is rejected by the backtracking test; in FIXED mode it
 * ends the solve with ENONFINITE.
 * Errors: ELINESEARCH / ENONFINITE (d_u_out holds the last accepted iterate), EINPUT. */
foe_status foe_solve(foe_solver* s, const float* d_f, const float* d_init, float* d_u_out, foe_summary* sum_host,
                     double* stats_host);

/* Resumable form: the iPiano state (x^n, x^{n-1}, L) lives in caller buffers d_x_cur and
 * d_x_prev (in the model's variable: w for the log models, u for IDIV) and *L_inout, and
 * is advanced by `iters` iterations in place.  Running 2 x 150 iterations gives the same
 * bits as one call of 300. */
foe_status foe_solve_from(foe_solver* s, const float* d_f, float* d_x_cur, float* d_x_prev, double* L_inout,
                          int32_t iters, foe_summary* sum_host, double* stats_host);

/* ---- Batches of images of uneven sizes (one fused launch over the tiles of all images per
 * trial, one decide block per image; per-image lambda, step size, Lipschitz estimate and
 * energies live on the device; every iteration round is replayed from HIP graphs).
 * shared: the parameters common to all images (height/width/looks/lambda fields ignored);
 * heights, widths, looks: [n]; lambda1, lambda2: [n] or NULL (=> the paper's values per looks).
 * Images are passed as packed planes: image i occupies floats [off_i, off_i + H_i W_i) with
 * off_0 = 0, off_{i+1} = off_i + H_i W_i (foe_batch_layout returns the n + 1 offsets).  The
 * handle is a foe_solver; foe_destroy releases it; foe_solve_from / foe_eval_energy accept
 * batch handles with per-image arrays (L_inout[n], F[n], G[n]). */
foe_status foe_batch_create(const foe_params* shared, int32_t n, const int32_t* heights, const int32_t* widths,
                            const double* lambda1, const double* lambda2, const int32_t* looks,
                            const float* filters_host, const float* weights_host, void* hip_stream,
                            foe_solver** out);
foe_status foe_batch_layout(foe_solver* s, int32_t* n_images, int64_t* offsets_host /* [n+1], nullable */);
/* Solve every image of the batch (max_iters iterations each).  d_init nullable (packed u^0).
 * sums_host: [n] summaries (nullable); stats_host: [n][max_iters][8] (nullable).
 * Returns the first failing image's status; the other images are still solved. */
foe_status foe_batch_solve(foe_solver* s, const float* d_f, const float* d_init, float* d_u_out,
                           foe_summary* sums_host, double* stats_host);

/* ---- Tile-shape autotuner.  Times `reps` fused trial launches of each tile configuration
 * (0: 32x32, 1: 32x16, 2: 32x8, 3: 64x8 output tiles; the BF16 engine takes 0 and 1 only,
 * foe_set_tile_config returns EINVAL for the others) on the solver's images with input d_f (packed), keeps the
 * fastest, and records it in the file named by the environment variable FOE_TUNE_CACHE
 * (when set; keyed by engine, boundary, filter count, fusion and the size bucket: the count of
 * 32 x 32 tiles of all images rounded up to a power of two, single image or batch) so later
 * solvers in the same bucket skip the timing.  *chosen receives the configuration index.
 * Results do not depend on the configuration beyond floating-point summation order. */
foe_status foe_autotune(foe_solver* s, const float* d_f, int32_t reps, int32_t* chosen);
foe_status foe_set_tile_config(foe_solver* s, int32_t cfg);

/* ---- Allocation-free solve, for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  The same solve as foe_create +
 * foe_solve + foe_destroy (same kernels, same launch order, same bits as foe_solve on the default 32 x 32
 * tiles), with every device buffer of the solver (x and gradient rings, tile list, partial sums, state,
 * stats, tap tables) placed in one static device workspace of 24 MiB that the library holds on each GPU it
 * runs on until the process ends; f is read in place.  No hipMalloc, hipFree or other allocating routine is
 * called; kernels are launched directly (no graphs).  Arguments as foe_create (p, filters_host,
 * weights_host, hip_stream) and foe_solve (d_f, d_init, d_u_out, sum_host, stats_host [max_iters][8]).
 * Run it with the device of hip_stream current.  Every call on a GPU shares that GPU's workspace: calls that
 * overlap on one GPU (two host threads, or two streams) race and must not be issued.  Nothing in the
 * workspace needs clearing between calls: each call writes every buffer before reading it.
 * Errors: EINVAL (parameters, UNFUSED fusion, or an image / max_iters whose buffers exceed the workspace:
 * about 1.2 M pixels at 300 iterations), EDEVICE, and the solve statuses of foe_solve. */
foe_status foe_solve_noalloc(const foe_params* p, const float* filters_host, const float* weights_host,
                             void* hip_stream, const float* d_f, const float* d_init, float* d_u_out,
                             foe_summary* sum_host, double* stats_host);

/* Probes running the same kernels as the solve path. */
/* d_grad = grad F(d_x). */
foe_status foe_eval_gradient(foe_solver* s, const float* d_x, float* d_grad);
/* F(d_x) and G(d_x; d_f) in double. */
foe_status foe_eval_energy(foe_solver* s, const float* d_x, const float* d_f, double* F, double* G);
/* d_out = prox_{tau G}(d_xhat) pixelwise (log models: the safeguarded Newton of the solve path). */
foe_status foe_eval_prox(foe_solver* s, const float* d_xhat, const float* d_f, double tau, float* d_out);
/* One trial step at a forced Lipschitz estimate L_forced (alpha = 1.9 (1 - beta) / L_forced, or
 * alpha_fixed in FIXED mode): d_xnext = prox(x - alpha grad F(x) + beta (x - xprev));
 * info_host (nullable, 4 doubles) = {F(x+), G(x+), <grad F(x), d>, |d|^2}. */
foe_status foe_step(foe_solver* s, const float* d_f, const float* d_x, const float* d_xprev, double L_forced,
                    float* d_xnext, double* info_host);

/* Per-image latency of the last foe_solve / foe_solve_from / foe_batch_solve, from device timestamps:
 * ms_host[i] (caller array of n_images doubles) = time from the start of the iterations (the decision on
 * the gradient at x^0) to the decision that completed image i (its last accepted trial; taken at the
 * start of the next launch, so within one launch of the image's last write), in milliseconds of the
 * device's wall clock; -1 for an image that did not complete.  Images of a batch that finish early stop
 * computing while the others continue, so the latencies differ per image.  Errors: EINVAL, EDEVICE. */
foe_status foe_batch_latency(foe_solver* s, double* ms_host);

/* Parameters of the real-SAR experiment (Sec. III-C: an L = 5 image, lambda1 = 50, lambda2 = 0.15), on
 * top of foe_default_params (the looks table would give the interpolated 406, 0.0128 for L = 5);
 * height and width are 0 (the caller sets them).  Errors: EINVAL (p NULL). */
foe_status foe_real_sar_params(foe_params* p);

/* Kernel time of the last foe_solve / foe_solve_from in milliseconds (HIP events on the
 * solver stream around the iteration loop), and the number of fused trial launches. */
foe_status foe_last_timing(foe_solver* s, double* ms, int32_t* trial_launches);

/* Measurement probe: launch the fused trial kernel `reps` times on the solver stream at the
 * state left by the last solve (the same trial is recomputed; nothing is accepted), each
 * launch bracketed by its own pair of HIP events; *ms_mean receives the mean per-launch
 * duration in milliseconds.  Requires a previous foe_solve / foe_solve_from. */
foe_status foe_profile_trial(foe_solver* s, int32_t reps, double* ms_mean);

/* ---- Warm-start network (an initialiser for the solve, outside the paper's method).
 * w0 = log f + net(log f - 4.5): six 3x3 convolutions with zero "same" padding
 * (1 -> 32, four times 32 -> 32, 32 -> 1), ReLU after the first five; the solve then starts
 * from u0 = e^{w0} (foe_solve's d_init).  Parameters: per layer the weights
 * W[co][ci][3][3] followed by the biases b[co], layers in order, foe_cnn_num_params() floats
 * in total.  The handle keeps FP32 master parameters and their BF16 rounding; every
 * convolution uses the BF16-rounded values with FP32 activations and accumulation (the four
 * 32 -> 32 layers, forward, backward-data and backward-weight, on the BF16 matrix cores with every
 * FP32 activation or gradient split into three BF16 parts: FP32 accuracy).
 * Batches are n images of one size H x W (H W < 2^25), packed [n][H][W] in device memory.
 * Activation workspace (13 planes of 32 n H W floats at most) is allocated on the first call of a
 * larger size and kept.  Calls synchronise the handle's stream before returning.
 * Errors: EINVAL (NULL or non-positive sizes, H W >= 2^25), ENOMEM, EDEVICE. */
typedef struct foe_cnn foe_cnn;
int64_t foe_cnn_num_params(void);
/* params_host: foe_cnn_num_params() floats, copied; Adam moments start at zero. */
foe_status foe_cnn_create(const float* params_host, void* hip_stream, foe_cnn** out);
foe_status foe_cnn_destroy(foe_cnn* c);
/* Copies of the FP32 master parameters and of their BF16 rounding (each nullable). */
foe_status foe_cnn_get_params(foe_cnn* c, float* master_host, float* bf16_host);
/* d_u0 = e^{w0} for a batch d_f (> 0). */
foe_status foe_cnn_infer(foe_cnn* c, const float* d_f, int32_t n, int32_t H, int32_t W, float* d_u0);
/* loss = mean over the batch of (w0 - log u_t)^2 (double, nullable) and its gradient with
 * respect to the BF16 parameters, copied to grad_host (nullable, parameter layout).  The
 * weight gradients are reduced in a fixed order: the result is deterministic. */
foe_status foe_cnn_loss_grad(foe_cnn* c, const float* d_f, const float* d_target_u, int32_t n, int32_t H, int32_t W,
                             double* loss, float* grad_host);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr > 0) on the loss of the
 * batch; the loss before the step goes to *loss (nullable). */
foe_status foe_cnn_train_step(foe_cnn* c, const float* d_f, const float* d_target_u, int32_t n, int32_t H, int32_t W,
                              double lr, double* loss);

/* ---- Quality index (reporting; not part of the iteration).  *ssim_out = the mean SSIM of d_u
 * against d_ref (both device planes H x W, row-major) with the 11 x 11 Gaussian window of standard
 * deviation 1.5, C1 = (0.01 peak)^2, C2 = (0.03 peak)^2, over the (H - 10) x (W - 10) positions where
 * the window lies inside the image -- the SSIM index the paper reports with PSNR (Sec. III-B).  Runs on
 * hip_stream (NULL = null stream) and synchronises it; allocates and frees a small block-sum buffer.
 * Errors: EINVAL (NULL, an image smaller than 11 x 11, peak <= 0), ENOMEM, EDEVICE. */
foe_status foe_ssim(const float* d_u, const float* d_ref, int32_t H, int32_t W, double peak, void* hip_stream,
                    double* ssim_out);

const char* foe_status_str(foe_status st);
const char* foe_last_error(void);
int32_t foe_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FOE_H */
