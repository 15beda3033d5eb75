/*
 * hh.h - C ABI of libhh, an MI355X (gfx950) solver for the 2D heterogeneous
 * Helmholtz equation with a multigrid-augmented CNN preconditioner.
 *
 * Method: Lerer, Ben-Yair and Treister, "Multigrid-Augmented Deep Learning
 * Preconditioners for the Helmholtz Equation using Compact Implicit Layers"
 * (arXiv 2306.17486).  Section / equation numbers below refer to that paper.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Grid: n x n unknowns u[i][j] (i = row, j = column), row-major, spacing
 *   h = 1/n, homogeneous Dirichlet ghosts one cell outside the grid (Sec. 3.4:
 *   the zero padding of the 3x3 stencil is the Dirichlet condition).
 * - Complex single precision ("c64") is two interleaved floats (re, im);
 *   complex double ("c128") two interleaved doubles.  Batches are stored
 *   right-hand side major: element (r, i, j) at offset (r*n + i)*n + j.
 * - Pointers named *_dev are device pointers on the context's device; the
 *   caller owns them and must keep them alive until the call returns.
 *   Pointers named *_host are host memory.
 * - All device work is ordered on the context's HIP stream.  Calls that write
 *   host outputs synchronise that stream before returning; the others are
 *   asynchronous with respect to the host.
 * - Library workspaces are allocated through the context's allocator
 *   callbacks (or hipMalloc when none are given) and freed by the matching
 *   destroy call.
 * - Return value: HH_OK (0) on success, HH_NOT_CONVERGED (1) when a solve hit
 *   its iteration cap, a negative HH_ERR_* code on failure.  On failure
 *   hh_last_error() returns a thread-local description.  Nothing throws.
 */
#ifndef HH_H_
#define HH_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int hh_status;
enum {
    HH_OK = 0,
    HH_NOT_CONVERGED = 1,
    HH_ERR_ARG = -1,       /* bad argument (sizes, null pointers, unsupported n) */
    HH_ERR_HIP = -2,       /* a HIP runtime call or kernel launch failed */
    HH_ERR_NOMEM = -3,     /* the allocator returned NULL */
    HH_ERR_STATE = -4,     /* call not valid in the object's current state */
    HH_ERR_BREAKDOWN = -5  /* NaN or Inf met in a solve (outside the network: a non-finite
                              network output switches that right-hand side to MG-only) */
};

enum { HH_MAX_LEVELS = 4, HH_MAX_RESTART = 16 };

typedef struct hh_ctx hh_ctx;
typedef struct hh_model hh_model;
typedef struct hh_net hh_net;

/* Device allocator callbacks.  alloc returns a device pointer (or NULL on
 * failure) of at least `bytes` bytes, aligned to 256 bytes, usable on the
 * context's stream; free releases it.  `user` is passed through unchanged. */
typedef void* (*hh_alloc_fn)(size_t bytes, void* user);
typedef void (*hh_free_fn)(void* ptr, void* user);

/* Library version string (static storage). */
const char* hh_version(void);

/* Thread-local description of the last error returned on this thread
 * (static storage until the next failing call on the same thread). */
const char* hh_last_error(void);

/* Create a context bound to HIP device `device` and HIP stream `stream`
 * (a hipStream_t; NULL = the device's null stream).  alloc/free may both be
 * NULL (hipMalloc / hipFree are used).  *out receives the new context. */
hh_status hh_ctx_create(int device, void* stream, hh_alloc_fn alloc, hh_free_fn free_fn, void* user,
                        hh_ctx** out);
hh_status hh_ctx_destroy(hh_ctx* ctx);

/* ------------------------------------------------------------------------
 * Problem model: one or more slowness models on the same n x n grid.
 * ---------------------------------------------------------------------- */
typedef struct {
    int n;                 /* grid points per dimension; n % 4 == 0, n >= 16 */
    double omega;          /* angular frequency (eq. 1) */
    int abl_width;         /* absorbing-layer width in cells (Sec. 3.1), default 16 */
    double abl_gamma_max;  /* attenuation at the edge cell, default 1 */
    double gamma0;         /* constant global attenuation gamma of eq. 1, default 0 */
    double sl_beta;        /* shifted-Laplacian imaginary shift beta (eq. 4), default 0.5 */
    int levels;            /* multigrid levels (Sec. 3.2), default 3, 2..HH_MAX_LEVELS */
    int nu_pre, nu_post;   /* damped-Jacobi sweeps before/after the coarse correction, 1/1 */
    double jacobi_w;       /* Jacobi damping, default 0.8 */
    int coarse_reduce;     /* coarsest exact solve: 1 eliminates the odd grid rows by their
                              tridiagonal inverses first (one level of cyclic reduction) and
                              runs the two-ended block elimination on the even rows (half the
                              sequential chain, about twice the factor memory); k = 2 .. 5
                              (default 4) does the same and runs each elimination chain 2^(k-1)
                              steps at a time with precomputed multi-step factors, the skipped
                              steps following in row-parallel phases (a chain 2^(k-1) times
                              shorter for 4 (k-1) parallel phases; about 1/4 + 1/8 + ... more
                              factor memory than 1); 0 runs the two-ended elimination on all
                              grid rows */
    int coarse_iters;      /* 0 (default): the coarsest level is solved exactly (above).  k in
                              1..16: instead k steps of GMRES on the coarsest shifted operator,
                              right-preconditioned by its diagonal (Jacobi), from zero, without
                              restart -- the iterative coarsest-grid solve of Sec. 3.4; no
                              factorisation is built (the option for coarsest grids where the
                              sequential elimination is too slow, e.g. 1024 x 1024) */
} hh_model_desc;

/* Fill *d with the defaults listed above (n and omega are set to 0). */
void hh_model_desc_default(hh_model_desc* d);

/* Build the model for `ninst` slowness models kappa_dev (float32
 * [ninst][n][n], device, read during the call only).  The operator is eqs.
 * 1-3 with gamma = gamma0 + ((w - d)/w)^2 * gamma_max on cells at distance
 * d < w = abl_width from the nearest edge.  Builds every multigrid level
 * (coefficients restricted by full weighting, eq. 8) and the exact
 * block-tridiagonal factorisation of the coarsest shifted operator.
 * Synchronises the stream.  Errors: HH_ERR_ARG for unsupported sizes. */
hh_status hh_model_create(hh_ctx* ctx, const hh_model_desc* d, int ninst, const float* kappa_dev,
                          hh_model** out);
hh_status hh_model_destroy(hh_model* m);

/* ------------------------------------------------------------------------
 * Flexible GMRES solve (Saad 1993; the Krylov method of Sec. 1 and Sec. 5).
 * ---------------------------------------------------------------------- */
enum { HH_PRECOND_MG = 0, HH_PRECOND_CNN_MG = 1 };

typedef struct {
    int restart;        /* FGMRES restart length m, default 10, <= HH_MAX_RESTART */
    int max_iters;      /* cap on preconditioner applications per RHS, default 2000 */
    double rtol;        /* stop when ||b - A x|| / ||b|| <= rtol (FP64), default 1e-6 */
    int precond;        /* HH_PRECOND_MG or HH_PRECOND_CNN_MG */
    int warm_mg_iters;  /* CNN_MG only: MG-only iterations before the network (Sec. 4.1), default 3 */
    int use_x0;         /* 1: x_dev holds the initial guess; 0: start from zero */
    int fixed_iters;    /* >0: run exactly this many iterations (single cycle, no
                           convergence test); used to generate training data (eq. 20) */
    int fallback;       /* CNN_MG only, default 1: per RHS, MG-only FGMRES judges the
                           network and the network judges MG-only.  A restart cycle that
                           cuts the FP64 residual by less than probe_ratio (end / start
                           above it) is followed by one cycle with the other preconditioner;
                           that one takes over if its cycle cut the residual more, otherwise
                           the previous one resumes and the wait before the next probe
                           doubles (2, 4, 8, ... cycles; a switch resets it).  0: CNN+MG
                           in every cycle after the warm start.  Either way, a network
                           application with a non-finite result ends its cycle: that
                           cycle's directions are dropped (x keeps its last finite value;
                           the applications count as iterations) and the right-hand side
                           continues with MG-only. */
    double probe_ratio; /* default 0.5 */
    int graph;          /* 1 (default): a restart cycle's launch sequence (every kernel
                           from the first preconditioner application to the update of x)
                           depends only on the cycle length, the warm start and the
                           counts of right-hand sides on each preconditioner; the second
                           cycle with a given configuration is captured into a HIP graph
                           and every later one replays it (the first runs eagerly, so
                           that lazy set-up and coarse-solve tuning happen outside a
                           capture).  Graphs live for one call.  Cycles run eagerly while
                           kernel-class profiling is on and when the coarse solve uses a
                           cooperative (split) variant.  0: every cycle eager.  Results are
                           identical either way (same kernels in the same order). */
} hh_solve_opts;

void hh_solve_opts_default(hh_solve_opts* o);

/* Solve A x = b for `nrhs` right-hand sides.
 *   inst_host: host int[nrhs], slowness model index of each RHS (NULL = all 0)
 *   b_dev:     c64 [nrhs][n][n] right-hand sides
 *   x_dev:     c128 [nrhs][n][n] solutions (initial guess when o->use_x0)
 *   res_hist_host: optional double [nrhs][o->max_iters + 1]; entry k = relative
 *              residual estimate after k iterations (entry 0 = initial true
 *              value); entries past the last iteration are set to -1
 *   iters_host, converged_host: optional int [nrhs]
 *   final_res_host: optional double [nrhs]: ||b - A x|| / ||b|| recomputed in FP64
 *   mg_cycles_host: optional int [nrhs]: restart cycles after the warm start that a
 *              CNN_MG solve ran with MG-only (judge probes and switches)
 *   cnn_iters_host: optional int [nrhs]: iterations preconditioned by CNN+MG
 * The stencil, V-cycle and network run in single precision / BF16; the
 * Gram-Schmidt sums, the Hessenberg least-squares problem, x and the restart
 * residual are FP64.  Returns HH_NOT_CONVERGED if any RHS stopped at
 * max_iters above rtol.  Synchronises the stream. */
hh_status hh_solve(hh_ctx* ctx, hh_model* m, int nrhs, const int* inst_host, const void* b_dev,
                   void* x_dev, const hh_solve_opts* o, double* res_hist_host, int* iters_host,
                   int* converged_host, double* final_res_host, int* mg_cycles_host, int* cnn_iters_host);

/* Several slowness models of any sizes solved together (the batched
 * multi-instance solve of Sec. 5: many media, several right-hand sides
 * each): model i (its own n, one or more slowness instances) gets nrhs[i]
 * right-hand sides b_dev[i] (c64 [nrhs[i]][n_i][n_i]), solutions x_dev[i]
 * (c128) and optional RHS -> instance maps inst_host[i] (host; the array or an
 * entry may be NULL).  Each model's FGMRES runs on its own internal stream
 * (default priority); the restart cycles of all models are issued in one
 * interleaved sequence (every model's restart residual, then one wait per
 * model, then every model's cycle), so the sizes overlap on the device.
 * Every model runs the kernels a single hh_solve with the same options runs,
 * so the results are those of separate hh_solve calls.  One options struct
 * for all (fixed_iters must be 0).  The per-model output arrays
 * (iters_host[i], ... host int/double [nrhs[i]]) may be NULL as a whole or
 * per entry.  The context's stream is synchronised before the solves start
 * and the model streams before the call returns.  Returns HH_NOT_CONVERGED if
 * any RHS of any model stopped at max_iters. */
hh_status hh_solve_batch(hh_ctx* ctx, int nmodels, hh_model* const* models, const int* nrhs,
                         const int* const* inst_host, const void* const* b_dev, void* const* x_dev,
                         const hh_solve_opts* o, int* const* iters_host, int* const* converged_host,
                         double* const* final_res_host, int* const* mg_cycles_host, int* const* cnn_iters_host);

/* Autotuner of the coarsest exact solve (the two-ended block-tridiagonal
 * elimination).  Variants: the chain, one workgroup per end for every R
 * right-hand sides (code R = 1, 2, 4, 8; each Schur inverse read serves R
 * solves), and the split solve, where the rows of every Schur inverse are
 * shared by ceil(m / RS) workgroups that meet after each step (code
 * 100 RS + R, RS = 8, 16, 32; cooperative launch, offered only when every
 * workgroup can be resident).  By default the variant is tuned per model and
 * per bucket of active right-hand sides (1, 2, 3-4, 5-8, ...): on the first
 * coarse solve of a bucket every variant is timed on that call's data and the
 * fastest kept (that call synchronises the stream).
 * hh_model_set_coarse_group fixes a variant or returns to tuning (0, which
 * also forgets earlier choices); hh_model_coarse_group returns the variant in
 * use for nact active right-hand sides (0: not tuned yet, -1: bad arguments).
 * A split-solve step wait that times out makes the solve return HH_ERR_HIP. */
hh_status hh_model_set_coarse_group(hh_model* m, int R);
int hh_model_coarse_group(const hh_model* m, int nact);

/* Tile heights of the V-cycle's fused kernels (kernel 0: pre-relaxation,
 * residual and restriction; 1: prolongation, correction and post-relaxation;
 * mode 0: zero initial guess, 1: a stored fine guess, 2: the network's
 * half-resolution output), autotuned per (kernel, mode, level size, batch)
 * on the first launch outside graph capture (each height timed on the call's
 * data, the fastest kept per device for the process).  Heights give
 * bit-identical results.  down: 2, 4 or 8 coarse rows (mode 2), 4 or 8 (mode 1),
 * 4, 8 or 16 (mode 0); up: 4, 8 or 16 fine rows (mode 2), 8, 16 or 32.
 * hh_vcycle_tuned_height: the choice for a key, 0 if not tuned yet;
 * hh_vcycle_force_height: use `height` for every launch of (kernel, mode), 0 to
 * autotune again; HH_ERR_ARG for a height the kernel does not have. */
int hh_vcycle_tuned_height(int device, int kernel, int mode, int n, int nrhs);
hh_status hh_vcycle_force_height(int kernel, int mode, int height);

/* rel_host[r] = ||b_r - A x_r|| / ||b_r|| in FP64 (A of eqs. 1-3 with the
 * model's coefficients) for solutions x_dev (c128 [nrhs][n][n], e.g. those
 * hh_solve returned) and right-hand sides b_dev (c64 [nrhs][n][n]); inst_host
 * as in hh_solve.  Synchronises the stream. */
hh_status hh_residual_norms(hh_ctx* ctx, hh_model* m, int nrhs, const int* inst_host, const void* b_dev,
                            const void* x_dev, double* rel_host);

/* hh_residual_norms without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): same arguments and results, same kernels, but the
 * partial sums live in a fixed 1 MiB device array of the library (one per
 * GPU, set up by hh_ctx_create on the context's device and held until the
 * process ends) and the inst map is read on the host (one launch triple per
 * right-hand side).  Limits: nrhs <= 256 and n <= 4096, else HH_ERR_ARG.
 * Every call on a GPU shares that GPU's array: calls that overlap on one GPU
 * (other threads, other streams) race and must be serialised by the caller.
 * Calls no allocator, torch's included.  Synchronises the stream. */
hh_status hh_residual_norms_noalloc(hh_ctx* ctx, hh_model* m, int nrhs, const int* inst_host, const void* b_dev,
                                    const void* x_dev, double* rel_host);

/* ------------------------------------------------------------------------
 * Building blocks exposed for parity tests (same kernels as the solve).
 * ---------------------------------------------------------------------- */

/* y = A_l x on multigrid level l (0 = finest, size n >> l) with the damping
 * shifted by `shift` (0 = Helmholtz operator of eqs. 1-3, sl_beta = the
 * shifted Laplacian of eq. 4).  x, y: c64 [nrhs][n_l][n_l]. */
hh_status hh_apply_operator(hh_model* m, int level, double shift, int nrhs, const int* inst_host,
                            const void* x_dev, void* y_dev);

/* One shifted-Laplacian V-cycle (Alg. 1 applied recursively, direct coarsest
 * solve): x = V(b; x0).  x0_dev may be NULL (zero initial guess).
 * b, x0, x: c64 [nrhs][n][n]. */
hh_status hh_apply_vcycle(hh_model* m, int nrhs, const int* inst_host, const void* b_dev,
                          const void* x0_dev, void* x_dev);

/* ------------------------------------------------------------------------
 * Encoder-solver network with the implicit coarsest layer (Sec. 4.1-4.4,
 * Sec. 5.3).  Parameters are one flat FP32 vector, layer by layer in the order
 *   encoder  enc1_d enc1_c1 enc1_c2 enc2_d enc2_c1 enc2_c2 enc3_d enc3_c1 enc3_c2
 *   solver   s1_d s1_c1 s1_c2 s2_d s2_c1 s2_c2 s3_d s3_c1 s3_c2 s4_d s4_c1 s4_c2
 *            u3_t u3_c1 u3_c2 u2_t u2_c1 u2_c2 u1_t u1_c1 u1_c2 out
 * each as the weights then the biases; convolution weights are (cout, cin, 3,
 * 3), transposed-convolution weights (the *_t layers) (cin, cout, 3, 3); then
 * the implicit kernels K[c][3][3] as (re, im) pairs, c < ch[3]/2.  Channels
 * per level (ch) must be (16, 32, 64, 64).  *_d layers are stride-2
 * convolutions (s4_d stride 1 when n < 512), *_t stride-2 transposed
 * convolutions (u3_t stride 1 when n < 512); ReLU follows every *_c* layer.
 * ---------------------------------------------------------------------- */
/* The lightweight network (HH_ARCH_LIGHT; Sec. 4.4, Sec. 5.3), same channels:
 *   encoder  enc1_d enc1_c1 enc1_c2 enc2_d enc2_c1 enc2_c2 enc3_d enc3_c1 enc3_c2
 *   solver   s1_d s1_e s1_w s1_s s2_d s2_e s2_w s2_s s3_d s3_e s3_w s3_s
 *            s4_d s4_c1 s4_c2 u3_t u3_c1 u3_c2 u2_t u2_c1 u2_c2 u1_t u1_c1 u1_c2 out
 * *_c* are 3x3 convolutions followed by batch normalisation and softplus;
 * sK_e (1x1, c -> 6c), sK_w (depthwise 3x3 on 6c channels) and sK_s (1x1,
 * 6c -> c) form an inverted bottleneck: softplus after the first two
 * normalisations, none after the third, whose output is added to the
 * bottleneck's input (the output of sK_d).  *_d, *_t and out are as above,
 * with biases and no activation.  Parameters per layer: the weights ((cout,
 * cin, 3, 3) for convolutions, (cin, cout, 3, 3) for *_t, (cout, cin) for 1x1,
 * (cout, 3, 3) for depthwise), then for batch-normalised layers the scale,
 * shift, running mean and running variance (cout each; such layers have no
 * bias), otherwise the biases; then the implicit kernels.  Training uses the
 * batch's statistics over (sample, row, column), biased variance, eps 1e-5,
 * and a training step with lr > 0 updates the running statistics with
 * momentum 0.1 (the unbiased variance); every other use (solves, hh_net_forward, hh_eval_loss)
 * applies the running statistics, folded into the weights. */
enum { HH_ARCH_UNET = 0, HH_ARCH_LIGHT = 1 };
typedef struct {
    int ch[4];
    int explicit_coarse;  /* 0 (the implicit U-Net): the coarsest level applies the Green's
                             function of each learned kernel K_c (eqs. 16-17); 1 (the explicit
                             U-Net of Sec. 5.2, the same network without the implicit step):
                             it convolves with K_c itself, y = sum_{a,e} K_c[a][e]
                             z[i - a + 1][j - e + 1].  Same parameters and layout. */
    int arch;             /* HH_ARCH_UNET: the network above.  HH_ARCH_LIGHT: the lightweight
                             network of Sec. 4.4 / 5.3 (layer list and parameter layout below). */
} hh_net_desc;

/* Create a network; params_host (host, nparams floats) may be NULL (zeros). */
hh_status hh_net_create(hh_ctx* ctx, const hh_net_desc* d, const float* params_host, hh_net** out);
hh_status hh_net_destroy(hh_net* net);
/* Number of FP32 parameters. */
size_t hh_net_num_params(const hh_net* net);
/* Copy the FP32 master parameters to / from host memory (synchronous). */
hh_status hh_net_get_params(hh_net* net, float* host);
hh_status hh_net_set_params(hh_net* net, const float* host);
/* Binary checkpoint: the architecture and coarsest-layer kind, parameters,
 * optimizer moments (when present) and step (files without the kind load as
 * the implicit U-Net). */
hh_status hh_net_save(hh_net* net, const char* path);
hh_status hh_net_load(hh_ctx* ctx, const char* path, hh_net** out);

/* Attach a network to a model (NULL detaches).  Runs the encoder on every
 * slowness model of the model and builds the implicit layer's transformed
 * Green's functions for the model's coarsest map (eq. 17); both are redone
 * automatically when the parameters change.  The network is not owned. */
hh_status hh_model_attach_net(hh_model* m, hh_net* net);

/* Network part of the CNN+MG preconditioner (Sec. 4.1): for every r_b,
 *   e_b = s_b P(Net(r_b / rms(r_b))),  s_b = h^2 rms(r_b),
 * P the bilinear prolongation; r, e c64 [nrhs][n][n]. */
hh_status hh_net_forward(hh_model* m, int nrhs, const int* inst_host, const void* r_dev, void* e_dev);

/* One application of the CNN+MG preconditioner (Sec. 4.1), as the solve
 * applies it: z = V(v; x0) with x0 = hh_net_forward(v), the network's output
 * interpolated inside the V-cycle's first kernels.  v, z c64 [nrhs][n][n];
 * inst_host as in hh_solve.  Synchronises the stream. */
hh_status hh_apply_cnn_precond(hh_model* m, int nrhs, const int* inst_host, const void* v_dev, void* z_dev);

/* Method-generated training pairs (Sec. 4.3, eq. 20) for nb samples on the
 * model's (training) operator, sample b using slowness model b (or the single
 * model when the model holds one):
 *   b_i = A x_i,  x~_i = kiters_host[i] iterations of MG-preconditioned FGMRES from 0,
 *   e_i = x_i - x~_i,  r_i = A e_i.
 * x_dev: c64 [nb][n][n] random vectors (an input); e_dev, r_dev: c64 outputs;
 * kiters_host: host int[nb], each in 1..HH_MAX_RESTART. */
hh_status hh_gen_training_pairs(hh_ctx* ctx, hh_model* m, int nb, const void* x_dev, const int* kiters_host,
                                void* e_dev, void* r_dev);

/* One training step on B pairs (r, e) (c64 [B][n][n]), sample b on slowness
 * model b of md (md->ninst == B), n a power of two from 64 to 512: BF16 forward and backward through
 * encoder, solver and implicit layer, loss (eq. 19 as a mean over samples and grid points)
 *   L = 1/(B n^2) sum_b || P(Net(r_b / rms(r_b))) - e_b / s_b ||^2,  s_b = h^2 rms(r_b),
 * FP32 gradients (hh_net_get_grads, unclipped), then one Adam step with learning
 * rate lr (betas 0.9, 0.999, eps 1e-8; lr = 0 computes the gradients only) on the
 * gradient scaled by min(1, max_grad_norm / ||g||) (max_grad_norm = 0: no clipping).
 * *loss_out receives L before the update, *grad_norm_out (may be NULL) ||g||.
 * Synchronises the stream. */
hh_status hh_train_step(hh_ctx* ctx, hh_net* net, hh_model* md, int B, const void* r_dev, const void* e_dev, double lr,
                        double max_grad_norm, double* loss_out, double* grad_norm_out);
/* The loss L of hh_train_step (same arguments and rules) without the backward
 * pass: no gradient, parameter or optimiser state changes.  For validation. */
hh_status hh_eval_loss(hh_ctx* ctx, hh_net* net, hh_model* md, int B, const void* r_dev, const void* e_dev,
                       double* loss_out);
/* FP32 gradients of the last training step, same layout as the parameters. */
hh_status hh_net_get_grads(hh_net* net, float* host);

/* Parity-test entry points (same kernels as the network).
 * hh_conv_test: one 3x3 convolution of BF16 NHWC x [B][Hin][Win][cin] with FP32
 *   weights w_dev; mode 0 = stride 1, 1 = stride 2, 2 = transposed stride 2;
 *   flipped = 0: w is (cout, cin, 3, 3) and the layer is a convolution;
 *   flipped = 1: w is (cin, cout, 3, 3) and the layer is a transposed convolution
 *   (mode 2 or, with mode 0, the stride-1 transposed convolution);
 *   bias (FP32, may be NULL), skip (BF16, output shape, may be NULL), act
 *   (0 none, 1 ReLU, 2 softplus, after bias and skip);
 *   y_dev BF16 output, yf_dev optional FP32 output; active_host (host int[B],
 *   may be NULL = all): batch entries with 0 are skipped (their outputs are
 *   left untouched), as the solve skips converged right-hand sides.
 * hh_implicit_test: the network's coarsest layer for coarsest size nc on BF16
 *   NHWC [B][nc][nc][ch[3]]: implicit (adjoint = 1 multiplies by conj(Ghat)) or,
 *   for an explicit network, the convolution with K (adjoint = 1: its adjoint).
 * hh_wgrad_test: the weight-gradient kernel of the training pass,
 *   out[oo][ii][t] = sum over b and output pixels p of
 *   a[b][p][oo] * x[b][s*p + (t/3 - 1, t%3 - 1)][ii]   (zero outside x),
 *   a BF16 NHWC [B][Ho][Wo][ca], x BF16 NHWC [B][Hi][Wi][cx], s = 1 (mode 0,
 *   Hi = Ho) or 2 (mode 1, Hi = 2 Ho); out FP32 [ca][cx][9], overwritten.
 *   (ca, cx, mode) in {(16,16,0), (32,32,0), (64,64,0), (32,16,1), (64,32,1),
 *   (64,64,1)}, otherwise HH_ERR_ARG. */
hh_status hh_conv_test(hh_ctx* ctx, int cin, int cout, int mode, int B, int Hin, int Win, const void* x_dev,
                       const float* w_dev, int flipped, const float* bias_dev, const void* skip_dev, int act,
                       void* y_dev, float* yf_dev, const int* active_host, int variant);

/* Tile autotuning of the 3x3 convolutions (stride 1 and 2; the transposed
 * layers have one kernel).  Each layer shape has several kernel variants
 * (tile heights, staging through registers or direct to LDS; code TR or
 * 100 + TR): on the first launch of a (shape, output size, batch) on a device,
 * outside graph capture, each variant is timed on that call's data and the
 * fastest is kept for the process.  All variants give bit-identical results.
 * hh_conv_variants: the variant codes of a shape (codes may be NULL; returns
 *   their count, 0 for an unknown shape; the first is the untuned default).
 * hh_conv_tuned_variant: the choice made for a key, 0 if not tuned yet.
 * hh_conv_force_variant: use `code` for every launch of the shape (0: autotune
 *   again); HH_ERR_ARG for a code the shape does not have.
 * hh_conv_test's `variant` (0: the autotuned choice) selects one variant. */
int hh_conv_variants(int cin, int cout, int mode, int* codes, int max);
/* Fused layer pair (mode 3 of the autotuner calls, cin = cout = 16): two
 * stride-1 3x3 convolutions with ReLU, y = relu(conv(w2, relu(conv(w1, x) + b1))
 * + b2), as the network's 16-channel levels apply them at inference (Sec. 5.3).
 * Variants: 16 and 8 (rows per tile of the fused kernel, the first layer's
 * output kept in LDS) and 1 (the two layers launched separately through mid).
 * All three give bit-identical y.
 * hh_conv_pair_test: x BF16 NHWC [B][H][W][16], w1/w2 FP32 (16, 16, 3, 3),
 *   b1/b2 FP32 [16] (may be NULL), mid and y BF16 NHWC [B][H][W][16] (mid is
 *   written by variant 1 only), active_host as for hh_conv_test, variant 0:
 *   the autotuned choice.  Synchronises the stream. */
hh_status hh_conv_pair_test(hh_ctx* ctx, int B, int H, int W, const void* x_dev, const float* w1_dev,
                            const float* b1_dev, const float* w2_dev, const float* b2_dev, void* mid_dev, void* y_dev,
                            const int* active_host, int variant);
int hh_conv_tuned_variant(int device, int cin, int cout, int mode, int Hout, int Wout, int B);
hh_status hh_conv_force_variant(int cin, int cout, int mode, int code);
hh_status hh_implicit_test(hh_net* net, int nc, int B, const void* x_dev, void* y_dev, int adjoint);
/* hh_implicit_ggrad_test: the training pass's gradient of the implicit layer's
 *   transformed Green's functions (eqs. 16-17): for BF16 NHWC z and gy
 *   [B][nc][nc][2 nk] (complex channel c = channels 2c, 2c+1), out (complex128
 *   [nk][2nc][2nc], natural frequency order, overwritten) =
 *   sum_b conj(FFT(pad z_b)) FFT(pad gy_b) / (2nc)^2; 2nc in {16, 32, 64, 128}. */
hh_status hh_implicit_ggrad_test(hh_ctx* ctx, int nk, int nc, int B, const void* z_dev, const void* gy_dev,
                                 void* out_dev);
/* hh_pointwise_test: the lightweight network's 1x1 convolution (Sec. 4.4) on
 *   BF16 x [npix][cin] with FP32 weights w [cout][cin]:
 *   y[p][o] = act(sum_c w[o][c] x[p][c] + bias[o]) + res[p][o]; bias (FP32) and
 *   res (BF16 [npix][cout]) may be NULL; act 0 none, 2 softplus; y BF16, yf
 *   optional FP32.  (cin, cout) in {(16,96), (96,16), (32,192), (192,32),
 *   (64,384), (384,64)}, otherwise HH_ERR_ARG.
 * hh_depthwise_test: its depthwise 3x3 convolution (stride 1, zero padding) on
 *   BF16 NHWC x [B][H][W][C] with FP32 w [C][3][3]:
 *   y[b][i][j][c] = act(sum_{a,e} w[c][a][e] x[b][i+a-1][j+e-1][c] + bias[c]),
 *   flip = 1 uses w[c][2-a][2-e]; C in {96, 192, 384}. */
hh_status hh_pointwise_test(hh_ctx* ctx, int cin, int cout, size_t npix, const void* x_dev, const float* w_dev,
                            const float* bias_dev, const void* res_dev, int act, void* y_dev, float* yf_dev);
hh_status hh_depthwise_test(hh_ctx* ctx, int C, int B, int H, int W, const void* x_dev, const float* w_dev,
                            const float* bias_dev, int act, int flip, void* y_dev, float* yf_dev);
hh_status hh_wgrad_test(hh_ctx* ctx, int ca, int cx, int mode, int B, int Ho, int Wo, int Hi, int Wi,
                        const void* a_dev, const void* x_dev, float* out_dev);

/* ------------------------------------------------------------------------
 * Kernel timing (HIP events on the context's stream).
 * ---------------------------------------------------------------------- */
enum {
    HH_K_OPERATOR = 0,     /* operator application (test entry point) */
    HH_K_VC_DOWN = 1,      /* V-cycle: relax + residual + restriction, finest level */
    HH_K_VC_UP = 2,        /* V-cycle: prolongation + correction + relax, finest level */
    HH_K_VC_COARSE = 3,    /* V-cycle: exact coarsest solve */
    HH_K_VC_MID = 4,       /* V-cycle: down/up kernels of the intermediate levels */
    HH_K_OP_DOTS = 5,      /* FGMRES: w = A z with the Gram-Schmidt inner products */
    HH_K_ORTHO = 6,        /* FGMRES: w -= sum h v, ||w|| */
    HH_K_SMALL = 7,        /* FGMRES: reductions, Givens, least squares */
    HH_K_RESTART = 8,      /* FGMRES: x update and FP64 residual */
    HH_K_CONV = 9,         /* network: convolutions */
    HH_K_NET_OTHER = 10,   /* network: implicit layer, scaling, upsampling */
    HH_K_NUM_CLASSES = 11
};

/* Start timing every launch of kernel class `cls` on this context, or of every
 * class when cls == HH_K_NUM_CLASSES (replaces a previous selection and clears
 * its records).  Each timed launch is bracketed by two events on the stream. */
hh_status hh_profile_begin(hh_ctx* ctx, int cls);
/* Stop timing; synchronises the stream and writes, per class, the summed
 * kernel time in milliseconds (total_ms[HH_K_NUM_CLASSES]) and the number of
 * timed launches (launches[HH_K_NUM_CLASSES]). */
hh_status hh_profile_end(hh_ctx* ctx, double* total_ms, long long* launches);

#ifdef __cplusplus
}
#endif

#endif /* HH_H_ */
