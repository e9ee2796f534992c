/* slnk.h -- C ABI of the MI355X (gfx950) semi-Lagrangian Newton--Krylov registration path.
 *
 * Method: Mang & Biros, "A semi-Lagrangian two-level preconditioned Newton--Krylov solver for
 * constrained diffeomorphic image registration" (arXiv:1604.02153).  The library evaluates, on
 * one GPU, the reduced-space quantities of the stationary-velocity registration problem
 *     min_v  1/2 ||m(1) - m_R||^2 + beta/2 <v, A v>,   d_t m + v . grad m = 0,  m(0) = m_T
 * (section 2, eq. e:varopt:objective without the mass-source term): the objective, the reduced
 * gradient (eq. e:control-elim), the Gauss--Newton reduced Hessian matvec (eq. e:hessian-matvec
 * with the lambda terms dropped, section 3.4.1), the preconditioners P_REG (eq. e:reg-precond) and
 * P_2L (section 3.4.2, nested two-level preconditioner with a CHEB(k) coarse solve), and the
 * globalised inexact Newton--PCG solve (sections 3.4.1, 3.5).  Every transport solve is the
 * semi-Lagrangian scheme of section 3.3.2 (Heun trace, periodic cubic spline interpolation).
 *
 * Conventions shared by every entry point
 *   - Grid: periodic [0, 2 pi)^2 with n1 x n2 nodes, x_i = 2 pi i / n_i.  A scalar field is a
 *     row-major [n1][n2] array (i2 fastest); a vector field is two consecutive scalar fields
 *     ([2][n1][n2]).  n1, n2 even, each a product of 2, 3, 5, at least 8; n2 at most 2048 and n1
 *     at most 2000 (the FP64 column transforms of larger n1 would not fit a workgroup's LDS).
 *   - Element type: double when params.prec == SLNK_PREC_FP64, float when SLNK_PREC_MIXED (fields
 *     in FP32; every inner product, norm, objective and Chebyshev/Lanczos scalar in FP64).
 *     Scalar outputs (J, norms, report) are always double.
 *   - Batch: a context holds B = params.batch independent problems of the same size (items).
 *     Every field argument then holds the B items one after the other ([B][n1][n2] for a scalar
 *     field, [B][2][n1][n2] for a vector field), every host scalar output is an array of B values
 *     (item order), and every call acts on all items.  Items share no data; the result of an
 *     item does not depend on the others (the iterations run in lock step with per-item scalars
 *     and stopping tests).  B = 1 is the single-problem case.
 *   - Memory: every field pointer is a DEVICE pointer owned by the caller (e.g. a torch tensor's
 *     data pointer); the library never frees it.  The library owns its workspace, allocated in
 *     slnk_create and released in slnk_destroy.
 *   - Streams: all device work is enqueued on the stream given to slnk_create.  Calls returning
 *     host scalars (J, the report, status of a solve) synchronise that stream; the others return
 *     after enqueueing their work, except that any call may synchronise to read a scalar it needs
 *     (the maximal displacement of a linearisation, the Chebyshev bounds).
 *   - Errors: no exception crosses the ABI.  Every call returns an slnk_status; the message of
 *     the last failure is available from slnk_last_error.  A context is used by one host thread
 *     at a time.
 */
#ifndef SLNK_H
#define SLNK_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct slnk_ctx slnk_ctx;

typedef enum {
  SLNK_OK = 0,
  SLNK_EINVAL = 1,          /* invalid argument, size, or call order */
  SLNK_ENOMEM = 2,          /* device allocation failed */
  SLNK_EDEVICE = 3,         /* HIP runtime error (message in slnk_last_error) */
  SLNK_ENAN = 4,            /* non-finite value in an input or an intermediate */
  SLNK_ELINESEARCH = 5,     /* Armijo backtracking found no acceptable step */
  SLNK_ENEGCURV = 6,        /* PCG met non-positive curvature (informational in the report) */
  SLNK_EMAXIT = 7,          /* iteration limit reached (informational in the report) */
  SLNK_ECHEB_DIVERGED = 8   /* P_2L stayed indefinite after e_max was re-estimated (per item, informational) */
} slnk_status;

typedef enum { SLNK_REG_H1 = 1, SLNK_REG_H2 = 2, SLNK_REG_H3 = 3 } slnk_reg;
typedef enum { SLNK_PREC_FP64 = 0, SLNK_PREC_MIXED = 1 } slnk_prec;
typedef enum { SLNK_PC_REG = 1, SLNK_PC_2L = 2 } slnk_pc;
typedef enum { SLNK_HESS_GN = 0, SLNK_HESS_FN = 1 } slnk_hessian;
typedef enum { SLNK_PROJ_NONE = 0, SLNK_PROJ_LERAY = 1 } slnk_proj;
typedef enum { SLNK_COARSE_CHEB = 0, SLNK_COARSE_PCG = 1 } slnk_coarse_solver;
typedef enum { SLNK_TRANSPORT_SL = 0, SLNK_TRANSPORT_RK2A = 1 } slnk_transport;

/* Problem and solver parameters (section 3.5 lists the paper's settings).
 *   nt            number of SL time steps on [0, 1] (ht = 1/nt), >= 1
 *   reg           regularisation seminorm H1/H2/H3: A = -Lap, Lap^2, -Lap^3 (eq. e:diffopregv)
 *   beta          regularisation weight beta_v > 0
 *   prec          element type of every field (see above)
 *   pc            SLNK_PC_REG: PCG on H with P_REG; SLNK_PC_2L: PCG on the split system
 *                 (I + S Q S) s = -S g, S = (beta A')^{-1/2}, with P_2L; coarse grid n/2
 *   cheb_iters    k of CHEB(k) (k steps, k - 1 coarse operator applications); paper: 10
 *   lanczos_steps Lanczos steps for e_max at v = 0 (paper: about 30; 2 to 1000 with P_2L)
 *   emax_safety   e_max = emax_safety * largest Ritz value (>= 1)
 *   lanczos_seed  seed of the SplitMix64 start vector of the Lanczos iteration
 *   use_graphs    1: replay the Hessian matvec and the preconditioner from captured HIP graphs
 *                 (recorded once per context and buffer pair); 0: launch every kernel
 *   batch         number of same-size problems B held by the context, 1 <= B <= 4096
 *   sl_path       SL step kernels: 0 = fused (LDS prefilter + gather in one kernel) whenever the
 *                 displacement halo fits in LDS, else coefficient pass + global gather; the fused
 *                 tile of 16 x 16 nodes runs 16 x 32 threads on launches of at most 512 tiles and
 *                 16 x 16 above; 1 = always the coefficient pass + global gather; 2, 3 = as 0 with
 *                 16 x 16 or 16 x 32 threads per fused tile whatever the launch size (tuning
 *                 choices: all give the same interpolant up to rounding)
 *   hessian       SLNK_HESS_GN (default): the Gauss--Newton matvec, which drops every lambda term of
 *                 eq. e:hessian-matvec; SLNK_HESS_FN: the full-Newton matvec, whose incremental
 *                 adjoint carries the source div(lambda vt) (eq. e:inc-adj-slm) and whose b~ adds
 *                 lambda grad m~ (table t:computational-complexity-theoretical, FN rows).  FN keeps
 *                 lambda^0..lambda^nt of the last gradient, (6 nt + 5) more fields per item with the
 *                 SL scheme, (nt + 3) with RK2A; the coarse operator of P_2L stays Gauss--Newton
 *                 (Chebyshev needs it positive definite)
 *   proj          SLNK_PROJ_NONE (default): the compressible case, K = identity; SLNK_PROJ_LERAY:
 *                 the incompressible case (w = 0), K = the Leray projection b - grad Lap^{-1} div b
 *                 applied to b in the gradient and to b~ in every matvec (section 3.1), on both
 *                 levels of P_2L
 *   coarse_solver SLNK_COARSE_CHEB (default): P_2L inverts the coarse split operator by CHEB(k);
 *                 SLNK_COARSE_PCG: by the nested PCG(eps) solve of section 3.4.2, CG on the coarse
 *                 split operator from zero to the relative residual coarse_eps times the outer
 *                 PCG tolerance (the forcing term; 1 in slnk_precond_apply), at most 200 steps
 *   coarse_eps    eps of PCG(eps), in (0, 1); the paper uses 1e-1
 *   transport     SLNK_TRANSPORT_SL (default): the semi-Lagrangian scheme of section 3.3.2;
 *                 SLNK_TRANSPORT_RK2A: the stabilised RK2 scheme of section 3.3.1 and the appendix
 *                 "Stabilized RK2 Scheme" -- the state, adjoint, incremental state and incremental
 *                 adjoint equations in antisymmetric form with pseudospectral derivatives, Heun's
 *                 method on the nt steps, and b, b~ in their antisymmetric forms.  Conditionally
 *                 stable: nt must follow the CFL condition (the paper uses CFL 0.2).  With P_REG
 *                 (the paper's earlier solver) and either matvec: full Newton adds the incremental
 *                 adjoint's source 1/2 (div(lambda vt) + vt . grad lambda + lambda div vt) and the
 *                 antisymmetric form of lambda grad m~ to b~; sl_path is ignored */
typedef struct {
  int n1, n2, nt;
  int reg;
  double beta;
  int prec;
  int pc;
  int cheb_iters;
  int lanczos_steps;
  double emax_safety;
  unsigned long long lanczos_seed;
  int use_graphs;
  int batch;
  int sl_path;
  int hessian;
  int proj;
  int coarse_solver;
  double coarse_eps;
  int transport;
} slnk_params;

/* Newton--Krylov options (sections 3.4.1, 3.5).  Stop when ||g||_inf / ||g_0||_inf <= gtol_rel or
 * ||g||_inf <= gtol_abs (g_0: gradient at v = 0) or after max_newton iterations.  PCG runs from
 * zero with the forcing term eta_k = min(0.5, ||g_k||_2 / ||g_0||_2) for at most max_pcg steps.
 * Armijo: alpha = 1 halved at most max_halvings times until
 * J(v + alpha vt) <= J(v) + armijo_c1 * alpha * <g, vt>_L2. */
typedef struct {
  int max_newton;
  double gtol_rel;
  double gtol_abs;
  int max_pcg;
  double armijo_c1;
  int max_halvings;
} slnk_solve_opts;

#define SLNK_REPORT_MAX_ITERS 64

/* Solve report of one item.  grel[k], J[k], pcg[k] for k <= newton_iters (grel[0] = 1 for a cold
 * start).  The times are those of the whole batched call (shared by its items). */
typedef struct {
  int status;               /* slnk_status of the solve */
  int newton_iters;
  int pcg_iters;            /* total over all Newton steps */
  int matvecs;              /* fine-grid Hessian (or split operator) applications */
  int coarse_matvecs;       /* coarse-grid split operator applications inside P_2L */
  int line_search_evals;    /* objective evaluations at trial points */
  double g0_inf, g0_two;    /* norms of the gradient at v = 0 */
  double emin, emax;        /* Chebyshev bounds (P_2L) */
  double grel[SLNK_REPORT_MAX_ITERS + 1];
  double J[SLNK_REPORT_MAX_ITERS + 1];
  int pcg[SLNK_REPORT_MAX_ITERS + 1];
  double time_total_ms;
  double time_gradient_ms;  /* linearisations + adjoint solves */
  double time_pcg_ms;       /* Krylov solves including preconditioner */
  double time_precond_ms;   /* preconditioner applications */
  double time_linesearch_ms;
  double time_to_stop_ms;   /* from the call's start until this item met its stop criterion */
  int fallback;             /* 1: the given start had no smaller ||g||_inf than v = 0 and was replaced by v = 0 */
  int cheb_reestimates;     /* times a PCG solve found CHEB(k) indefinite (a step's r.z <= 0) and e_max was
                               re-estimated by Lanczos at the current coarse linearisation (section 4.2.1) */
} slnk_solve_report;

/* Default parameters / options (paper settings: CHEB(10), 30 Lanczos steps, gtol 1e-2, 1e-5). */
void slnk_default_params(slnk_params* p);
void slnk_default_opts(slnk_solve_opts* o);

/* Create a context on the current HIP device.  'hip_stream' is a hipStream_t (NULL: the null
 * stream).  Allocates the whole workspace; EINVAL on unsupported sizes, ENOMEM on failure. */
slnk_status slnk_create(const slnk_params* params, void* hip_stream, slnk_ctx** out);
void slnk_destroy(slnk_ctx* ctx);
const char* slnk_last_error(const slnk_ctx* ctx);
/* Bytes of device workspace the context owns. */
unsigned long long slnk_workspace_bytes(const slnk_ctx* ctx);

/* Set the reference m_R and template m_T ([n1][n2] each, device).  Copies them; for P_2L also
 * builds the coarse problem (spectral restriction of both images) and the Chebyshev bounds:
 * e_max from Lanczos on the coarse split operator at v = 0, e_min = min_k 1 + 1/(beta a'(k))
 * (section 3.4.2, eigenvalue estimates).  ENAN if an image holds a non-finite value. */
slnk_status slnk_set_images(slnk_ctx* ctx, const void* m_R, const void* m_T);

/* m1 = m(1) for the initial value m0 transported by the stationary velocity v (state equation,
 * eq. e:state-slm, nt SL steps).  v [2][n1][n2], m0 and m1 [n1][n2]; may be called before
 * slnk_set_images.  Does not change the linearisation point. */
slnk_status slnk_transport_state(slnk_ctx* ctx, const void* v, const void* m0, void* m1);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): slnk_transport_state without a context.  params gives
 * n1, n2, nt, prec (FP64: double fields, MIXED: float fields), batch (items in v [B][2][n1][n2],
 * m0 and m1 [B][n1][n2], device pointers the caller owns; m1 may alias m0) and sl_path; its other
 * fields are ignored.  Work goes on hip_stream (a hipStream_t, NULL: the null stream); the call
 * synchronises it once, to read the displacement bound.  It allocates nothing: its working memory
 * is one 16 MiB device array of the library (per GPU, held until the process ends: one item of
 * up to 448^2 points in FP32 or 320^2 in FP64), and sizes whose working set exceeds it return
 * SLNK_EINVAL.  Calls that overlap on one GPU (other threads or streams) share that array
 * and race; each call rewrites every part it reads.  msg (may be NULL) receives a message of at
 * most msg_len bytes when the call fails.  Results equal slnk_transport_state's up to rounding. */
slnk_status slnk_transport_state_noalloc(const slnk_params* params, void* hip_stream, const void* v, const void* m0,
                                         void* m1, char* msg, size_t msg_len);

/* J[v] of every item (eq. e:varopt:objective) into J[0..B).  Makes v the linearisation point. */
slnk_status slnk_objective(slnk_ctx* ctx, const void* v, double* J);

/* Reduced gradient g = beta A v + K int_0^1 lambda grad m dt (eq. e:control-elim) into g
 * [2][n1][n2]; J (B values, may be NULL) receives the objective.  Makes v the linearisation point of the
 * Hessian and, with P_2L, of the coarse problem. */
slnk_status slnk_gradient(slnk_ctx* ctx, const void* v, void* g, double* J);

/* Hvt = beta A vt + int_0^1 lambda~ grad m dt, the Gauss--Newton matvec (eqs. e:hessian-matvec,
 * e:inc-state-slm, e:inc-adj-slm) at the last linearisation point; with hessian = SLNK_HESS_FN
 * the full-Newton matvec beta A vt + int_0^1 (lambda~ grad m + lambda grad m~) dt.  EINVAL before
 * any slnk_gradient. */
slnk_status slnk_hessian_matvec(slnk_ctx* ctx, const void* vt, void* Hvt);

/* out = (I + S Q S) s, the split spectrally preconditioned Hessian (section 3.4.2; Q of the
 * Gauss--Newton or full-Newton matvec the parameters select, K applied) at the last
 * linearisation point (the operator P_2L preconditions). */
slnk_status slnk_split_matvec(slnk_ctx* ctx, const void* s, void* out);

/* z = P^{-1} r.  SLNK_PC_REG: P_REG^{-1} = (beta A')^{-1} (eq. e:reg-precond).  SLNK_PC_2L:
 * P_2L^{-1} r = (I - L) r + Pro C(M_c) Res r at the last linearisation point (section 3.4.2),
 * acting on the split variable, with C = CHEB_k or (coarse_solver = SLNK_COARSE_PCG) CG on M_c to
 * the relative residual coarse_eps.  EINVAL for P_2L before any slnk_gradient. */
slnk_status slnk_precond_apply(slnk_ctx* ctx, const void* r, void* z);

/* Chebyshev bounds of P_2L of every item (arrays of B; after slnk_set_images). */
slnk_status slnk_get_cheb_bounds(const slnk_ctx* ctx, double* emin, double* emax);

/* Copy an internal field of the current linearisation into 'out' (device, element type as
 * above): which = 0: m(1) [n1][n2]; 1: forward displacements [2][n1][n2] in cells;
 * 2: adjoint displacements; 3: adjoint step factor gamma [n1][n2]; 4: lambda(0) of the last
 * gradient [n1][n2]. */
slnk_status slnk_get_field(slnk_ctx* ctx, int which, void* out);

/* Chebyshev upper bounds e_max [B] (host) of a P_2L context with images set, in place of the
 * Lanczos estimate: e.g. an estimate rescaled from a solve with another beta ((e_max - 1) beta does
 * not depend on beta, section 4.2.1).  EINVAL unless every e_max > e_min is finite.  A solve that
 * finds the bound too low re-estimates it (slnk_newton_solve). */
slnk_status slnk_set_cheb_emax(slnk_ctx* ctx, const double* emax);

/* Profiling support: launch one kernel of the hot path 'reps' times back to back on the
 * context's stream between one pair of HIP events and return the elapsed time divided by reps in
 * *avg_ms (each launch covers all items).  which = 0: state SL step, 1: adjoint SL step, 2: incremental state SL step,
 * 3: incremental adjoint SL step (all at the current linearisation, fused LDS variant when the
 * halo allows), 4: Heun trace of both characteristics, 5: one spectral operator on a vector field
 * (three launches: row, column and inverse row passes), 6: spectral gradients of the state at all
 * nt + 1 time levels (three launches).  EINVAL before any slnk_gradient. */
slnk_status slnk_time_kernel(slnk_ctx* ctx, int which, int reps, double* avg_ms);

/* Globalised inexact GN--Krylov solve from the velocity in v_inout (device [B][2][n1][n2]); the
 * result overwrites it.  A nonzero start is kept only if its ||g||_inf is below that at v = 0,
 * else the item starts from v = 0 (report.fallback = 1).  opts NULL: defaults.  report (array of B, may be NULL) receives one
 * report per item.  Each item stops on its own criteria; the call returns when all have stopped.
 * A PCG solve whose step had r.z <= 0 (P_2L with CHEB(k) not positive definite: e_max below the
 * coarse operator's spectrum) re-estimates that item's e_max by Lanczos on the coarse split
 * operator at the current iterate and runs again from zero (report.cheb_reestimates).
 * An item's report.status is SLNK_OK when it met a stop criterion, SLNK_EMAXIT when max_newton
 * iterations ended it first, SLNK_ELINESEARCH when backtracking failed, SLNK_ECHEB_DIVERGED when
 * the preconditioner stayed indefinite after the re-estimate (in the last two cases its velocity
 * is its last accepted iterate).  Returns SLNK_OK when every item met a stop criterion, else the
 * status of a failed item, or SLNK_EMAXIT (informational) when the only shortfall is the Newton
 * limit. */
slnk_status slnk_newton_solve(slnk_ctx* ctx, void* v_inout, const slnk_solve_opts* opts,
                              slnk_solve_report* report);

/* ---- Learned warm start -----------------------------------------------------------------------
 * A periodic convolutional U-Net (a form added to the paper's method): input (m_R, m_T), output
 * an initial velocity v_0 [2][H][W] for the Newton--Krylov solve.  'levels' resolutions (H and W
 * divisible by 2^(levels-1), the coarsest H W a multiple of 64), base_channels C (a multiple of
 * 32) doubling per level, two 3x3 periodic convolutions + ReLU per level, 2x2 average pooling,
 * nearest upsampling with concatenated skips, a linear 3x3 output convolution.  Weights and
 * activations are BF16 on the matrix cores with FP32 sums; Adam (beta1 0.9, beta2 0.999,
 * eps 1e-8) updates FP32 master weights.  Parameters: one FP32 array of slnk_unet_param_count
 * values; layer k (encoder levels first, then decoder levels from coarse to fine, then the
 * output layer) holds W[9][cout][cin] (tap 3 (dy + 1) + (dx + 1) reads pixel (y + dy, x + dx))
 * then bias[cout], each padded to a multiple of 64 values; last come the scalar head's
 * w[2 C_top] and bias[1] (each padded to 64), C_top = base_channels 2^(levels-1).  The head reads
 * the per-channel pixel means (w[0..C_top)) and maxima (w[C_top..2 C_top)) of the coarsest
 * level's output and predicts y = log(beta (e_max - 1)) of the two-level preconditioner's
 * Chebyshev bound (the coarse-grid part of the learned form).  All arrays are device FP32 unless
 * stated; calls enqueue on the network's stream, train_step and the parameter copies synchronise
 * it.  A network is used by one host thread at a time. */
typedef struct slnk_unet slnk_unet;
typedef struct {
  int height, width;
  int levels;
  int base_channels;
  int max_batch;                 /* largest batch of any call */
  unsigned long long seed;       /* SplitMix64 seed of the He-uniform initialisation */
  int start_kmax;                /* learned solve: Fourier modes |k| <= start_kmax of the network's
                                    velocity are kept as the start (0: all); the regulariser
                                    beta A weighs the others by up to beta |k|^(2 reg) */
} slnk_unet_params;

void slnk_unet_default_params(slnk_unet_params* p);  /* 256 x 256, 4 levels, 32 channels, batch 16 */
slnk_status slnk_unet_create(const slnk_unet_params* p, void* hip_stream, slnk_unet** out);
void slnk_unet_destroy(slnk_unet* u);
const char* slnk_unet_last_error(const slnk_unet* u);
long long slnk_unet_param_count(const slnk_unet* u);
/* host FP32 arrays of slnk_unet_param_count values; set_params also resets the Adam moments */
slnk_status slnk_unet_get_params(slnk_unet* u, float* host);
slnk_status slnk_unet_set_params(slnk_unet* u, const float* host);
/* gradient of the loss of the last train_step with respect to every parameter (host FP32) */
slnk_status slnk_unet_get_grads(slnk_unet* u, float* host);
/* Diagnostic: launches of the convolution kernel's variants in this process since the last reset
 * (reset != 0 clears them after reading).  counts[3 (mw - 1) + j]: mw = 1 for output tiles of 16
 * pixels (H W an odd multiple of 64), 2 for 32 pixels; j = 0, 1, 2 for the reduction over input
 * channels split 1, 2 or 4 ways across the block's wavefronts (chosen from the number of output
 * tiles, so that a launch keeps about eight wavefronts per compute unit); counts[6], counts[7]:
 * the LDS-tiled kernel (input halo patch and weights of each 32-channel chunk staged once per
 * block) with 32 or 64 output channels per block, taken by launches of at least 512 blocks. */
void slnk_unet_conv_variants(long long counts[8], int reset);
/* v [batch][2][H][W] = network(m_R, m_T), images [batch][H][W]; head [batch] (may be NULL)
 * receives the scalar head's output */
slnk_status slnk_unet_forward(slnk_unet* u, int batch, const float* m_R, const float* m_T, float* v,
                              float* head);
/* One training step.  With v_target: mean squared error mean((v - v_target)^2) over
 * batch x 2 x H x W, backpropagated through the convolution layers.  With head_target [batch]:
 * mean (head - head_target)^2, which trains the head alone (its gradient does not reach the
 * convolution layers).  At least one target; lr > 0 applies one Adam step to the parameters
 * that received gradients.  *loss, *head_loss (may be NULL) receive the losses before the step. */
slnk_status slnk_unet_train_step(slnk_unet* u, int batch, const float* m_R, const float* m_T,
                                 const float* v_target, const float* head_target, double lr, double* loss,
                                 double* head_loss);
/* slnk_set_images with the network: copies m_R, m_T, runs the network once, and (P_2L) takes
 * e_max = 1 + 1.1 exp(head) / beta from the head instead of the Lanczos iteration (e_min as in
 * slnk_set_images).  The network's start velocity is kept for the next slnk_newton_solve_learned.
 * Mixed-precision contexts whose grid matches the network. */
slnk_status slnk_set_images_learned(slnk_ctx* ctx, slnk_unet* u, const void* m_R, const void* m_T);
/* Learned solve of a mixed-precision context whose grid matches the network: v_out (device,
 * [B][2][n1][n2]) = the modes |k| <= start_kmax of network(m_R, m_T) for every item (kept from
 * slnk_set_images_learned, else computed here), then slnk_newton_solve from there (with its
 * fallback to v = 0).  The report times include a forward pass computed here. */
slnk_status slnk_newton_solve_learned(slnk_ctx* ctx, slnk_unet* u, void* v_out, const slnk_solve_opts* opts,
                                      slnk_solve_report* report);

/* ---- Ragged batches ---------------------------------------------------------------------------
 * A batch holds npairs independent problems whose grids may differ in size.  Pairs of one size
 * form a bucket served by one batched context (as slnk_create with batch = pairs of that size) on
 * a stream of its own; the calls below run every bucket from its own host thread, so buckets
 * overlap on the GPU, and return when all buckets have finished (they synchronise).  Device work
 * is ordered after the work already enqueued on the stream given to slnk_batch_create.
 * Per-pair arguments are arrays of npairs device pointers (pair p: [n1[p]][n2[p]] for an image,
 * [2][n1[p]][n2[p]] for a vector field, element type per base->prec); host scalar outputs are
 * arrays of npairs.  Each pair's results equal those of a batch-1 context with the same
 * parameters (same sl_path).  Errors name the bucket; a batch is used by one host thread at a
 * time. */
typedef struct slnk_batch slnk_batch;

/* 'base' gives every parameter except n1, n2, batch (taken per pair).  Allocates every bucket's
 * workspace plus staging for the stacked per-bucket layout. */
slnk_status slnk_batch_create(const slnk_params* base, int npairs, const int* n1, const int* n2,
                              void* hip_stream, slnk_batch** out);
void slnk_batch_destroy(slnk_batch* b);
const char* slnk_batch_last_error(const slnk_batch* b);
/* k < 0: *count = number of buckets.  Else bucket k's size, pair count and tuned settings. */
slnk_status slnk_batch_bucket_info(const slnk_batch* b, int k, int* n1, int* n2, int* count,
                                   int* sl_path, int* use_graphs);
slnk_status slnk_batch_set_images(slnk_batch* b, const void* const* m_R, const void* const* m_T);
slnk_status slnk_batch_gradient(slnk_batch* b, const void* const* v, void* const* g, double* J);
slnk_status slnk_batch_hessian_matvec(slnk_batch* b, const void* const* vt, void* const* Hvt);
/* reports: array of npairs (may be NULL); report p's time_to_stop_ms counts from the start of
 * its bucket's solve. */
slnk_status slnk_batch_newton_solve(slnk_batch* b, void* const* v_inout, const slnk_solve_opts* opts,
                                    slnk_solve_report* reports);
/* Autotuner: for every bucket (one at a time), time 'reps' applications of the Krylov operator
 * at the current linearisation (set by slnk_batch_gradient) on the direction vt under each of
 * sl_path in {1, 2, 3} (two-kernel step; fused step with 16 x 16 or 16 x 32 threads per tile) x
 * use_graphs in {0, 1}, and keep the fastest.  best_ms (array of buckets,
 * may be NULL) receives the winning time per bucket. */
slnk_status slnk_batch_autotune(slnk_batch* b, const void* const* vt, int reps, double* best_ms);

#ifdef __cplusplus
}
#endif

#endif /* SLNK_H */
