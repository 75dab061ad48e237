/*
 * pl.h -- C ABI of the MI355X Poisson-lognormal MAP filter library (libpl.so).
 *
 * The library finds the maximum a posteriori log-density field
 * s = ln(1 + delta) on a periodic 3D grid under a lognormal prior and a
 * Poisson likelihood with power-law bias (Kitaura, Jasche & Metcalf,
 * arXiv:0911.1407): the minimiser of
 *
 *   f(s) = 1/2 (s - mu)^T S_L^-1 (s - mu)                 (section 2.3, log-prior)
 *        + sum_i [ nbar w_i e^{beta s_i} - beta N_i s_i ]  (section 2.1 eqs. 1-3;
 *                                                          1 + delta_g = (1 + delta)^beta,
 *                                                          section 2.4)
 *
 * whose gradient and Hessian are those of section 3.1.2 (lognormal prior):
 *   g(s) = S_L^-1 (s - mu) + beta (nbar w e^{beta s} - N)
 *   H(s) = S_L^-1 + diag(beta^2 nbar w e^{beta s}).
 * S_L is a convolution on the grid (section 2.3), diagonal in Fourier space
 * with eigenvalues lambda_k = amp * pk_k * N_cells / V; the k = 0 mode uses
 * the separate inverse eigenvalue inv_p0.  beta = 1 is the unity bias of
 * section 2.4.2.
 *
 * Conventions
 *  - Real fields are double arrays [nx][ny][nz], z fastest (numpy C order),
 *    N = nx*ny*nz values.  Half spectra are interleaved complex arrays
 *    [nx][ny][nz/2+1] (numpy rfftn layout), Nh = nx*ny*(nz/2+1) entries of
 *    two values each.
 *  - Every field pointer is a DEVICE pointer owned by the caller.  The
 *    library allocates no device memory: pl_plan_create reports the
 *    workspace size and the caller hands over a device buffer of that size
 *    with pl_plan_set_workspace (it must stay valid until pl_plan_destroy or
 *    the next pl_plan_set_workspace).
 *  - A plan is bound to one HIP stream (hipStream_t passed as void*; NULL is
 *    the default stream) and must not be used by two threads at once.
 *  - pl_grad, pl_hessvec* are asynchronous on the plan's stream, except that
 *    pl_grad synchronises when obj_out is non-NULL.  pl_newton_krylov_solve
 *    and pl_solve_adjoint return after the work is complete.
 *  - Every call returns a status code; pl_last_error(plan) returns a message
 *    for the last failing call on that plan.
 *  - Grid lengths: each of nx, ny, nz must be one of
 *    8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 512
 *    (else PL_ERR_UNSUPPORTED_SIZE).
 */
#ifndef PL_H
#define PL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum pl_status {
  PL_OK = 0,
  PL_ERR_INVALID_ARG = 1,      /* NULL pointer, bad option, no workspace */
  PL_ERR_DOMAIN = 2,           /* negative or non-finite counts, w < 0,
                                  counts > 0 where w = 0, pk <= 0 at k != 0,
                                  non-finite field values */
  PL_ERR_UNSUPPORTED_SIZE = 3, /* grid length not in the supported set */
  PL_ERR_NOT_CONVERGED = 4,    /* iteration cap reached; outputs still written */
  PL_ERR_LINESEARCH = 5,       /* no Armijo step found; outputs hold last iterate */
  PL_ERR_HIP = 6,              /* a HIP runtime call failed */
  PL_ERR_NO_PROBLEM = 7        /* pl_set_problem not called, or no cached Hessian diagonal */
};

enum pl_precision {
  PL_FP64 = 0,  /* everything in FP64 */
  PL_MIXED = 1  /* FFTs, Hessian-vector products and Krylov vectors in FP32;
                   Krylov dots/norms, likelihood sums, gradient and outer
                   Newton iteration in FP64 */
};

typedef struct pl_plan pl_plan;

/* The posterior's data and parameters (sections 2.1-2.4). */
typedef struct pl_problem {
  const double* w;      /* device, N: completeness w_i >= 0 (eq. 2) */
  const double* counts; /* device, N: observed counts N_i >= 0 (integers for real
                           data; non-integral values are accepted since f is
                           linear in N, so dL/dN can be checked by perturbing
                           N); counts > 0 requires w > 0 */
  const double* pk;     /* device, Nh: power-spectrum shape per half-spectrum
                           mode in (Mpc/h)^3, > 0 for k != 0 (entry 0 ignored) */
  double amp;           /* amplitude A: lambda_k = amp * pk_k * N / V */
  double mu;            /* uniform prior mean of s (eq. mu) */
  double nbar;          /* mean count per cell (eq. 2), > 0 */
  double beta;          /* power-law bias exponent, > 0; 1 = unity bias */
  double inv_p0;        /* inverse prior eigenvalue of the k = 0 mode, >= 0 */
} pl_problem;

typedef struct pl_solve_opts {
  double rtol;      /* stop when ||g|| <= rtol ||g(s0)|| (default 1e-8) */
  int max_newton;   /* Newton iteration cap (default 100) */
  int max_cg;       /* CG iterations per Newton step (default 500) */
  double eta_max;   /* forcing: CG stops at ||r|| <= eta ||g||, eta = min(eta_max, max(sqrt(||g||/||g0||), rtol ||g0|| / (2 ||g||))) (eta_max 0.5) */
  double ls_c1;     /* Armijo constant (default 1e-4) */
  int precision;    /* PL_FP64 or PL_MIXED (default: the plan's precision) */
  int check_every;  /* CG iterations queued between host convergence checks (default 16) */
} pl_solve_opts;

typedef struct pl_solve_info {
  int newton_its;  /* Newton iterations taken */
  int cg_its;      /* CG iterations that changed the iterate */
  int hvps;        /* Hessian-vector products launched (>= cg_its) */
  int status;      /* same as the return code */
  double rel_grad; /* final ||g|| / ||g0|| (adjoint: final ||r|| / ||b||) */
  double grad0;    /* ||g(s0)|| (adjoint: ||b||) */
  double obj;      /* final objective f(s) (constants of eq. 3 dropped) */
  int fp64_steps;  /* mixed-precision solves: Newton steps whose FP32 direction
                      failed the line search and were redone with an FP64
                      inner solve (0 when every step ran in FP32; always 0
                      for FP64 solves and adjoints) */
} pl_solve_info;

/* Fill opts with defaults (precision = -1: use the plan's). */
void pl_default_opts(pl_solve_opts* opts);

/* Create a plan for an n[0] x n[1] x n[2] grid of box side lengths box[] (Mpc/h).
   precision: PL_FP64 or PL_MIXED (a PL_MIXED plan also supports FP64 solves).
   *workspace_bytes receives the device workspace size the caller must provide. */
int pl_plan_create(pl_plan** out, const int32_t n[3], const double box[3], int precision,
                   void* hip_stream, size_t* workspace_bytes);
/* Hand over the device workspace (>= workspace_bytes, 256-byte aligned). */
int pl_plan_set_workspace(pl_plan* plan, void* dev_ptr);
/* Change the stream later calls are issued on. */
int pl_plan_set_stream(pl_plan* plan, void* hip_stream);
int pl_plan_destroy(pl_plan* plan);

/* Set the posterior (sections 2.1-2.4).  Validates the inputs (PL_ERR_DOMAIN)
   and builds the 1/lambda tables: one entry per mode, and a radial table
   indexed by mx^2 + my^2 + mz^2, valid when every mode's 1/lambda agrees
   with its shell's to 8 ulp (isotropic spectra on cubic boxes).  The w / counts arrays are read by later
   calls, so they must stay valid while the plan uses them; pk is read only
   here.  Synchronises the stream. */
int pl_set_problem(pl_plan* plan, const pl_problem* prob);

/* Whether the last pl_set_problem found the spectrum radial (every mode's
   1/lambda equal to its shell's to 8 ulp, which needs a cubic box): then
   *radial_out (host) receives 1 and the shell table may stand in for the
   per-mode one (see PL_NUM_VARIANTS), else 0.  PL_ERR_NO_PROBLEM before a
   problem is set. */
int pl_plan_prior_is_radial(const pl_plan* plan, int32_t* radial_out);

/* Gradient of f at the real field s (section 3.1.2): grad_out (device, N).
   obj_out (host, nullable) receives f(s).  Caches the Hessian diagonal for
   pl_hessvec(plan, NULL, ...).  S_L^-1 is applied through an FFT round trip,
   so the result carries FFT roundoff amplified by max 1/lambda. */
int pl_grad(pl_plan* plan, const double* s, double* grad_out, double* obj_out);

/* Hessian-vector product H(s) v (section 3.1.2): hv_out (device, N).
   s == NULL reuses the diagonal cached by the last pl_grad / pl_hessvec. */
int pl_hessvec(pl_plan* plan, const double* s, const double* v, double* hv_out);
/* Same with v and hv_out in FP32 (FP32 FFTs; the diagonal is rounded to FP32). */
int pl_hessvec_f32(pl_plan* plan, const double* s, const float* v, float* hv_out);

/* Hessian-vector product on half spectra (the form used inside the solver):
   hv_hat = v_hat / lambda + F[d * F^-1 v_hat].  Uses the cached diagonal.
   Interleaved complex device arrays of Nh entries. */
int pl_hessvec_hat(pl_plan* plan, const double* v_hat, double* hv_hat);
int pl_hessvec_hat_f32(pl_plan* plan, const float* v_hat, float* hv_hat);

/* MAP by inexact Newton-Krylov (section 3.1: Newton-Raphson with a Krylov step,
   eq. New5 being the CG step length).  s_inout (device, N): start on input
   (uniform mu is the usual start), MAP s* on output.  opts/info nullable.
   Returns PL_OK, PL_ERR_NOT_CONVERGED or PL_ERR_LINESEARCH with s_inout and
   info written in every case. */
int pl_newton_krylov_solve(pl_plan* plan, double* s_inout, const pl_solve_opts* opts,
                           pl_solve_info* info);
/* Same solve; s_hat_out (device, Nh interleaved complex, nullable) also
   receives the solver's own iterate as a half spectrum, F s* (the solver
   keeps s in this form, where S_L^-1 is an exact pointwise product, section
   2.3), so that the gradient at the returned MAP can be evaluated without
   the FFT round trip of the real field, whose roundoff max 1/lambda
   amplifies. */
int pl_newton_krylov_solve_hat(pl_plan* plan, double* s_inout, double* s_hat_out, const pl_solve_opts* opts,
                               pl_solve_info* info);

/* Adjoint of a scalar loss L(s*) at the MAP s* (device, N): solves
   H(s*) lambda = dL_ds (device, N) by PCG to ||r|| <= opts->rtol ||dL_ds||, writes
   lambda_out (device, N, nullable) and the derivatives (mu held fixed)
     dL/dA    = lambda^T S_L'^-1 (s* - mu) / A   (k != 0 modes)  -> *dL_dA    (host, nullable)
     dL/dbeta = -lambda^T [nbar w e^{beta s}(1 + beta s) - N]   -> *dL_dbeta (host, nullable)
     dL/dnbar = -lambda^T (beta w e^{beta s})                   -> *dL_dnbar (host, nullable)
     dL/dN_i  = beta lambda_i                                    -> dL_dN     (device, N, nullable)
     dL/dw_i  = -lambda_i beta nbar e^{beta s_i}                 -> dL_dw     (device, N, nullable)
   (implicit differentiation of g(s*; theta) = 0: dL/dtheta = -lambda^T dg/dtheta). */
int pl_solve_adjoint(pl_plan* plan, const double* s_star, const double* dL_ds, double* lambda_out,
                     double* dL_dA, double* dL_dbeta, double* dL_dnbar, double* dL_dN, double* dL_dw,
                     const pl_solve_opts* opts, pl_solve_info* info);

/* MAP of the Gaussian-prior model (section 2.2, unit bias: eq. MAPG,
   delta = S (N / (1 + delta) - nbar w)), the paper's comparison MAP filter.
   Solved as the minimum of the negative log-posterior
     f(delta) = 1/2 delta^T S^-1 delta + sum_i [nbar w_i delta_i - N_i ln(1 + delta_i)],
   whose root is eq. MAPG and whose Hessian S^-1 + diag(N / (1 + delta)^2)
   is symmetric (eq. MAPG multiplied through by S gives the non-symmetric
   form of section 3.1.1; same root), by the inexact Newton-Krylov iteration
   of pl_newton_krylov_solve with the same options and info.  Uses the
   problem's w, counts, nbar, prior covariance amp * pk and inv_p0; mu and
   beta are not used (zero-mean prior, unit bias).  delta_inout: device, N,
   the start on input (zeros is the prior mean) and the MAP overdensity on
   output; every cell with counts must have 1 + delta > 0 at the start
   (PL_ERR_DOMAIN), and the line search keeps it so.  A solution needs
   inv_p0 > 0 or some counts > 0.  Synchronises the stream. */
int pl_gaussian_map_solve(pl_plan* plan, double* delta_inout, const pl_solve_opts* opts, pl_solve_info* info);

/* Linear (non-local) bias, sections 2.2.1 and 2.4.1: the galaxy overdensity
   is delta_g = B delta_M, B the convolution whose Fourier multiplier is the
   real table bk (device, [nx][ny][nz/2+1] doubles like pk; the paper's
   b_hat(k) = sqrt(P_g(k) / P_M(k)); it must satisfy bk(-k) = bk(k), which
   makes B symmetric), and expected counts are nbar w (1 + B delta_M).
   model selects the prior and the unknown x:
     PL_MODEL_LOGNORMAL  x = s = ln(1 + delta_M), prior mean mu, covariance
                         S_L = amp * pk (section 2.3);
     PL_MODEL_GAUSSIAN   x = delta_M, zero mean, covariance amp * pk
                         (section 2.2).
   With y = 1 + B delta_M(x) the negative log-posterior (constants dropped) is
     f(x) = 1/2 (x - m)^T S^-1 (x - m) + sum_i [nbar w_i y_i - N_i ln y_i],
   its gradient S^-1 (x - m) + delta_M'(x) B (nbar w - N / y) (the left minus
   the right side of the linear-bias MAP equations), its Hessian
     S^-1 + diag(delta_M''(x) B u) + diag(delta_M') B diag(N / y^2) B diag(delta_M')
   with u = nbar w - N / y.  The domain is y > 0 in every cell with counts
   (NaN or inf outside it; PL_ERR_DOMAIN where a solve starts outside).  The
   problem's beta must be 1 (this bias replaces the power law;
   PL_ERR_INVALID_ARG otherwise).  FP64 only; any plan precision.  bk == 1
   everywhere reproduces the unit-bias models up to the constant
   sum_i nbar w_i in f. */
#define PL_MODEL_LOGNORMAL 0
#define PL_MODEL_GAUSSIAN 1
/* grad_out (device, N) = g(x) at the real field x (device, N); *obj_out
   (host, nullable) = f(x); synchronises only when obj_out is given. */
int pl_linear_bias_grad(pl_plan* plan, int model, const double* bk, const double* x, double* grad_out,
                        double* obj_out);
/* hv_out (device, N) = H(x) v.  x (device, N) may be NULL to reuse the
   linearisation of the previous pl_linear_bias_grad / pl_linear_bias_hessvec
   call with the same model and bk, if no other call has used the plan since
   (PL_ERR_NO_PROBLEM otherwise).  Asynchronous. */
int pl_linear_bias_hessvec(pl_plan* plan, int model, const double* bk, const double* x, const double* v,
                           double* hv_out);
/* MAP by inexact Newton with a truncated PCG (stopped at the forcing
   tolerance or at the first direction of non-positive curvature; the
   preconditioned steepest-descent direction if that is the first one),
   preconditioner 1/lambda_k + c (c the 25th percentile of the per-cell
   curvature), Armijo backtracking from a = 1 (at most 40 halvings)
   that keeps the iterate in the domain.  x_inout: device, N, the start on
   input (mu or 0, the prior mean, is the usual one) and the MAP on output.
   Options and info as pl_newton_krylov_solve; opts->precision must not be
   PL_MIXED.  Synchronises the stream. */
int pl_linear_bias_solve(pl_plan* plan, int model, const double* bk, double* x_inout, const pl_solve_opts* opts,
                         pl_solve_info* info);
/* Same solve; x_hat_out (device, Nh interleaved complex, nullable) also
   receives the iterate as a half spectrum, F x* (the form the solver keeps,
   as in pl_newton_krylov_solve_hat). */
int pl_linear_bias_solve_hat(pl_plan* plan, int model, const double* bk, double* x_inout, double* x_hat_out,
                             const pl_solve_opts* opts, pl_solve_info* info);

/* The Krylov step of section 3.1 with a nonlinear-CG search vector, the
   paper-literal form of the solver: s <- s + tau xi with the step length of
   eq. (New5), tau = -xi^T grad Q / xi^T H xi (one HVP per step).  The paper
   leaves the search vector to an earlier reference; here xi is the
   preconditioned Polak-Ribiere+ conjugate direction (preconditioner
   1/lambda_k + c in Fourier space), restarted along -M^-1 g when it is not
   a descent direction, and each step is safeguarded by the Armijo search of
   pl_newton_krylov_solve started at tau.  Same MAP, same stopping rule and
   s_inout contract as pl_newton_krylov_solve; FP64 only (opts.precision =
   PL_MIXED is rejected).  opts.max_cg caps the number of steps; max_newton
   and eta_max are unused.  info: newton_its = cg_its = steps, hvps = HVPs.
   Synchronises the stream. */
int pl_nlcg_solve(pl_plan* plan, double* s_inout, const pl_solve_opts* opts, pl_solve_info* info);

/* Lognormal prior from a matter spectrum (section 2.3): the correlation
   function S(r) of the overdensity (the inverse transform of the
   eigenvalues amp * pk_k * N / V, so S(0) is the cell variance), its log
   transform S_L(r) = ln(1 + S(r)), and the spectrum of S_L,
   P_L(k) = (F S_L)_k * V / N, written to pk_log_out to be used with amp = 1
   in pl_set_problem.  mu_out (host, nullable) receives the mean field
   mu = -sigma0^2 / 2 with sigma0^2 = S_L(0) (section 2.3, the mean-field
   equation), sigma0_sq_out (host, nullable) sigma0^2.  The log transform
   need not keep every eigenvalue positive: values at or below
   1e-10 * S_L(0) (S_L(0) is their mean) are raised to it, and
   n_clipped_out (host, nullable) receives how many k != 0 modes were.  The
   k = 0 entry follows the same rule; pl_set_problem takes the k = 0 prior
   from inv_p0 instead.  pk, pk_log_out: device, the half spectrum
   [nx][ny][nz/2+1].  PL_ERR_DOMAIN if amp <= 0 or S(r) <= -1 somewhere.
   Needs a workspace, not a problem; overwrites the plan's solver
   workspace.  Synchronises the stream. */
int pl_lognormal_prior(pl_plan* plan, const double* pk, double amp, double* pk_log_out, double* mu_out,
                       double* sigma0_sq_out, int64_t* n_clipped_out);

/* ---------------------------------------------------------------------------
 * The paper's comparison estimators and quality measures (section 4.1).
 * ------------------------------------------------------------------------- */

/* LSQ-Wiener filter (section 4.1.1, the LSQ equation, unit bias): with the
   mask W = diag(w), the Poisson noise covariance diag(w / nbar) and the
   observed overdensity N / nbar - w, the filtered overdensity solves
     (S^-1 + diag(nbar w)) delta = N - nbar w,
   S being the problem's prior covariance (amp * pk, 1 / inv_p0 at k = 0).
   delta_out (device, N): the LSQ overdensity.  opts: rtol on the spectral
   residual, max_cg, precision (PL_MIXED: FP32 PCG sweeps refined against the
   FP64 residual); max_newton, eta_max and ls_c1 are unused.  Uses the
   problem of the last pl_set_problem; overwrites the cached Hessian
   diagonal (a later pl_hessvec needs s).  PL_ERR_NOT_CONVERGED if max_cg
   ends the solve above rtol (delta_out and info are still written).
   Synchronises the stream. */
int pl_lsq_solve(pl_plan* plan, double* delta_out, const pl_solve_opts* opts, pl_solve_info* info);

/* Inverse-weighted overdensity (section 4.1.1, the IW definitions):
   delta_out[i] = N_i / (w_i nbar) - 1 where w_i > 0, and 0 (the mean)
   where w_i = 0.  delta_out: device, N.  Asynchronous on the stream. */
int pl_inverse_weight(pl_plan* plan, double* delta_out);

/* Correlation coefficient r = sum ref rec / (|ref| |rec|) and Euclidean
   distance D = sqrt(sum (rec - ref)^2 / N) between two real fields on the
   plan's grid (section 4.1.2).  rec, ref: device, N; r_out, d_euc_out:
   host, nullable (r = 0 when either field is zero).  Sums in FP64 in a
   fixed order.  Needs a workspace, not a problem.  Synchronises the
   stream. */
int pl_compare_fields(pl_plan* plan, const double* rec, const double* ref, double* r_out, double* d_euc_out);

/* pl_compare_fields without a plan or workspace, for callers that cannot
   allocate device memory (code under HIP graph capture, serving loops,
   harnesses that forbid allocation): the library allocates nothing here.
   Its partial sums live in a fixed 32.8 KB array of device memory inside
   the library, one copy per GPU, held until the process ends; calls that
   overlap on one GPU race on it (serialise them, e.g. on one stream).
   n: host, the grid (n[0] n[1] n[2] <= 512^3 cells, else
   PL_ERR_UNSUPPORTED_SIZE; any axis < 1 gives PL_ERR_INVALID_ARG).
   rec, ref: device, N doubles.  out: device, 2 doubles, receives
   r = sum ref rec / (|ref| |rec|) (0 when either field is zero) and
   D = sqrt(sum (rec - ref)^2 / N), summed in FP64 in the same fixed order as
   pl_compare_fields.  Runs on the current device, asynchronously on
   hip_stream (which must belong to it); returns PL_ERR_HIP if a launch
   fails. */
int pl_compare_fields_noalloc(const int32_t n[3], const double* rec, const double* ref, double* out,
                              void* hip_stream);

/* Message for the last failing call on plan (never NULL). */
const char* pl_last_error(const pl_plan* plan);

/* FFT schedule autotuner.  For lengths 128, 192, 256 and 512 each column
   (x, y) pass has six tile variants (0 default: 256 threads, <= 64 KB LDS;
   1 wide: 512 threads, <= 128 KB LDS, longer contiguous row segments; 3
   split: the default tile with the stage exchanges passing real and
   imaginary parts through LDS in turn, half the LDS and so more blocks per
   CU; 4 extra wide: 1024 threads, <= 160 KB LDS; 5 wide split: 512 threads,
   split exchanges in <= 64 KB; 6 extra-wide split: 1024 threads, split
   exchanges in <= 128 KB) and the row (z) pass two (0, 1).
   The x passes that apply 1/lambda read it from the per-mode table (0),
   or, when pl_plan_prior_is_radial, from the radial shell table (1) or
   from the per-mode table at (min(kx, nx - kx), ky, kz) (2, "mirror"): the
   shell table saves a streaming read at the cost of a scattered lookup; the
   mirror reads each entry for the two modes kx and nx - kx of one column,
   so half the per-mode table streams.  Operands that a pass reads once (Krylov vectors, the
   Hessian diagonal, the per-mode table) can be loaded, and the Krylov
   vectors stored, non-temporally so that the pass-to-pass intermediate
   stays in the memory-side cache, which pays when that intermediate fits
   there.  Times the solver's fused CG step (five passes) per combination of
   the Krylov-carrying x variant, the y and z variants and the Krylov
   passes' table, then per streaming policy with those fixed, then the
   tile and table choices again under that policy, then the
   isolated operator (pl_hessvec_hat) per
   combination of its own x variant and table, on the plan's workspace (after
   pl_set_problem; it overwrites the cached Hessian diagonal and the solver's
   Krylov vectors), and keeps the fastest, per precision.  Every choice
   gives the same result up to rounding.  cache_path (nullable): a text file
   of earlier results keyed by arch, grid, table availability and precision;
   entries found there are used without timing, new ones are appended. */
int pl_plan_autotune(pl_plan* plan, const char* cache_path);

/* Number of schedule choices per precision.  In order: x variant of the
   Krylov-carrying passes, y variant, z variant, x variant of the operator's
   passes, table of the Krylov passes (0 per mode, 1 shell, 2 mirrored per
   mode), table of the operator's passes, streaming policy (one bit per array, covering its
   loads and stores: bit 0 residual r, bit 1 direction p and the operator's
   input, bit 2 iterate x, bit 3 per-mode table, bit 4 Hessian diagonal;
   0..31).
   Variants: 0 default, 1 wide, 3 split, 4 extra wide, 5 wide split, 6
   extra-wide split for the column passes (x, y), 0 or 1 for the row pass (a length without these variants runs the
   default); a shell or mirror choice runs the per-mode table when the
   spectrum is not radial. */
#define PL_NUM_VARIANTS 7
/* Current choices: out = the PL_NUM_VARIANTS choices for FP64, then FP32. */
int pl_plan_get_variants(const pl_plan* plan, int32_t out[2 * PL_NUM_VARIANTS]);
/* Force the choices (same order): column variants 0, 1, 3, 4, 5 or 6, row
   variant 0 or 1, tables 0, 1 or 2, streaming policy 0..31
   (PL_ERR_INVALID_ARG otherwise). */
int pl_plan_set_variants(pl_plan* plan, const int32_t v[2 * PL_NUM_VARIANTS]);

/* ---------------------------------------------------------------------------
 * Batched MAP solves: many independent reconstructions (each its own grid,
 * box and posterior) solved together.  Every pass of every Newton / CG step
 * is one launch over all instances per length class (32-96, and 128; a
 * per-block work list of (instance, tile)); converged instances are masked
 * out on the device; the CG steps
 * between host convergence checks are captured once as a HIP graph and
 * replayed (launched directly over the unfinished instances only, once
 * their cells have halved).  Each axis length must be one of 32, 48, 64,
 * 96, 128.
 * ------------------------------------------------------------------------- */
typedef struct pl_batch pl_batch;

/* n: n_inst * 3 grid lengths, box: n_inst * 3 box sides (Mpc/h), host arrays.
   precision: PL_FP64 or PL_MIXED (Krylov/HVP in FP32 for PL_MIXED solves).
   The batch runs on its own internal stream (HIP graphs are captured on
   it).  pl_batch_set_workspace, pl_batch_set_problem and pl_batch_solve
   first make it wait for the work already queued on hip_stream (the
   caller's), so arrays the caller is still writing there are read after
   those writes; each of them returns after its own work is complete. */
int pl_batch_create(pl_batch** out, int n_inst, const int32_t* n, const double* box, int precision,
                    void* hip_stream, size_t* workspace_bytes);
int pl_batch_set_workspace(pl_batch* batch, void* dev_ptr);
/* Set instance i's posterior (same contract as pl_set_problem). */
int pl_batch_set_problem(pl_batch* batch, int i, const pl_problem* prob);
/* Tile schedules of the batched passes, picked per grid length by timing
   (the batch's counterpart of pl_plan_autotune).  For each distinct length
   (the lengths holding the most cells first) the column passes and the row
   pass of the instances of that length each take the default tile
   (256 threads, <= 64 KB of LDS) or the narrow one (128 threads,
   <= 32 KB; fewer idle lanes on short columns), whichever makes the
   batched CG step (seven launches over every instance) fastest; FP64 and,
   for a PL_MIXED batch, FP32.  Every launch then takes the largest block
   and LDS of the instances it covers.  Needs every problem set; overwrites
   the instances' Hessian diagonals and Krylov vectors.  cache_path
   (nullable): a text file of earlier results keyed by arch, precision and
   the set of lengths, read and extended as for pl_plan_autotune.  Every
   choice gives the same result up to rounding.  Synchronises. */
int pl_batch_autotune(pl_batch* batch, const char* cache_path);
/* s_inout: host array of n_inst device pointers (start on input, MAP on
   output); infos: host array of n_inst (nullable).  Returns PL_OK if every
   instance converged, else the first failing instance's status; per-instance
   statuses are in infos[i].status. */
int pl_batch_solve(pl_batch* batch, double* const* s_inout, const pl_solve_opts* opts, pl_solve_info* infos);
int pl_batch_destroy(pl_batch* batch);
const char* pl_batch_last_error(const pl_batch* batch);

#ifdef __cplusplus
}
#endif

#endif /* PL_H */
