// Host side of libpl.so: plans, workspace carving, problem set-up, the
// gradient / Hessian-vector pipelines, the inexact Newton-Krylov MAP solver
// and the adjoint solve.  See include/pl.h for the public contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>

#include <rocprofiler-sdk-roctx/roctx.h>
#include <string>
#include <vector>

#include "../../include/pl.h"
#define PL_OPS_KERNELS 1
#include "pl_batch_kernels.hpp"
#include "pl_passes.hpp"
#include "pl_linbias_kernels.hpp"

using namespace pl;

namespace {

// A named range for rocprofv3 --marker-trace (Newton steps, CG chunks,
// HVPs, batch rounds); free when no tool is attached.
struct Range {
  explicit Range(const char* name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

constexpr int NB_RED = 1024;  // blocks of the grid-stride reduction kernels
// relative tolerance of each FP32 sweep of a mixed-precision linear solve
constexpr double kRefineInnerRtol = 1e-3;
// eigenvalues of the lognormal prior covariance below this fraction of
// S_L(0) (their mean) are raised to it (pl_lognormal_prior)
constexpr double kPriorFloorRel = 1e-10;

struct Status {
  int code = PL_OK;
  std::string msg;
};

// Schedule choices per precision, in the order of pl_plan_get_variants.
enum VarSlot { V_XCG = 0, V_Y, V_Z, V_XOP, V_TAB_CG, V_TAB_OP, V_NT, V_COUNT };
static_assert(V_COUNT == PL_NUM_VARIANTS, "schedule slots");

// Values a schedule slot takes: column passes 0 (default tile), 1 (wide),
// 3 (split LDS exchange), 4 (extra wide); the row pass 0 or 1; tables 0 or
// 1; the streaming policy 0..NT_ALL.  (2 is the batched passes' narrow
// tile.)
bool variant_allowed(int slot, int v) {
  switch (slot) {
    case V_XCG: case V_Y: case V_XOP: return v >= 0 && v <= 6 && v != 2;
    case V_NT: return v >= 0 && v <= 31;
    case V_TAB_CG: case V_TAB_OP: return v >= 0 && v <= 2;
    default: return v == 0 || v == 1;
  }
}

}  // namespace

struct pl_plan {
  int n[3];
  double box[3];
  int precision;
  hipStream_t stream;
  long N, Nh;
  Grid g;
  size_t ws_bytes = 0;
  char* ws = nullptr;
  // spectral FP64 vectors
  cx<double>*s_hat = nullptr, *g_hat = nullptr, *x64 = nullptr, *r64 = nullptr, *p64 = nullptr, *t64 = nullptr;
  // spectral FP32 vectors (mixed precision)
  cx<float>*x32 = nullptr, *r32 = nullptr, *p32 = nullptr, *t32 = nullptr;
  // real fields
  double *s_ws = nullptr, *e = nullptr, *d = nullptr, *preal = nullptr, *rtmp = nullptr;
  float *d32 = nullptr, *preal32 = nullptr;
  // 1/lambda tables
  double *tab_mode = nullptr, *tab_rad = nullptr;
  float *tab_mode32 = nullptr, *tab_rad32 = nullptr;
  long rad_len = 0;
  int radial = 0;
  // twiddles per axis
  cx<double>* tw64[3] = {nullptr, nullptr, nullptr};
  cx<float>* tw32[3] = {nullptr, nullptr, nullptr};
  // reductions
  double* partials = nullptr;
  long partials_len = 0;
  double* scal = nullptr;
  int* flags = nullptr;
  int* hist = nullptr;       // preconditioner-constant histogram (zeroed after use)
  double* h_scal = nullptr;  // pinned host mirror of scal
  // problem
  bool has_problem = false;
  pl_problem prob{};
  bool d_valid = false;    // d holds the diagonal of the last linearisation
  bool d32_valid = false;  // d32 mirrors d
  // schedule choices per precision [FP64/FP32] (see VarSlot); the table
  // choices apply only when the radial table is valid
  int var[2][V_COUNT] = {{0, 0, 0, 0, 0, 0, 0}, {0, 0, 0, 0, 1, 1, 0}};
  // posterior model of the running solve (MODEL_*); the lognormal one
  // except inside pl_gaussian_map_solve
  int model = MODEL_LOGNORMAL;
  // the linear-bias linearisation (e, d, rtmp) is current for this model and
  // b_hat table; any other entry point clears it
  bool lb_ready = false;
  int lb_model = -1;
  const double* lb_bk = nullptr;
  std::string err;
};

namespace {

int fail(pl_plan* p, int code, const std::string& m) {
  if (p) p->err = m;
  return code;
}

#define HIPCHK(plan, expr)                                                                        \
  do {                                                                                            \
    hipError_t _e = (expr);                                                                       \
    if (_e != hipSuccess)                                                                         \
      return fail(plan, PL_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e));           \
  } while (0)

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

// Carve the workspace; with base == nullptr only computes the size.
size_t carve(pl_plan* p, char* base) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* r = base ? base + off : nullptr;
    off += align_up(bytes);
    return r;
  };
  const size_t c64 = sizeof(cx<double>) * p->Nh, c32 = sizeof(cx<float>) * p->Nh;
  const size_t r64 = sizeof(double) * p->N, r32 = sizeof(float) * p->N;
  p->s_hat = (cx<double>*)take(c64);
  p->g_hat = (cx<double>*)take(c64);
  p->x64 = (cx<double>*)take(c64);
  p->r64 = (cx<double>*)take(c64);
  p->p64 = (cx<double>*)take(c64);
  p->t64 = (cx<double>*)take(c64);
  p->s_ws = (double*)take(r64);
  p->e = (double*)take(r64);
  p->d = (double*)take(r64);
  p->preal = (double*)take(r64);
  p->rtmp = (double*)take(r64);
  p->tab_mode = (double*)take(sizeof(double) * p->Nh);
  p->rad_len = (long)(p->n[0] / 2) * (p->n[0] / 2) + (long)(p->n[1] / 2) * (p->n[1] / 2) +
               (long)(p->n[2] / 2) * (p->n[2] / 2) + 1;
  p->tab_rad = (double*)take(sizeof(double) * p->rad_len);
  for (int a = 0; a < 3; ++a) p->tw64[a] = (cx<double>*)take(sizeof(cx<double>) * p->n[a]);
  if (p->precision == PL_MIXED) {
    p->x32 = (cx<float>*)take(c32);
    p->r32 = (cx<float>*)take(c32);
    p->p32 = (cx<float>*)take(c32);
    p->t32 = (cx<float>*)take(c32);
    p->d32 = (float*)take(r32);
    p->preal32 = (float*)take(r32);
    p->tab_mode32 = (float*)take(sizeof(float) * p->Nh);
    p->tab_rad32 = (float*)take(sizeof(float) * p->rad_len);
    for (int a = 0; a < 3; ++a) p->tw32[a] = (cx<float>*)take(sizeof(cx<float>) * p->n[a]);
  }
  // partial sums: the largest block count of any reducing launch, times 4
  long maxb = NB_RED;
  {
    long ncx = (long)p->n[1] * (p->n[2] / 2 + 1);
    maxb = std::max(maxb, ncx / 8 + 1);                    // x pass, B >= 8
    maxb = std::max(maxb, (long)p->n[0] * p->n[1] / 2 + 1);  // row pass, >= 1 pair per block
  }
  p->partials_len = maxb * 4;
  // three regions: the fused CG keeps the first pass's partials while the z
  // pass writes its own, and the last pass's until the next first pass
  p->partials = (double*)take(sizeof(double) * p->partials_len * 3);
  p->scal = (double*)take(sizeof(double) * SC_COUNT);
  p->flags = (int*)take(sizeof(int) * 4);
  p->hist = (int*)take(sizeof(int) * DQ_BINS);
  return off;
}

int grid_blocks(long n) { return (int)std::min<long>(NB_RED, std::max<long>(1, (n + RED_THREADS - 1) / RED_THREADS)); }

template <typename T>
std::vector<cx<T>> make_twiddles(int n) {
  std::vector<cx<T>> tw(n);
  for (int e = 0; e < n; ++e) {
    long double ang = -2.0L * 3.141592653589793238462643383279502884L * (long double)e / (long double)n;
    tw[e] = {(T)cosl(ang), (T)sinl(ang)};
  }
  return tw;
}

// ---------------------------------------------------------------------------
// Precision-dependent views of the plan
// ---------------------------------------------------------------------------

template <typename T>
struct View;
template <>
struct View<double> {
  static cx<double>* x(pl_plan* p) { return p->x64; }
  static cx<double>* r(pl_plan* p) { return p->r64; }
  static cx<double>* pv(pl_plan* p) { return p->p64; }
  static cx<double>* t(pl_plan* p) { return p->t64; }
  static double* preal(pl_plan* p) { return p->preal; }
  // the table elementwise kernels read: the per-mode one streams, where
  // the shell table would be a scattered lookup per element
  static const double* tab(pl_plan* p) { return p->tab_mode; }
  static const double* tab(pl_plan* p, int radial) { return radial ? p->tab_rad : p->tab_mode; }
  static const cx<double>* tw(pl_plan* p, int a) { return p->tw64[a]; }
};
template <>
struct View<float> {
  static cx<float>* x(pl_plan* p) { return p->x32; }
  static cx<float>* r(pl_plan* p) { return p->r32; }
  static cx<float>* pv(pl_plan* p) { return p->p32; }
  static cx<float>* t(pl_plan* p) { return p->t32; }
  static float* preal(pl_plan* p) { return p->preal32; }
  static const float* tab(pl_plan* p) { return p->tab_mode32; }
  static const float* tab(pl_plan* p, int radial) { return radial ? p->tab_rad32 : p->tab_mode32; }
  static const cx<float>* tw(pl_plan* p, int a) { return p->tw32[a]; }
};

// ---------------------------------------------------------------------------
// Passes
// ---------------------------------------------------------------------------

// Prior mean of the running solve's field: mu (lognormal model) or 0
// (Gaussian prior on delta).
double prior_mean(const pl_plan* p) { return p->model == MODEL_GAUSSIAN ? 0.0 : p->prob.mu; }

template <typename T>
ColArgs<T> col_args(pl_plan* p, int axis, const cx<T>* in, cx<T>* out) {
  ColArgs<T> a{};
  a.n = p->n[axis];
  a.in = in;
  a.out = out;
  a.tw = View<T>::tw(p, axis);
  a.g = p->g;
  a.inv_lam = View<T>::tab(p);
  a.radial = TAB_MODE;
  a.partials = p->partials;
  a.out_scale = T(1);
  a.nt = p->var[sizeof(T) == 4 ? 1 : 0][V_NT];
  const long h = p->g.h;
  if (axis == 0) {  // x: columns = (ky, kz) pairs
    a.ncols = (int)(p->n[1] * h);
    a.row_stride = (long)p->n[1] * h;
    a.slab_stride = 0;
  } else {  // y: slabs = kx, columns = kz
    a.ncols = (int)h;
    a.row_stride = h;
    a.slab_stride = (long)p->n[1] * h;
  }
  return a;
}

template <typename T>
hipError_t run_col(pl_plan* p, int axis, bool inverse, int op, const ColArgs<T>& a, int* nb) {
  int dummy;
  const int pi = sizeof(T) == 4 ? 1 : 0;
  const bool krylov = op == COL_CG_FIRST || op == COL_CG_LAST || op == COL_CG_INIT;
  const int v = axis == 1 ? p->var[pi][V_Y] : p->var[pi][krylov ? V_XCG : V_XOP];
  const int nslabs = axis == 0 ? 1 : p->n[0];
  if (op == COL_PLAIN) return launch_col<T>(p->n[axis], inverse, op, a, nslabs, p->stream, nb ? nb : &dummy, v);
  ColArgs<T> b = a;  // the 1/lambda table this pass reads (TabKind)
  b.radial = p->radial ? p->var[pi][krylov ? V_TAB_CG : V_TAB_OP] : TAB_MODE;
  b.inv_lam = View<T>::tab(p, b.radial == TAB_SHELL);
  return launch_col<T>(p->n[axis], inverse, op, b, nslabs, p->stream, nb ? nb : &dummy, v);
}

template <typename T>
RowArgs<T> row_args(pl_plan* p) {
  RowArgs<T> a{};
  a.n = p->n[2];
  a.nunits = (int)((long)p->n[0] * p->n[1] / 2);
  a.tw = View<T>::tw(p, 2);
  a.scale = T(1.0 / (double)p->N);
  a.d = p->d;
  a.d32 = p->d32;
  a.w = p->prob.w;
  a.counts = p->prob.counts;
  a.nbar = p->prob.nbar;
  a.beta = p->prob.beta;
  a.partials = p->partials;
  a.nt = p->var[sizeof(T) == 4 ? 1 : 0][V_NT];
  a.model = p->model;
  return a;
}

template <typename T>
hipError_t run_row(pl_plan* p, int op, const RowArgs<T>& a, int* nb) {
  int dummy;
  return launch_row<T>(p->n[2], op, a, p->stream, nb ? nb : &dummy, p->var[sizeof(T) == 4 ? 1 : 0][V_Z]);
}

hipError_t finalize(pl_plan* p, int nb, int K, int kind, int dst, double scale, double aux = 0.0,
                    const double* partials = nullptr, const double* partials2 = nullptr, int nb2 = 0,
                    double scale2 = 0.0) {
  if (K < 1 || K > 4) return hipErrorInvalidValue;  // finalize_body sums at most 4 partials per block
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(FIN_THREADS), 0, p->stream, partials ? partials : p->partials, nb, K,
                     kind, dst, scale, p->scal, aux, partials2, nb2, scale2);
  return hipGetLastError();
}

hipError_t set_scalar(pl_plan* p, int idx, double v) {
  hipLaunchKernelGGL(set_scalar_kernel, dim3(1), dim3(64), 0, p->stream, p->scal, idx, v);
  return hipGetLastError();
}

int read_scalars(pl_plan* p) {
  HIPCHK(p, hipMemcpyAsync(p->h_scal, p->scal, sizeof(double) * SC_COUNT, hipMemcpyDeviceToHost, p->stream));
  HIPCHK(p, hipStreamSynchronize(p->stream));
  return PL_OK;
}

// real [N] -> half spectrum out (T precision): z r2c, y fwd, x fwd
template <typename T>
int fwd_r2c(pl_plan* p, const T* in, cx<T>* out) {
  RowArgs<T> ra = row_args<T>(p);
  ra.in_r = in;
  ra.out_c = out;
  HIPCHK(p, run_row<T>(p, ROW_R2C, ra, nullptr));
  HIPCHK(p, run_col<T>(p, 1, false, COL_PLAIN, col_args<T>(p, 1, out, out), nullptr));
  HIPCHK(p, run_col<T>(p, 0, false, COL_PLAIN, col_args<T>(p, 0, out, out), nullptr));
  return PL_OK;
}

// half spectrum in -> real out (times 1/N): x inv, y inv, z c2r.  tmp may alias in.
template <typename T>
int inv_c2r(pl_plan* p, const cx<T>* in, cx<T>* tmp, T* out) {
  HIPCHK(p, run_col<T>(p, 0, true, COL_PLAIN, col_args<T>(p, 0, in, tmp), nullptr));
  HIPCHK(p, run_col<T>(p, 1, true, COL_PLAIN, col_args<T>(p, 1, tmp, tmp), nullptr));
  RowArgs<T> ra = row_args<T>(p);
  ra.in_c = tmp;
  ra.out_r = out;
  HIPCHK(p, run_row<T>(p, ROW_C2R, ra, nullptr));
  return PL_OK;
}

// q = H p on half spectra; partial sums (p^H q, |q|^2, .) left for a finalize
// with K = 3 over *nb blocks.
template <typename T>
int hvp_hat(pl_plan* p, const cx<T>* pin, cx<T>* q, int* nb) {
  Range range("pl hvp");
  cx<T>* t = View<T>::t(p);
  HIPCHK(p, run_col<T>(p, 0, true, COL_PLAIN, col_args<T>(p, 0, pin, t), nullptr));
  HIPCHK(p, run_col<T>(p, 1, true, COL_PLAIN, col_args<T>(p, 1, t, t), nullptr));
  RowArgs<T> ra = row_args<T>(p);
  ra.in_c = t;
  ra.out_c = t;
  HIPCHK(p, run_row<T>(p, ROW_HVP, ra, nullptr));
  HIPCHK(p, run_col<T>(p, 1, false, COL_PLAIN, col_args<T>(p, 1, t, t), nullptr));
  ColArgs<T> ca = col_args<T>(p, 0, t, q);
  ca.base = pin;
  ca.k0_shift = 0.0;
  HIPCHK(p, run_col<T>(p, 0, false, COL_ADDPRIOR, ca, nb));
  return PL_OK;
}

// Gradient at the spectral iterate s_hat: g_hat, and s (real, written to
// s_out), e, d; scalars GG, PRIOR (finalized), LIK, DSUM.
// step_dir (nullable): s_out holds the real field of the previous iterate
// and s_hat has just been advanced by alpha = SC_LS_ALPHA (<= 0: not at
// all) times the direction whose real field is step_dir; then s = s_out +
// alpha step_dir in real space (equal to F^-1 s_hat up to FFT rounding of
// the direction) and the two inverse column passes are skipped.
int grad_hat(pl_plan* p, double* s_out, const double* step_dir = nullptr) {
  cx<double>* t = p->t64;
  RowArgs<double> ra = row_args<double>(p);
  if (step_dir) {
    ra.s_in = s_out;
    ra.v = step_dir;
    ra.scal = p->scal;
  } else {
    HIPCHK(p, run_col<double>(p, 0, true, COL_PLAIN, col_args<double>(p, 0, p->s_hat, t), nullptr));
    HIPCHK(p, run_col<double>(p, 1, true, COL_PLAIN, col_args<double>(p, 1, t, t), nullptr));
    ra.in_c = t;
  }
  ra.out_c = t;
  ra.s_out = s_out;
  ra.e_out = p->e;
  ra.d_out = p->d;
  int nb = 0;
  HIPCHK(p, run_row<double>(p, step_dir ? ROW_GRAD_STEP : ROW_GRAD, ra, &nb));
  HIPCHK(p, finalize(p, nb, 2, FIN_STORE, SC_LIK, 1.0));
  HIPCHK(p, run_col<double>(p, 1, false, COL_PLAIN, col_args<double>(p, 1, t, t), nullptr));
  ColArgs<double> ca = col_args<double>(p, 0, t, p->g_hat);
  ca.base = p->s_hat;
  ca.k0_shift = (double)p->N * prior_mean(p);
  HIPCHK(p, run_col<double>(p, 0, false, COL_ADDPRIOR, ca, &nb));
  HIPCHK(p, finalize(p, nb, 3, FIN_STORE, SC_GG - 1, 1.0 / (double)p->N));
  p->d_valid = true;
  p->d32_valid = false;
  return PL_OK;
}

// Preconditioner constant from the current d (device only; see dquant_*).
int set_precond_constant(pl_plan* p, const double* d = nullptr) {
  hipLaunchKernelGGL(dquant_hist_kernel, dim3(1024), dim3(RED_THREADS), 0, p->stream, d ? d : p->d, p->N, p->scal,
                     p->hist);
  HIPCHK(p, hipGetLastError());
  hipLaunchKernelGGL(dquant_select_kernel, dim3(1), dim3(DQ_SELECT_THREADS), 0, p->stream, p->hist, p->N, p->scal);
  HIPCHK(p, hipGetLastError());
  return PL_OK;
}

int ensure_d32(pl_plan* p) {
  if (p->precision != PL_MIXED) return fail(p, PL_ERR_INVALID_ARG, "FP32 path needs a PL_MIXED plan");
  if (!p->d32_valid) {
    hipLaunchKernelGGL(d_to_f32_kernel, dim3(grid_blocks(p->N)), dim3(RED_THREADS), 0, p->stream, p->d, p->d32,
                       p->N);
    HIPCHK(p, hipGetLastError());
    p->d32_valid = true;
  }
  return PL_OK;
}

// ---------------------------------------------------------------------------
// Preconditioned CG on H x = sign * rhs (spectral, T-precision vectors), with
// the vector updates fused into the Hessian-vector passes:
//   pass 1 (x, inverse):  p = M^-1 r + beta p; partial p^H Lambda^-1 p
//   passes 2-4:           y inverse, z (c2r, times d, r2c; partial sum d v^2), y forward
//   finalize:             alpha = r^H M^-1 r / (p^H Lambda^-1 p + sum d v^2)
//   pass 5 (x, forward):  r -= alpha (F[d v] + p/lambda); x += alpha p;
//                         partials r^H r, r^H M^-1 r
//   finalize:             beta, convergence
// alpha = -(xi^T grad Q)/(xi^T H xi) is the step of eq. (New5) for the
// local quadratic model; it is known before the last pass, which applies it
// to r and x without storing H p.  Iterations queued after convergence exit
// at once on the device (the passes read the done flag).
// *its receives iterations that changed x, *hvps the Hessian products run.
// ---------------------------------------------------------------------------
// CG iterations to queue after a host check found the solve still running:
// the residual fell from rr0 to rr in its iterations, so at that rate it
// needs its * ln(rr / tol2) / ln(rr0 / rr) more.  PCG speeds up as it goes
// (measured on the selection workloads: the rest took 0.25-0.65 of that
// estimate), so half of it is queued: at least 4, at most its (the residual
// norm is not monotone: a slow start must not queue a long tail of
// iterations that will be skipped).  An iteration queued past convergence
// costs about as much as one more host check.
int next_cg_chunk(const double* sc, int check_every) {
  const double its = sc[SC_ITS], rr = sc[SC_RR], rr0 = sc[SC_RR0], tol2 = sc[SC_TOL2];
  if (!(its > 0.0 && rr > tol2 && tol2 > 0.0 && rr0 > rr)) return check_every;
  const double est = its * std::log(rr / tol2) / std::log(rr0 / rr);
  const int want = (int)std::ceil(0.5 * est);
  return std::max(4, std::min(want, (int)its));
}

// With tol_rel_of_rhs == 0 (an absolute tolerance known in advance) the
// first iteration's first pass forms the initial residual itself
// (COL_CG_INIT), so no separate initialisation pass runs;
// with a tolerance relative to ||rhs|| an initialisation pass and one
// read-back of ||rhs|| come first.  first_chunk (> 0) sets how many
// iterations are queued before the first host check; later chunks are
// sized from the residual decrease so far (next_cg_chunk).
template <typename T>
int pcg(pl_plan* p, const cx<double>* rhs, double sign, double tol_abs, double tol_rel_of_rhs, int max_cg,
        int check_every, int* its, int* hvps, double* rel_res, double* rhs_norm, int first_chunk = 0) {
  cx<T>*x = View<T>::x(p), *r = View<T>::r(p), *pp = View<T>::pv(p), *t = View<T>::t(p);
  const T* tab = View<T>::tab(p);
  const double invN = 1.0 / (double)p->N;
  double* part_a = p->partials;
  double* part_b = p->partials + p->partials_len;
  const bool fused = !(tol_rel_of_rhs > 0.0);
  double rr0 = 0.0;
  if (fused) {
    hipLaunchKernelGGL(cg_start_kernel, dim3(1), dim3(64), 0, p->stream, p->scal, tol_abs * tol_abs);
    HIPCHK(p, hipGetLastError());
  } else {
    HIPCHK(p, set_scalar(p, SC_TOL2, tol_abs * tol_abs));
    hipLaunchKernelGGL((cg_init_kernel<T>), dim3(NB_RED), dim3(RED_THREADS), 0, p->stream, rhs, sign, x, r, pp, tab,
                       TAB_MODE, p->g, p->Nh, p->scal, p->partials);
    HIPCHK(p, hipGetLastError());
    HIPCHK(p, finalize(p, NB_RED, 2, FIN_CG_INIT, 0, invN));
    int rc = read_scalars(p);
    if (rc) return rc;
    rr0 = p->h_scal[SC_RR];
    double tol2 = tol_rel_of_rhs * tol_rel_of_rhs * rr0;
    HIPCHK(p, set_scalar(p, SC_TOL2, tol2));
    HIPCHK(p, set_scalar(p, SC_DONE, rr0 <= tol2 ? 1.0 : 0.0));
  }
  // Per iteration k: the first x pass (p = M^-1 r + beta p, which from k = 1
  // on also closes iteration k - 1: beta, the convergence test and the
  // bookkeeping, from the last pass's partials in part_c), y, z (with
  // p^H H p), y (whose extra workgroup finalizes alpha), the last x pass
  // (r, x and the partials of r^H r, r^H M^-1 r).  After each chunk one
  // finalize closes its last iteration for the host's check.
  double* part_c = p->partials + 2 * p->partials_len;
  int launched = 0, nb5 = 0;
  while (launched < max_cg) {
    const int want = launched == 0 ? (first_chunk > 0 ? first_chunk : check_every)
                                   : next_cg_chunk(p->h_scal, check_every);
    int chunk = std::min(want, max_cg - launched);
    Range range("pl cg chunk");
    for (int k = 0; k < chunk; ++k) {
      const int kg = launched + k;  // iterations before this one
      int nb1 = 0, nb3 = 0;
      const bool first = fused && kg == 0;
      const double* skip = p->scal + SC_DONE;
      ColArgs<T> c1 = col_args<T>(p, 0, pp, t);
      c1.cg_r = r;
      c1.scal = p->scal;
      c1.partials = part_a;
      c1.skip = skip;
      c1.cg_rhs = rhs;
      c1.cg_rhs_sign = sign;
      c1.cg_x = x;
      if (kg > 0) {
        c1.beta_part = part_c;
        c1.beta_nb = nb5;
        c1.beta_scale = invN;
        c1.cg_k = kg;
        c1.cg_max = (double)max_cg;
      }
      HIPCHK(p, run_col<T>(p, 0, true, first ? COL_CG_INIT : COL_CG_FIRST, c1, &nb1));
      ColArgs<T> c2 = col_args<T>(p, 1, t, t);
      c2.skip = skip;
      HIPCHK(p, run_col<T>(p, 1, true, COL_PLAIN, c2, nullptr));
      RowArgs<T> ra = row_args<T>(p);
      ra.in_c = t;
      ra.out_c = t;
      ra.partials = part_b;
      ra.skip = skip;
      HIPCHK(p, run_row<T>(p, ROW_HVP, ra, &nb3));
      // alpha = r^H z / p^H H p, finalized by an extra workgroup of the y
      // pass that follows (which does not need it; the last x pass does)
      ColArgs<T> c4 = col_args<T>(p, 1, t, t);
      c4.skip = skip;
      c4.fin_on = 1;
      c4.fin = FinArgs{part_b, nb3, 2, first ? FIN_CG_ALPHA_FIRST : FIN_CG_ALPHA, 0, 1.0, p->scal,
                       (double)cg_rz_slot(kg), part_a, nb1, invN};
      HIPCHK(p, run_col<T>(p, 1, false, COL_PLAIN, c4, nullptr));
      ColArgs<T> c5 = col_args<T>(p, 0, t, t);
      c5.base = pp;
      c5.cg_r = r;
      c5.cg_x = x;
      c5.scal = p->scal;
      c5.partials = part_c;
      c5.skip = skip;
      HIPCHK(p, run_col<T>(p, 0, false, COL_CG_LAST, c5, &nb5));
    }
    launched += chunk;
    HIPCHK(p, finalize(p, nb5, 2, FIN_CG_BETA_K, launched, invN, (double)max_cg, part_c));
    int rc = read_scalars(p);
    if (rc) return rc;
    if (p->h_scal[SC_DONE] != 0.0) break;
  }
  *its = (int)p->h_scal[SC_ITS];
  // Hessian products that ran: one per counted iteration, plus the partial
  // one of a breakdown (or of a fused first iteration whose residual was
  // already below the tolerance); queued iterations after convergence exit
  // at once
  *hvps = *its + ((p->h_scal[SC_DONE] == 2.0 || (fused && *its == 0)) ? 1 : 0);
  if (rel_res) *rel_res = std::sqrt(std::max(0.0, p->h_scal[SC_RR]));
  if (rhs_norm) *rhs_norm = std::sqrt(rr0);
  return PL_OK;
}

int check_ready(pl_plan* p) {
  if (!p) return PL_ERR_INVALID_ARG;
  p->lb_ready = false;
  if (!p->ws) return fail(p, PL_ERR_INVALID_ARG, "workspace not set");
  if (!p->has_problem) return fail(p, PL_ERR_NO_PROBLEM, "pl_set_problem has not been called");
  return PL_OK;
}

int check_finite(pl_plan* p, const double* x, long n, const char* what) {
  HIPCHK(p, hipMemsetAsync(p->flags, 0, sizeof(int), p->stream));
  hipLaunchKernelGGL(finite_kernel, dim3(grid_blocks(n)), dim3(RED_THREADS), 0, p->stream, x, n, p->flags);
  HIPCHK(p, hipGetLastError());
  int h = 0;
  HIPCHK(p, hipMemcpyAsync(&h, p->flags, sizeof(int), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(p, hipStreamSynchronize(p->stream));
  if (h) return fail(p, PL_ERR_DOMAIN, std::string(what) + " has non-finite values");
  return PL_OK;
}

pl_solve_opts resolve_opts(pl_plan* p, const pl_solve_opts* o) {
  pl_solve_opts r;
  pl_default_opts(&r);
  if (o) r = *o;
  if (r.precision < 0) r.precision = p->precision;
  if (r.check_every <= 0) r.check_every = 16;
  return r;
}

// Armijo backtracking along the spectral direction x from s_hat (section
// 3.1 gives the step; the globalisation is this build's reading): the
// decrease f(s + a p) - f(s) = a b + a^2 c / 2 + sum_i [e_i expm1(a beta p_i)
// - a beta N_i p_i] (b = p^T S^-1 (s - mu), c = p^T S^-1 p, p = F^-1 x) is
// tested against c1 a p^T g for a = a0, a0/2, a0/4, ... (4 per pass, at
// most 32).  *alpha = the accepted step or -1; *descent = (p^T g < 0).
// Host-driven form (the nonlinear-CG solve); the Newton solve queues the
// same test on the device (newton_step_queue / newton_step_finish).
template <typename T>
int line_search(pl_plan* p, cx<T>* x, double a_start, const pl_solve_opts& o, double* alpha, bool* descent) {
  const double invN = 1.0 / (double)p->N;
  int rc = inv_c2r<T>(p, x, View<T>::t(p), View<T>::preal(p));
  if (rc) return rc;
  hipLaunchKernelGGL((ls_dots_kernel<T>), dim3(NB_RED), dim3(RED_THREADS), 0, p->stream, x, p->s_hat, p->g_hat,
                     p->tab_mode, TAB_MODE, p->g, p->Nh, (double)p->N * prior_mean(p),
                     p->partials);
  HIPCHK(p, hipGetLastError());
  HIPCHK(p, finalize(p, NB_RED, 3, FIN_STORE, SC_LS_B, invN));
  // the first batch of trial steps does not depend on the dots: it is
  // launched before the one read-back that returns both
  auto eval_batch = [&](double a0) -> int {
    if (p->model == MODEL_GAUSSIAN)
      hipLaunchKernelGGL((ls_eval_gauss_kernel<T>), dim3(NB_RED), dim3(RED_THREADS), 0, p->stream,
                         View<T>::preal(p), p->e, p->prob.w, p->prob.counts, p->prob.nbar, a0, p->N, p->partials);
    else
      hipLaunchKernelGGL((ls_eval_kernel<T>), dim3(NB_RED), dim3(RED_THREADS), 0, p->stream, View<T>::preal(p),
                         p->e, p->prob.counts, p->prob.beta, a0, p->N, p->partials);
    HIPCHK(p, hipGetLastError());
    HIPCHK(p, finalize(p, NB_RED, 4, FIN_STORE, SC_DF, 1.0));
    return read_scalars(p);
  };
  rc = eval_batch(a_start);
  if (rc) return rc;
  const double b = p->h_scal[SC_LS_B], c = p->h_scal[SC_LS_C], slope = p->h_scal[SC_LS_SLOPE];
  *alpha = -1.0;
  *descent = slope < 0.0;
  if (slope < 0.0) {
    double a0 = a_start;
    for (int batch = 0; batch < 8 && *alpha < 0.0; ++batch) {
      if (batch > 0) {
        rc = eval_batch(a0);
        if (rc) return rc;
      }
      double a = a0;
      for (int j = 0; j < 4; ++j, a *= 0.5) {
        double df = a * b + 0.5 * a * a * c + p->h_scal[SC_DF + j];
        if (df <= o.ls_c1 * a * slope) {
          *alpha = a;
          break;
        }
      }
      a0 *= 1.0 / 16.0;
    }
  }
  return PL_OK;
}

// Trial steps a0, a0/2, a0/4, a0/8 of the line search along the real
// direction preal from the current linearisation (e), queued with their
// finalize into SC_DF..SC_DF+3.
template <typename T>
int ls_eval_queue(pl_plan* p, double a0) {
  if (p->model == MODEL_GAUSSIAN)
    hipLaunchKernelGGL((ls_eval_gauss_kernel<T>), dim3(NB_RED), dim3(RED_THREADS), 0, p->stream,
                       View<T>::preal(p), p->e, p->prob.w, p->prob.counts, p->prob.nbar, a0, p->N, p->partials);
  else
    hipLaunchKernelGGL((ls_eval_kernel<T>), dim3(NB_RED), dim3(RED_THREADS), 0, p->stream, View<T>::preal(p), p->e,
                       p->prob.counts, p->prob.beta, a0, p->N, p->partials);
  HIPCHK(p, hipGetLastError());
  HIPCHK(p, finalize(p, NB_RED, 4, FIN_STORE, SC_DF, 1.0));
  return PL_OK;
}

// One Newton step at the current spectral iterate, queued on the stream:
// the inner PCG on H x = -g in T precision (the host checks convergence
// between chunks of CG steps, the first chunk sized by first_chunk), then
// the Armijo line search of line_search's first batch (a = 1, 1/2, 1/4,
// 1/8) with the test itself on the device (ls_select_kernel ->
// SC_LS_ALPHA), and s_hat += alpha x on the device when a step was
// accepted.  The gradient that follows and its one read-back tell the host
// the outcome (newton_step_finish).  *its: CG iterations of the step.
template <typename T>
int newton_step_queue(pl_plan* p, double eta_gn, const pl_solve_opts& o, pl_solve_info& inf, int first_chunk,
                      int* its_out) {
  int rc;
  if constexpr (sizeof(T) == 4) {
    rc = ensure_d32(p);
    if (rc) return rc;
  }
  int its = 0, hv = 0;
  rc = pcg<T>(p, p->g_hat, -1.0, eta_gn, 0.0, o.max_cg, o.check_every, &its, &hv, nullptr, nullptr, first_chunk);
  if (rc) return rc;
  inf.cg_its += its;
  inf.hvps += hv;
  *its_out = its;
  cx<T>* x = View<T>::x(p);
  const double invN = 1.0 / (double)p->N;
  rc = inv_c2r<T>(p, x, View<T>::t(p), View<T>::preal(p));
  if (rc) return rc;
  hipLaunchKernelGGL((ls_dots_kernel<T>), dim3(NB_RED), dim3(RED_THREADS), 0, p->stream, x, p->s_hat, p->g_hat,
                     p->tab_mode, TAB_MODE, p->g, p->Nh, (double)p->N * prior_mean(p),
                     p->partials);
  HIPCHK(p, hipGetLastError());
  HIPCHK(p, finalize(p, NB_RED, 3, FIN_STORE, SC_LS_B, invN));
  rc = ls_eval_queue<T>(p, 1.0);
  if (rc) return rc;
  hipLaunchKernelGGL(ls_select_kernel, dim3(1), dim3(64), 0, p->stream, p->scal, 1.0, o.ls_c1);
  HIPCHK(p, hipGetLastError());
  hipLaunchKernelGGL((axpy_hat_dev_kernel<T>), dim3(NB_RED), dim3(RED_THREADS), 0, p->stream, p->s_hat, x,
                     p->scal + SC_LS_ALPHA, p->Nh);
  HIPCHK(p, hipGetLastError());
  return PL_OK;
}

// After a queued Newton step and the gradient that follows it have been
// read back (h_scal current): the step the device accepted, or, if the
// first batch of trial steps accepted none along a descent direction, the
// rest of the backtracking on the host (batches from 1/16, at most 32
// trial steps in all), the step applied and the gradient recomputed.
// *alpha = the accepted step or -1; *descent = (p^T g < 0).
template <typename T>
int newton_step_finish(pl_plan* p, double* s_io, const pl_solve_opts& o, double* alpha, bool* descent) {
  *alpha = p->h_scal[SC_LS_ALPHA];
  const double b = p->h_scal[SC_LS_B], c = p->h_scal[SC_LS_C], slope = p->h_scal[SC_LS_SLOPE];
  *descent = slope < 0.0;
  if (*alpha > 0.0 || !*descent) return PL_OK;
  *alpha = -1.0;
  double a0 = 1.0 / 16.0;
  for (int batch = 1; batch < 8 && *alpha < 0.0; ++batch) {
    // the direction and the linearisation at the (unchanged) iterate are
    // still in preal and e
    int rc = ls_eval_queue<T>(p, a0);
    if (rc) return rc;
    rc = read_scalars(p);
    if (rc) return rc;
    double a = a0;
    for (int j = 0; j < 4; ++j, a *= 0.5) {
      double df = a * b + 0.5 * a * a * c + p->h_scal[SC_DF + j];
      if (df <= o.ls_c1 * a * slope) {
        *alpha = a;
        break;
      }
    }
    a0 *= 1.0 / 16.0;
  }
  if (*alpha > 0.0) {
    hipLaunchKernelGGL((axpy_hat_kernel<T>), dim3(NB_RED), dim3(RED_THREADS), 0, p->stream, p->s_hat, View<T>::x(p),
                       *alpha, p->Nh);
    HIPCHK(p, hipGetLastError());
    int rc = grad_hat(p, s_io);
    if (rc) return rc;
    rc = read_scalars(p);
    if (rc) return rc;
  }
  return PL_OK;
}

// CG iterations queued before the first host check of a Newton step.  PCG
// on an SPD system needs about sqrt(kappa)/2 * ln(2/eta) iterations to cut
// the residual by eta, and kappa moves little between late Newton steps, so
// the previous step's count scaled by ln(2/eta)/ln(2/eta_prev) predicts
// this one; a small margin on top makes one check the usual case.  While
// the forcing term sits at its cap (the first, far-from-MAP steps) the
// counts jump between 1 and tens of iterations from step to step, so there
// at most 8 are queued before the first check.  Each check costs a host
// round trip (the copy, then the first launches of the next batch run as
// fast as the host issues them); each iteration queued past convergence
// costs its launches, which exit at once: two or three of those cost about
// one check.
int first_cg_chunk(int prev_its, double prev_eta, double eta, double eta_max) {
  if (prev_its <= 0 || !(prev_eta > 0.0 && prev_eta < 1.0) || !(eta > 0.0 && eta < 1.0)) return 8;
  const double pred = prev_its * std::log(2.0 / eta) / std::log(2.0 / prev_eta);
  const int want = std::max(4, (int)std::ceil(1.0625 * pred) + 2);
  return prev_eta >= eta_max ? std::min(want, 8) : want;
}

// Inexact Newton-Krylov from the current s_io.  Each Newton step is queued
// whole (CG, line search, the accepted update and the next gradient) and
// read back once, besides the checks between CG chunks.  In mixed
// precision (T = float) a step whose FP32 direction fails the line search
// is redone with an FP64 inner solve (refinement against the FP64
// gradient), and counted in info->fp64_steps.
template <typename T>
int newton_solve(pl_plan* p, double* s_io, const pl_solve_opts& o, pl_solve_info* info) {
  pl_solve_info inf{};
  int rc = fwd_r2c<double>(p, s_io, p->s_hat);
  if (rc) return rc;
  rc = grad_hat(p, s_io);
  if (rc) return rc;
  rc = read_scalars(p);
  if (rc) return rc;
  const double g0 = std::sqrt(std::max(0.0, p->h_scal[SC_GG]));
  double gn = g0;
  double obj = 0.5 * p->h_scal[SC_PRIOR] + p->h_scal[SC_LIK];
  inf.grad0 = g0;
  inf.obj = obj;
  if (!std::isfinite(g0) || !std::isfinite(obj)) {
    if (info) *info = inf;
    return fail(p, PL_ERR_DOMAIN, "gradient at the starting point is not finite");
  }
  int status = PL_OK;
  int prev_its = 0;
  double prev_eta = 0.0;
  if (g0 > 0.0) {
    for (int it = 0;; ++it) {
      if (gn <= o.rtol * g0) break;
      if (it >= o.max_newton) {
        status = PL_ERR_NOT_CONVERGED;
        p->err = "Newton iteration cap reached";
        break;
      }
      // forcing term: sqrt(||g||/||g0||), but no tighter than needed to
      // reach the stopping tolerance from here (half of it, for margin)
      const double eta = std::min(o.eta_max, std::max(std::sqrt(gn / g0), 0.5 * o.rtol * g0 / gn));
      Range range("pl newton step");
      rc = set_precond_constant(p);
      if (rc) return rc;
      int its = 0;
      rc = newton_step_queue<T>(p, eta * gn, o, inf, first_cg_chunk(prev_its, prev_eta, eta, o.eta_max), &its);
      if (rc) return rc;
      // FP64 directions: the step is applied to the real field too (their
      // real form from the line search is exact to FP64 rounding); FP32 ones
      // (whose real form carries FP32 transform rounding) go through s_hat
      rc = grad_hat(p, s_io, sizeof(T) == 8 ? p->preal : nullptr);
      if (rc) return rc;
      rc = read_scalars(p);
      if (rc) return rc;
      double alpha = -1.0;
      bool descent = false;
      rc = newton_step_finish<T>(p, s_io, o, &alpha, &descent);
      if (rc) return rc;
      if constexpr (sizeof(T) == 4) {
        if (alpha < 0.0) {
          // the iterate, its gradient and Hessian diagonal are unchanged;
          // the FP32 count at the same forcing term predicts the FP64 one
          int its64 = 0;
          rc = newton_step_queue<double>(p, eta * gn, o, inf, first_cg_chunk(its, eta, eta, o.eta_max), &its64);
          if (rc) return rc;
          rc = grad_hat(p, s_io, p->preal);
          if (rc) return rc;
          rc = read_scalars(p);
          if (rc) return rc;
          rc = newton_step_finish<double>(p, s_io, o, &alpha, &descent);
          if (rc) return rc;
          ++inf.fp64_steps;
        }
      }
      prev_its = its;
      prev_eta = eta;
      if (alpha < 0.0) {
        status = PL_ERR_LINESEARCH;
        p->err = descent ? "no step satisfies the Armijo condition" : "Newton direction is not a descent direction";
        break;
      }
      gn = std::sqrt(std::max(0.0, p->h_scal[SC_GG]));
      obj = 0.5 * p->h_scal[SC_PRIOR] + p->h_scal[SC_LIK];
      inf.newton_its = it + 1;
      if (!std::isfinite(gn)) {
        status = PL_ERR_DOMAIN;
        p->err = "gradient became non-finite";
        break;
      }
    }
  }
  inf.rel_grad = g0 > 0.0 ? gn / g0 : 0.0;
  inf.obj = obj;
  inf.status = status;
  if (info) *info = inf;
  return status;
}

// Solve H x_hat = g_hat (FP64 right-hand side in the plan's g_hat) with the
// plan's current Hessian diagonal d; the solution is left in x64 (FP64).
// T = double: one FP64 PCG.  T = float: iterative refinement -- each sweep
// solves H dl = r with FP32 PCG to a loose relative tolerance; x
// accumulates in FP64 and r = b - H x is recomputed with an FP64 HVP, so
// the FP32 rounding of the Krylov recurrences limits neither the attainable
// accuracy nor (through lost orthogonality) the iteration count.
// *rres: final residual norm, *bnorm: norm of the right-hand side.
template <typename T>
int solve_spd(pl_plan* p, const pl_solve_opts& o, int* its_out, int* hv_out, double* rres_out, double* bnorm_out) {
  int its = 0, hv = 0;
  double rres = 0.0, bnorm = 0.0;
  int rc = PL_OK;
  const double invN = 1.0 / (double)p->N;
  if constexpr (sizeof(T) == 8) {
    rc = pcg<double>(p, p->g_hat, 1.0, 0.0, o.rtol, o.max_cg, o.check_every, &its, &hv, &rres, &bnorm);
    if (rc) return rc;
  } else {
    HIPCHK(p, hipMemsetAsync(p->x64, 0, sizeof(cx<double>) * p->Nh, p->stream));
    const cx<double>* rhs = p->g_hat;
    double rn = 0.0, rn_prev = 0.0;
    for (int sweep = 0; its < o.max_cg; ++sweep) {
      const double target = sweep == 0 ? o.rtol : o.rtol * bnorm / rn;  // relative to this sweep's rhs
      const double eta = std::max(kRefineInnerRtol, target);
      int it = 0, h = 0;
      double rr_abs = 0.0, rhs_n = 0.0;
      rc = pcg<float>(p, rhs, 1.0, 0.0, eta, o.max_cg - its, o.check_every, &it, &h, &rr_abs, &rhs_n);
      if (rc) return rc;
      if (sweep == 0) bnorm = rhs_n;
      its += it;
      hv += h;
      if (bnorm == 0.0) break;
      hipLaunchKernelGGL((axpy_hat_kernel<float>), dim3(NB_RED), dim3(RED_THREADS), 0, p->stream, p->x64, p->x32,
                         1.0, p->Nh);
      HIPCHK(p, hipGetLastError());
      int nb = 0;
      rc = hvp_hat<double>(p, p->x64, p->p64, &nb);
      if (rc) return rc;
      ++hv;
      hipLaunchKernelGGL(resid_hat_kernel, dim3(NB_RED), dim3(RED_THREADS), 0, p->stream, p->g_hat, p->p64, p->r64,
                         p->g, p->Nh, p->partials);
      HIPCHK(p, hipGetLastError());
      HIPCHK(p, finalize(p, NB_RED, 1, FIN_STORE, SC_DF, invN));
      rc = read_scalars(p);
      if (rc) return rc;
      rn_prev = sweep == 0 ? bnorm : rn;
      rn = std::sqrt(std::max(0.0, p->h_scal[SC_DF]));
      rhs = p->r64;
      if (rn <= o.rtol * bnorm) break;
      if (it == 0 || rn > 0.9 * rn_prev) break;  // the sweeps stopped reducing the residual
    }
    rres = rn;
  }
  *its_out = its;
  *hv_out = hv;
  *rres_out = rres;
  *bnorm_out = bnorm;
  return PL_OK;
}

template <typename T>
int adjoint_solve(pl_plan* p, const double* s_star, const double* dL_ds, double* lambda_out, double* dA,
                  double* dbeta, double* dnbar, double* dN, double* dw, const pl_solve_opts& o,
                  pl_solve_info* info) {
  pl_solve_info inf{};
  const double invN = 1.0 / (double)p->N;
  // linearise at s*: s_hat = F s*, gradient pipeline gives d, e
  int rc = fwd_r2c<double>(p, s_star, p->s_hat);
  if (rc) return rc;
  rc = grad_hat(p, p->s_ws);
  if (rc) return rc;
  rc = read_scalars(p);
  if (rc) return rc;
  rc = set_precond_constant(p);
  if (rc) return rc;
  if constexpr (sizeof(T) == 4) {
    rc = ensure_d32(p);
    if (rc) return rc;
  }
  // rhs spectrum in g_hat
  rc = fwd_r2c<double>(p, dL_ds, p->g_hat);
  if (rc) return rc;
  int its = 0, hv = 0;
  double rres = 0.0, bnorm = 0.0;
  rc = solve_spd<T>(p, o, &its, &hv, &rres, &bnorm);
  if (rc) return rc;
  inf.cg_its = its;
  inf.hvps = hv;
  inf.grad0 = bnorm;
  inf.rel_grad = bnorm > 0.0 ? rres / bnorm : 0.0;
  double* lam = lambda_out ? lambda_out : p->rtmp;
  rc = inv_c2r<double>(p, p->x64, p->t64, lam);
  if (rc) return rc;
  // dL/dA from the spectral prior dot (k != 0)
  hipLaunchKernelGGL(adjoint_prior_dot_kernel, dim3(NB_RED), dim3(RED_THREADS), 0, p->stream, p->x64, p->s_hat,
                     p->tab_mode, TAB_MODE, p->g, p->Nh, p->partials);
  HIPCHK(p, hipGetLastError());
  HIPCHK(p, finalize(p, NB_RED, 1, FIN_STORE, SC_ADJ + 3, invN));
  hipLaunchKernelGGL(adjoint_cells_kernel, dim3(NB_RED), dim3(RED_THREADS), 0, p->stream, lam, s_star, p->prob.w,
                     p->prob.counts, p->prob.nbar, p->prob.beta, dN, dw, p->N, p->partials);
  HIPCHK(p, hipGetLastError());
  HIPCHK(p, finalize(p, NB_RED, 3, FIN_STORE, SC_ADJ, 1.0));
  rc = read_scalars(p);
  if (rc) return rc;
  if (dbeta) *dbeta = -p->h_scal[SC_ADJ];
  if (dnbar) *dnbar = -p->h_scal[SC_ADJ + 1];
  if (dA) *dA = p->h_scal[SC_ADJ + 3] / p->prob.amp;
  inf.status = inf.rel_grad > o.rtol ? PL_ERR_NOT_CONVERGED : PL_OK;
  if (inf.status) p->err = "adjoint solve stopped above the tolerance";
  if (info) *info = inf;
  return inf.status;
}

// The Krylov step of section 3.1 with a nonlinear-CG search vector:
// x <- x + tau xi with tau = -xi^T grad Q / xi^T H xi (eq. New5, one HVP per
// step).  The paper leaves the scheme for xi to an earlier reference; here
// xi is the preconditioned Polak-Ribiere+ conjugate direction
//   xi = -M^-1 g + beta xi_old,  beta = max(0, g^T M^-1 (g - g_old) / g_old^T M^-1 g_old),
// M = 1/lambda_k + dbar in Fourier space, restarted (beta = 0) when xi is not
// a descent direction, and each step is safeguarded by the Armijo search
// started at tau.  FP64; opts.max_cg caps the number of steps.
constexpr int kNlcgPrecondEvery = 16;  // steps between refreshes of dbar

int nlcg_solve(pl_plan* p, double* s_io, const pl_solve_opts& o, pl_solve_info* info) {
  pl_solve_info inf{};
  const double invN = 1.0 / (double)p->N;
  int rc = fwd_r2c<double>(p, s_io, p->s_hat);
  if (rc) return rc;
  rc = grad_hat(p, s_io);
  if (rc) return rc;
  rc = read_scalars(p);
  if (rc) return rc;
  const double g0 = std::sqrt(std::max(0.0, p->h_scal[SC_GG]));
  double gn = g0;
  inf.grad0 = g0;
  inf.obj = 0.5 * p->h_scal[SC_PRIOR] + p->h_scal[SC_LIK];
  if (!std::isfinite(g0) || !std::isfinite(inf.obj)) {
    if (info) *info = inf;
    return fail(p, PL_ERR_DOMAIN, "gradient at the starting point is not finite");
  }
  cx<double>* xi = p->x64;
  cx<double>* g_old = p->r64;
  cx<double>* q = p->p64;
  const double* tab = p->tab_mode;
  double gz_old = 0.0;
  bool restart = true;
  int status = PL_OK;
  for (int it = 0; g0 > 0.0; ++it) {
    if (gn <= o.rtol * g0) break;
    if (it >= o.max_cg) {
      status = PL_ERR_NOT_CONVERGED;
      p->err = "nonlinear-CG step cap reached";
      break;
    }
    if (it % kNlcgPrecondEvery == 0) {
      rc = set_precond_constant(p);
      if (rc) return rc;
    }
    // search vector
    hipLaunchKernelGGL(nlcg_dots_kernel, dim3(NB_RED), dim3(RED_THREADS), 0, p->stream, p->g_hat, g_old, tab,
                       TAB_MODE, p->g, p->Nh, p->scal, p->partials);
    HIPCHK(p, hipGetLastError());
    HIPCHK(p, finalize(p, NB_RED, 2, FIN_STORE, SC_DF, invN));
    rc = read_scalars(p);
    if (rc) return rc;
    const double gz = p->h_scal[SC_DF], gzo = p->h_scal[SC_DF + 1];
    double beta = (restart || !(gz_old > 0.0)) ? 0.0 : std::max(0.0, (gz - gzo) / gz_old);
    double slope = 0.0;
    for (int attempt = 0; attempt < 2; ++attempt) {
      hipLaunchKernelGGL(nlcg_update_kernel, dim3(NB_RED), dim3(RED_THREADS), 0, p->stream, p->g_hat, g_old, xi,
                         beta, tab, TAB_MODE, p->g, p->Nh, p->scal, p->partials);
      HIPCHK(p, hipGetLastError());
      HIPCHK(p, finalize(p, NB_RED, 1, FIN_STORE, SC_DF + 2, invN));
      rc = read_scalars(p);
      if (rc) return rc;
      slope = p->h_scal[SC_DF + 2];
      if (slope < 0.0 || beta == 0.0) break;
      beta = 0.0;  // not a descent direction: restart along -M^-1 g
    }
    gz_old = gz;
    restart = false;
    if (!(slope < 0.0)) {
      status = PL_ERR_LINESEARCH;
      p->err = "preconditioned gradient is not a descent direction";
      break;
    }
    // step length of eq. (New5) on the local quadratic model
    int nb = 0;
    rc = hvp_hat<double>(p, xi, q, &nb);
    if (rc) return rc;
    HIPCHK(p, finalize(p, nb, 3, FIN_STORE, SC_ADJ, invN));
    rc = read_scalars(p);
    if (rc) return rc;
    inf.hvps += 1;
    const double xhx = p->h_scal[SC_ADJ];
    if (!(xhx > 0.0)) {
      status = PL_ERR_LINESEARCH;
      p->err = "non-positive curvature along the search vector";
      break;
    }
    const double tau = -slope / xhx;
    double alpha = -1.0;
    bool descent = false;
    rc = line_search<double>(p, xi, tau, o, &alpha, &descent);
    if (rc) return rc;
    if (alpha < 0.0) {
      status = PL_ERR_LINESEARCH;
      p->err = "no step along the search vector satisfies the Armijo condition";
      break;
    }
    if (alpha < tau) restart = true;  // a shortened step: rebuild conjugacy from -M^-1 g
    hipLaunchKernelGGL((axpy_hat_kernel<double>), dim3(NB_RED), dim3(RED_THREADS), 0, p->stream, p->s_hat, xi,
                       alpha, p->Nh);
    HIPCHK(p, hipGetLastError());
    rc = grad_hat(p, s_io);
    if (rc) return rc;
    rc = read_scalars(p);
    if (rc) return rc;
    gn = std::sqrt(std::max(0.0, p->h_scal[SC_GG]));
    inf.obj = 0.5 * p->h_scal[SC_PRIOR] + p->h_scal[SC_LIK];
    inf.newton_its = it + 1;
    inf.cg_its = it + 1;
    if (!std::isfinite(gn)) {
      status = PL_ERR_DOMAIN;
      p->err = "gradient became non-finite";
      break;
    }
  }
  inf.rel_grad = g0 > 0.0 ? gn / g0 : 0.0;
  inf.status = status;
  if (info) *info = inf;
  return status;
}

// LSQ-Wiener filter, the paper's linear comparison estimator (section
// 4.1.1, the LSQ equation): with the mask operator
// W = diag(w), the Poisson noise covariance diag(w / nbar), the observed
// overdensity delta_o = N / nbar - w and unit bias, the filter
// (S^-1 + W^T N^-1 W)^-1 W^T N^-1 delta_o is the solution of
//   (S^-1 + diag(nbar w)) delta = N - nbar w,
// the Hessian system of the MAP pipeline with the constant diagonal
// d = nbar w.  S is the plan's prior covariance (A pk, inv_p0 at k = 0).
template <typename T>
int lsq_solve(pl_plan* p, double* delta_out, const pl_solve_opts& o, pl_solve_info* info) {
  pl_solve_info inf{};
  hipLaunchKernelGGL(lsq_setup_kernel, dim3(grid_blocks(p->N)), dim3(RED_THREADS), 0, p->stream, p->prob.w,
                     p->prob.counts, p->prob.nbar, p->d, p->rtmp, p->N);
  HIPCHK(p, hipGetLastError());
  p->d_valid = true;
  p->d32_valid = false;
  // sum of d (the preconditioner's percentile is taken relative to its mean)
  hipLaunchKernelGGL(sum_kernel, dim3(NB_RED), dim3(RED_THREADS), 0, p->stream, p->d, p->N, p->partials);
  HIPCHK(p, hipGetLastError());
  HIPCHK(p, finalize(p, NB_RED, 1, FIN_STORE, SC_DSUM, 1.0));
  int rc = set_precond_constant(p);
  if (rc) return rc;
  if constexpr (sizeof(T) == 4) {
    rc = ensure_d32(p);
    if (rc) return rc;
  }
  rc = fwd_r2c<double>(p, p->rtmp, p->g_hat);
  if (rc) return rc;
  int its = 0, hv = 0;
  double rres = 0.0, bnorm = 0.0;
  rc = solve_spd<T>(p, o, &its, &hv, &rres, &bnorm);
  if (rc) return rc;
  rc = inv_c2r<double>(p, p->x64, p->t64, delta_out);
  if (rc) return rc;
  HIPCHK(p, hipStreamSynchronize(p->stream));
  p->d_valid = false;  // nbar w is not a linearisation of the posterior
  p->d32_valid = false;
  inf.cg_its = its;
  inf.hvps = hv;
  inf.grad0 = bnorm;
  inf.rel_grad = bnorm > 0.0 ? rres / bnorm : 0.0;
  inf.status = inf.rel_grad > o.rtol ? PL_ERR_NOT_CONVERGED : PL_OK;
  if (inf.status) p->err = "LSQ solve stopped above the tolerance";
  if (info) *info = inf;
  return inf.status;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

void pl_default_opts(pl_solve_opts* o) {
  if (!o) return;
  o->rtol = 1e-8;
  o->max_newton = 100;
  o->max_cg = 500;
  o->eta_max = 0.5;
  o->ls_c1 = 1e-4;
  o->precision = -1;
  o->check_every = 16;
}

int pl_plan_create(pl_plan** out, const int32_t n[3], const double box[3], int precision, void* hip_stream,
                   size_t* workspace_bytes) {
  if (!out || !n || !box || !workspace_bytes) return PL_ERR_INVALID_ARG;
  *out = nullptr;
  for (int a = 0; a < 3; ++a) {
    if (!supported_length(n[a])) return PL_ERR_UNSUPPORTED_SIZE;
    if (!(box[a] > 0.0) || !std::isfinite(box[a])) return PL_ERR_INVALID_ARG;
  }
  if (precision != PL_FP64 && precision != PL_MIXED) return PL_ERR_INVALID_ARG;
  pl_plan* p = new pl_plan();
  for (int a = 0; a < 3; ++a) {
    p->n[a] = n[a];
    p->box[a] = box[a];
  }
  p->precision = precision;
  p->stream = (hipStream_t)hip_stream;
  p->N = (long)n[0] * n[1] * n[2];
  p->Nh = (long)n[0] * n[1] * (n[2] / 2 + 1);
  p->g = Grid{n[0], n[1], n[2], n[2] / 2 + 1, (long)n[1] * (n[2] / 2 + 1)};
  p->ws_bytes = carve(p, nullptr);
  // default tile variants (measured on MI355X): wide tiles for 512-point
  // FP64 transforms, the default tiles elsewhere; pl_plan_autotune refines
  p->var[0][V_XCG] = p->var[0][V_XOP] = (n[0] == 512) ? 1 : 0;
  p->var[0][V_Y] = (n[1] == 512) ? 1 : 0;
  p->var[0][V_Z] = (n[2] == 512) ? 1 : 0;
  if (hipHostMalloc((void**)&p->h_scal, sizeof(double) * SC_COUNT, hipHostMallocDefault) != hipSuccess) {
    delete p;
    return PL_ERR_HIP;
  }
  std::memset(p->h_scal, 0, sizeof(double) * SC_COUNT);
  *workspace_bytes = p->ws_bytes;
  *out = p;
  return PL_OK;
}

int pl_plan_set_workspace(pl_plan* p, void* dev_ptr) {
  if (!p) return PL_ERR_INVALID_ARG;
  if (!dev_ptr || ((uintptr_t)dev_ptr & 255)) return fail(p, PL_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  p->ws = (char*)dev_ptr;
  p->lb_ready = false;
  carve(p, p->ws);
  for (int a = 0; a < 3; ++a) {
    auto t64 = make_twiddles<double>(p->n[a]);
    HIPCHK(p, hipMemcpyAsync(p->tw64[a], t64.data(), sizeof(cx<double>) * p->n[a], hipMemcpyHostToDevice, p->stream));
    if (p->precision == PL_MIXED) {
      auto t32 = make_twiddles<float>(p->n[a]);
      HIPCHK(p, hipMemcpyAsync(p->tw32[a], t32.data(), sizeof(cx<float>) * p->n[a], hipMemcpyHostToDevice, p->stream));
    }
    HIPCHK(p, hipStreamSynchronize(p->stream));
  }
  HIPCHK(p, hipMemsetAsync(p->scal, 0, sizeof(double) * SC_COUNT, p->stream));
  HIPCHK(p, hipMemsetAsync(p->hist, 0, sizeof(int) * DQ_BINS, p->stream));
  HIPCHK(p, hipStreamSynchronize(p->stream));
  p->has_problem = false;
  p->d_valid = false;
  return PL_OK;
}

int pl_plan_set_stream(pl_plan* p, void* hip_stream) {
  if (!p) return PL_ERR_INVALID_ARG;
  p->stream = (hipStream_t)hip_stream;
  return PL_OK;
}

int pl_plan_destroy(pl_plan* p) {
  if (!p) return PL_ERR_INVALID_ARG;
  if (p->h_scal) (void)hipHostFree(p->h_scal);
  delete p;
  return PL_OK;
}

const char* pl_last_error(const pl_plan* p) {
  if (!p) return "null plan";
  return p->err.c_str();
}

int pl_set_problem(pl_plan* p, const pl_problem* pr) {
  if (!p || !pr) return PL_ERR_INVALID_ARG;
  p->lb_ready = false;
  if (!p->ws) return fail(p, PL_ERR_INVALID_ARG, "workspace not set");
  if (!pr->w || !pr->counts || !pr->pk) return fail(p, PL_ERR_INVALID_ARG, "null problem array");
  if (!(pr->amp > 0.0) || !std::isfinite(pr->amp)) return fail(p, PL_ERR_DOMAIN, "amp must be > 0");
  if (!(pr->nbar > 0.0) || !std::isfinite(pr->nbar)) return fail(p, PL_ERR_DOMAIN, "nbar must be > 0");
  if (!(pr->beta > 0.0) || !std::isfinite(pr->beta)) return fail(p, PL_ERR_DOMAIN, "beta must be > 0");
  if (!(pr->inv_p0 >= 0.0) || !std::isfinite(pr->inv_p0)) return fail(p, PL_ERR_DOMAIN, "inv_p0 must be >= 0");
  if (!std::isfinite(pr->mu)) return fail(p, PL_ERR_DOMAIN, "mu must be finite");
  p->has_problem = false;
  p->d_valid = false;
  HIPCHK(p, hipMemsetAsync(p->flags, 0, sizeof(int) * 4, p->stream));
  hipLaunchKernelGGL(validate_kernel, dim3(grid_blocks(p->N)), dim3(RED_THREADS), 0, p->stream, pr->w, pr->counts,
                     p->N, p->flags);
  HIPCHK(p, hipGetLastError());
  const double vol = p->box[0] * p->box[1] * p->box[2];
  const double coef = vol / ((double)p->N * pr->amp);
  hipLaunchKernelGGL(inv_lam_mode_kernel, dim3(grid_blocks(p->Nh)), dim3(RED_THREADS), 0, p->stream, pr->pk, coef,
                     pr->inv_p0, p->g, p->Nh, p->tab_mode, p->flags + 1);
  HIPCHK(p, hipGetLastError());
  hipLaunchKernelGGL(radial_scatter_kernel, dim3(grid_blocks(p->Nh)), dim3(RED_THREADS), 0, p->stream, p->tab_mode,
                     p->g, p->Nh, p->tab_rad);
  HIPCHK(p, hipGetLastError());
  hipLaunchKernelGGL(radial_check_kernel, dim3(grid_blocks(p->Nh)), dim3(RED_THREADS), 0, p->stream, p->tab_mode,
                     p->g, p->Nh, p->tab_rad, p->flags + 2);
  HIPCHK(p, hipGetLastError());
  int h[4] = {0, 0, 0, 0};
  HIPCHK(p, hipMemcpyAsync(h, p->flags, sizeof(int) * 4, hipMemcpyDeviceToHost, p->stream));
  HIPCHK(p, hipStreamSynchronize(p->stream));
  if (h[0] & 1) return fail(p, PL_ERR_DOMAIN, "counts must be finite and >= 0");
  if (h[0] & 2) return fail(p, PL_ERR_DOMAIN, "completeness w must be finite and >= 0");
  if (h[0] & 4) return fail(p, PL_ERR_DOMAIN, "counts > 0 in a cell with w = 0");
  if (h[1]) return fail(p, PL_ERR_DOMAIN, "pk must be finite and > 0 for k != 0");
  p->radial = h[2] ? 0 : 1;
  if (p->precision == PL_MIXED) {
    hipLaunchKernelGGL(to_f32_kernel, dim3(grid_blocks(p->Nh)), dim3(RED_THREADS), 0, p->stream, p->tab_mode,
                       p->tab_mode32, p->Nh);
    HIPCHK(p, hipGetLastError());
    hipLaunchKernelGGL(to_f32_kernel, dim3(grid_blocks(p->rad_len)), dim3(RED_THREADS), 0, p->stream, p->tab_rad,
                       p->tab_rad32, p->rad_len);
    HIPCHK(p, hipGetLastError());
    HIPCHK(p, hipStreamSynchronize(p->stream));
  }
  p->prob = *pr;
  p->has_problem = true;
  return PL_OK;
}

int pl_grad(pl_plan* p, const double* s, double* grad_out, double* obj_out) {
  int rc = check_ready(p);
  if (rc) return rc;
  if (!s || !grad_out) return fail(p, PL_ERR_INVALID_ARG, "null pointer");
  cx<double>* t = p->t64;
  RowArgs<double> ra = row_args<double>(p);
  ra.in_r = s;
  ra.out_c = t;
  HIPCHK(p, run_row<double>(p, ROW_R2C, ra, nullptr));
  HIPCHK(p, run_col<double>(p, 1, false, COL_PLAIN, col_args<double>(p, 1, t, t), nullptr));
  ColArgs<double> ca = col_args<double>(p, 0, t, t);
  ca.k0_shift = (double)p->N * p->prob.mu;
  int nb = 0;
  HIPCHK(p, run_col<double>(p, 0, false, COL_PRIOR, ca, &nb));
  HIPCHK(p, finalize(p, nb, 1, FIN_STORE, SC_PRIOR, 1.0 / (double)p->N));
  HIPCHK(p, run_col<double>(p, 1, true, COL_PLAIN, col_args<double>(p, 1, t, t), nullptr));
  RowArgs<double> rb = row_args<double>(p);
  rb.in_c = t;
  rb.out_r = grad_out;
  rb.s_in = s;
  rb.d_out = p->d;
  HIPCHK(p, run_row<double>(p, ROW_C2R_GRADLIK, rb, &nb));
  HIPCHK(p, finalize(p, nb, 2, FIN_STORE, SC_LIK, 1.0));
  p->d_valid = true;
  p->d32_valid = false;
  if (obj_out) {
    rc = read_scalars(p);
    if (rc) return rc;
    *obj_out = 0.5 * p->h_scal[SC_PRIOR] + p->h_scal[SC_LIK];
  }
  return PL_OK;
}

}  // extern "C"

namespace {
int linearize_at(pl_plan* p, const double* s) {
  if (s) {
    hipLaunchKernelGGL(linearize_kernel, dim3(grid_blocks(p->N)), dim3(RED_THREADS), 0, p->stream, s, p->prob.w,
                       p->prob.nbar, p->prob.beta, p->e, p->d, p->N);
    HIPCHK(p, hipGetLastError());
    p->d_valid = true;
    p->d32_valid = false;
  }
  if (!p->d_valid) return fail(p, PL_ERR_NO_PROBLEM, "no cached Hessian diagonal: pass s or call pl_grad first");
  return PL_OK;
}

template <typename T>
int hessvec_real(pl_plan* p, const double* s, const T* v, T* hv) {
  int rc = check_ready(p);
  if (rc) return rc;
  if (!v || !hv) return fail(p, PL_ERR_INVALID_ARG, "null pointer");
  rc = linearize_at(p, s);
  if (rc) return rc;
  if constexpr (sizeof(T) == 4) {
    rc = ensure_d32(p);
    if (rc) return rc;
  }
  cx<T>* t = View<T>::t(p);
  RowArgs<T> ra = row_args<T>(p);
  ra.in_r = v;
  ra.out_c = t;
  HIPCHK(p, run_row<T>(p, ROW_R2C, ra, nullptr));
  HIPCHK(p, run_col<T>(p, 1, false, COL_PLAIN, col_args<T>(p, 1, t, t), nullptr));
  ColArgs<T> ca = col_args<T>(p, 0, t, t);
  ca.k0_shift = 0.0;
  HIPCHK(p, run_col<T>(p, 0, false, COL_PRIOR, ca, nullptr));
  HIPCHK(p, run_col<T>(p, 1, true, COL_PLAIN, col_args<T>(p, 1, t, t), nullptr));
  RowArgs<T> rb = row_args<T>(p);
  rb.in_c = t;
  rb.out_r = hv;
  rb.v = v;
  HIPCHK(p, run_row<T>(p, ROW_C2R_DIAG, rb, nullptr));
  return PL_OK;
}

}  // namespace

extern "C" {

int pl_hessvec(pl_plan* p, const double* s, const double* v, double* hv_out) {
  return hessvec_real<double>(p, s, v, hv_out);
}

int pl_hessvec_f32(pl_plan* p, const double* s, const float* v, float* hv_out) {
  return hessvec_real<float>(p, s, v, hv_out);
}

int pl_hessvec_hat(pl_plan* p, const double* v_hat, double* hv_hat) {
  int rc = check_ready(p);
  if (rc) return rc;
  if (!v_hat || !hv_hat) return fail(p, PL_ERR_INVALID_ARG, "null pointer");
  if (!p->d_valid) return fail(p, PL_ERR_NO_PROBLEM, "no cached Hessian diagonal");
  int nb = 0;
  return hvp_hat<double>(p, (const cx<double>*)v_hat, (cx<double>*)hv_hat, &nb);
}

int pl_hessvec_hat_f32(pl_plan* p, const float* v_hat, float* hv_hat) {
  int rc = check_ready(p);
  if (rc) return rc;
  if (!v_hat || !hv_hat) return fail(p, PL_ERR_INVALID_ARG, "null pointer");
  if (!p->d_valid) return fail(p, PL_ERR_NO_PROBLEM, "no cached Hessian diagonal");
  rc = ensure_d32(p);
  if (rc) return rc;
  int nb = 0;
  return hvp_hat<float>(p, (const cx<float>*)v_hat, (cx<float>*)hv_hat, &nb);
}

int pl_newton_krylov_solve_hat(pl_plan* p, double* s_inout, double* s_hat_out, const pl_solve_opts* opts,
                               pl_solve_info* info) {
  int rc = check_ready(p);
  if (rc) return rc;
  if (!s_inout) return fail(p, PL_ERR_INVALID_ARG, "null s_inout");
  pl_solve_opts o = resolve_opts(p, opts);
  if (!(o.rtol >= 0.0) || o.max_newton < 0 || o.max_cg <= 0 || !(o.eta_max > 0.0) || !(o.ls_c1 > 0.0 && o.ls_c1 < 1.0))
    return fail(p, PL_ERR_INVALID_ARG, "invalid solve options");
  rc = check_finite(p, s_inout, p->N, "s_inout");
  if (rc) return rc;
  if (o.precision == PL_MIXED && p->precision != PL_MIXED)
    return fail(p, PL_ERR_INVALID_ARG, "mixed solve needs a PL_MIXED plan");
  rc = o.precision == PL_MIXED ? newton_solve<float>(p, s_inout, o, info) : newton_solve<double>(p, s_inout, o, info);
  if (s_hat_out && (rc == PL_OK || rc == PL_ERR_NOT_CONVERGED || rc == PL_ERR_LINESEARCH)) {
    HIPCHK(p, hipMemcpyAsync(s_hat_out, p->s_hat, sizeof(cx<double>) * p->Nh, hipMemcpyDeviceToDevice, p->stream));
    HIPCHK(p, hipStreamSynchronize(p->stream));
  }
  return rc;
}

int pl_newton_krylov_solve(pl_plan* p, double* s_inout, const pl_solve_opts* opts, pl_solve_info* info) {
  return pl_newton_krylov_solve_hat(p, s_inout, nullptr, opts, info);
}

int pl_solve_adjoint(pl_plan* p, const double* s_star, const double* dL_ds, double* lambda_out, double* dL_dA,
                     double* dL_dbeta, double* dL_dnbar, double* dL_dN, double* dL_dw, const pl_solve_opts* opts,
                     pl_solve_info* info) {
  int rc = check_ready(p);
  if (rc) return rc;
  if (!s_star || !dL_ds) return fail(p, PL_ERR_INVALID_ARG, "null pointer");
  pl_solve_opts o = resolve_opts(p, opts);
  if (!(o.rtol >= 0.0) || o.max_cg <= 0) return fail(p, PL_ERR_INVALID_ARG, "invalid solve options");
  rc = check_finite(p, dL_ds, p->N, "dL_ds");
  if (rc) return rc;
  if (o.precision == PL_MIXED) {
    if (p->precision != PL_MIXED) return fail(p, PL_ERR_INVALID_ARG, "mixed adjoint needs a PL_MIXED plan");
    return adjoint_solve<float>(p, s_star, dL_ds, lambda_out, dL_dA, dL_dbeta, dL_dnbar, dL_dN, dL_dw, o, info);
  }
  return adjoint_solve<double>(p, s_star, dL_ds, lambda_out, dL_dA, dL_dbeta, dL_dnbar, dL_dN, dL_dw, o, info);
}

int pl_gaussian_map_solve(pl_plan* p, double* delta_inout, const pl_solve_opts* opts, pl_solve_info* info) {
  int rc = check_ready(p);
  if (rc) return rc;
  if (!delta_inout) return fail(p, PL_ERR_INVALID_ARG, "null pointer");
  pl_solve_opts o = resolve_opts(p, opts);
  if (!(o.rtol >= 0.0) || o.max_newton < 0 || o.max_cg <= 0 || !(o.eta_max > 0.0) || !(o.ls_c1 > 0.0 && o.ls_c1 < 1.0))
    return fail(p, PL_ERR_INVALID_ARG, "invalid solve options");
  rc = check_finite(p, delta_inout, p->N, "delta_inout");
  if (rc) return rc;
  if (o.precision == PL_MIXED && p->precision != PL_MIXED)
    return fail(p, PL_ERR_INVALID_ARG, "mixed solve needs a PL_MIXED plan");
  // the start must lie where every cell with counts has 1 + delta > 0
  HIPCHK(p, hipMemsetAsync(p->flags, 0, sizeof(int), p->stream));
  hipLaunchKernelGGL(gauss_domain_kernel, dim3(grid_blocks(p->N)), dim3(RED_THREADS), 0, p->stream, delta_inout,
                     p->prob.counts, p->N, p->flags);
  HIPCHK(p, hipGetLastError());
  int h = 0;
  HIPCHK(p, hipMemcpyAsync(&h, p->flags, sizeof(int), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(p, hipStreamSynchronize(p->stream));
  if (h) return fail(p, PL_ERR_DOMAIN, "1 + delta <= 0 in a cell with counts at the start");
  p->model = MODEL_GAUSSIAN;
  rc = o.precision == PL_MIXED ? newton_solve<float>(p, delta_inout, o, info)
                               : newton_solve<double>(p, delta_inout, o, info);
  p->model = MODEL_LOGNORMAL;
  p->d_valid = false;  // the cached diagonal belongs to the Gaussian model
  return rc;
}

int pl_nlcg_solve(pl_plan* p, double* s_inout, const pl_solve_opts* opts, pl_solve_info* info) {
  int rc = check_ready(p);
  if (rc) return rc;
  if (!s_inout) return fail(p, PL_ERR_INVALID_ARG, "null pointer");
  pl_solve_opts o = resolve_opts(p, opts);
  if (!(o.rtol >= 0.0) || o.max_cg <= 0 || !(o.ls_c1 > 0.0 && o.ls_c1 < 1.0))
    return fail(p, PL_ERR_INVALID_ARG, "invalid solve options");
  if (opts && opts->precision == PL_MIXED)
    return fail(p, PL_ERR_INVALID_ARG, "the nonlinear-CG solve runs in FP64 only");
  rc = check_finite(p, s_inout, p->N, "s_inout");
  if (rc) return rc;
  return nlcg_solve(p, s_inout, o, info);
}

int pl_lognormal_prior(pl_plan* p, const double* pk, double amp, double* pk_log_out, double* mu_out,
                       double* sigma0_sq_out, int64_t* n_clipped_out) {
  if (!p) return PL_ERR_INVALID_ARG;
  p->lb_ready = false;
  if (!p->ws) return fail(p, PL_ERR_INVALID_ARG, "workspace not set");
  if (!pk || !pk_log_out) return fail(p, PL_ERR_INVALID_ARG, "null pointer");
  if (!(amp > 0.0) || !std::isfinite(amp)) return fail(p, PL_ERR_DOMAIN, "amp must be finite and > 0");
  const double coef = amp * (double)p->N / (p->box[0] * p->box[1] * p->box[2]);
  cx<double>* t = p->t64;
  double* field = p->s_ws;
  HIPCHK(p, hipMemsetAsync(p->flags, 0, sizeof(int) * 4, p->stream));
  // S(r): inverse transform of the eigenvalues of S (the 1/N of the inverse
  // makes S(0) the cell variance (1/V) sum_k amp pk_k)
  hipLaunchKernelGGL(spectrum_to_half_kernel, dim3(grid_blocks(p->Nh)), dim3(RED_THREADS), 0, p->stream, pk, coef, t,
                     p->Nh);
  HIPCHK(p, hipGetLastError());
  int rc = inv_c2r<double>(p, t, t, field);
  if (rc) return rc;
  hipLaunchKernelGGL(log1p_field_kernel, dim3(grid_blocks(p->N)), dim3(RED_THREADS), 0, p->stream, field, p->N,
                     p->flags);
  HIPCHK(p, hipGetLastError());
  double s_l0 = 0.0;
  int h[4] = {0, 0, 0, 0};
  HIPCHK(p, hipMemcpyAsync(&s_l0, field, sizeof(double), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(p, hipMemcpyAsync(h, p->flags, sizeof(int) * 4, hipMemcpyDeviceToHost, p->stream));
  HIPCHK(p, hipStreamSynchronize(p->stream));
  if (h[0]) return fail(p, PL_ERR_DOMAIN, "the correlation function reaches -1: ln(1 + S) is undefined");
  rc = fwd_r2c<double>(p, field, t);
  if (rc) return rc;
  // the mean of lambda^L over the full spectrum is S_L(0) = sigma0^2
  const double floor_val = kPriorFloorRel * std::fabs(s_l0);
  // P_L = lambda^L V / N: the log-field spectrum itself (use it with amp = 1)
  const double v_over_n = p->box[0] * p->box[1] * p->box[2] / (double)p->N;
  hipLaunchKernelGGL(half_to_spectrum_kernel, dim3(grid_blocks(p->Nh)), dim3(RED_THREADS), 0, p->stream, t,
                     v_over_n, floor_val, pk_log_out, p->Nh, p->flags);
  HIPCHK(p, hipGetLastError());
  HIPCHK(p, hipMemcpyAsync(h, p->flags, sizeof(int) * 4, hipMemcpyDeviceToHost, p->stream));
  HIPCHK(p, hipStreamSynchronize(p->stream));
  if (sigma0_sq_out) *sigma0_sq_out = s_l0;
  if (mu_out) *mu_out = -0.5 * s_l0;
  if (n_clipped_out) *n_clipped_out = h[1];
  return PL_OK;
}

int pl_lsq_solve(pl_plan* p, double* delta_out, const pl_solve_opts* opts, pl_solve_info* info) {
  int rc = check_ready(p);
  if (rc) return rc;
  if (!delta_out) return fail(p, PL_ERR_INVALID_ARG, "null pointer");
  pl_solve_opts o = resolve_opts(p, opts);
  if (!(o.rtol >= 0.0) || o.max_cg <= 0) return fail(p, PL_ERR_INVALID_ARG, "invalid solve options");
  if (o.precision == PL_MIXED) {
    if (p->precision != PL_MIXED) return fail(p, PL_ERR_INVALID_ARG, "mixed LSQ solve needs a PL_MIXED plan");
    return lsq_solve<float>(p, delta_out, o, info);
  }
  return lsq_solve<double>(p, delta_out, o, info);
}

int pl_inverse_weight(pl_plan* p, double* delta_out) {
  int rc = check_ready(p);
  if (rc) return rc;
  if (!delta_out) return fail(p, PL_ERR_INVALID_ARG, "null pointer");
  hipLaunchKernelGGL(inverse_weight_kernel, dim3(grid_blocks(p->N)), dim3(RED_THREADS), 0, p->stream, p->prob.w,
                     p->prob.counts, p->prob.nbar, delta_out, p->N);
  HIPCHK(p, hipGetLastError());
  return PL_OK;
}

int pl_compare_fields(pl_plan* p, const double* rec, const double* ref, double* r_out, double* d_euc_out) {
  if (!p) return PL_ERR_INVALID_ARG;
  if (!p->ws) return fail(p, PL_ERR_INVALID_ARG, "workspace not set");
  if (!rec || !ref) return fail(p, PL_ERR_INVALID_ARG, "null pointer");
  hipLaunchKernelGGL(compare_fields_kernel, dim3(NB_RED), dim3(RED_THREADS), 0, p->stream, rec, ref, p->N,
                     p->partials);
  HIPCHK(p, hipGetLastError());
  HIPCHK(p, finalize(p, NB_RED, 4, FIN_STORE, SC_DF, 1.0));
  int rc = read_scalars(p);
  if (rc) return rc;
  const double srr = p->h_scal[SC_DF], sxx = p->h_scal[SC_DF + 1], syy = p->h_scal[SC_DF + 2],
               sdd = p->h_scal[SC_DF + 3];
  if (r_out) *r_out = (sxx > 0.0 && syy > 0.0) ? srr / (std::sqrt(sxx) * std::sqrt(syy)) : 0.0;
  if (d_euc_out) *d_euc_out = std::sqrt(sdd / (double)p->N);
  return PL_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free variant of pl_compare_fields
// ---------------------------------------------------------------------------

namespace {

// Its scratch: NB_RED blocks x 4 per-block partial sums, then the 4 sums.
// One copy of this array per GPU, alive until the process ends; every call
// on a GPU overwrites it completely before reading it (nothing needs to
// start at zero), and calls that overlap on one GPU race on it.
constexpr int kNoallocPartials = NB_RED * 4;
constexpr int kNoallocDoubles = kNoallocPartials + 4;
constexpr long kNoallocMaxCells = 512L * 512L * 512L;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[kNoallocDoubles];

std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (host code must not use the array's name as an address).
int scratch_on_current_device(double** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return PL_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return PL_ERR_HIP;
    g_scratch_dev[dev] = (double*)ptr;
  }
  *out = g_scratch_dev[dev];
  return PL_OK;
}

// r and D_euc from the four sums (section 4.1.2), as pl_compare_fields forms
// them on the host.
__global__ void compare_out_kernel(const double* __restrict__ sums, long n, double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  const double srr = sums[0], sxx = sums[1], syy = sums[2], sdd = sums[3];
  out[0] = (sxx > 0.0 && syy > 0.0) ? srr / (sqrt(sxx) * sqrt(syy)) : 0.0;
  out[1] = sqrt(sdd / (double)n);
}

}  // namespace

extern "C" int pl_compare_fields_noalloc(const int32_t n[3], const double* rec, const double* ref, double* out,
                                         void* hip_stream) {
  if (!n || !rec || !ref || !out) return PL_ERR_INVALID_ARG;
  long cells = 1;
  for (int a = 0; a < 3; ++a) {
    if (n[a] < 1) return PL_ERR_INVALID_ARG;
    cells *= n[a];
    if (cells > kNoallocMaxCells) return PL_ERR_UNSUPPORTED_SIZE;
  }
  double* sc = nullptr;
  int rc = scratch_on_current_device(&sc);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)hip_stream;
  hipLaunchKernelGGL(compare_fields_kernel, dim3(NB_RED), dim3(RED_THREADS), 0, st, rec, ref, cells, sc);
  if (hipGetLastError() != hipSuccess) return PL_ERR_HIP;
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(FIN_THREADS), 0, st, sc, NB_RED, 4, (int)FIN_STORE, 0, 1.0,
                     sc + kNoallocPartials, 0.0, (const double*)nullptr, 0, 0.0);
  if (hipGetLastError() != hipSuccess) return PL_ERR_HIP;
  hipLaunchKernelGGL(compare_out_kernel, dim3(1), dim3(64), 0, st, sc + kNoallocPartials, cells, out);
  if (hipGetLastError() != hipSuccess) return PL_ERR_HIP;
  return PL_OK;
}

namespace pl {
bool supported_length(int n) {
  switch (n) {
    case 8: case 12: case 16: case 24: case 32: case 48: case 64: case 96: case 128: case 192: case 256: case 512:
      return true;
    default:
      return false;
  }
}
}  // namespace pl

// ===========================================================================
// Tile-variant autotuner
// ===========================================================================

namespace {

std::string arch_name() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

// Time one fused CG step (the solver's hot loop: pass 1 with the Krylov
// prologue, y inverse, z, y forward, pass 5 with the Krylov updates), average
// of `reps`, with the plan's current variants.  Runs on zeroed vectors with
// zero step lengths, so nothing is left in a meaningful state.
template <typename T>
int fill_hash(pl_plan* p, T* x, long n, unsigned seed, double lo = -1.0, double span = 2.0) {
  hipLaunchKernelGGL((fill_hash_kernel<T>), dim3(grid_blocks(n)), dim3(RED_THREADS), 0, p->stream, x, n, seed, lo,
                     span);
  HIPCHK(p, hipGetLastError());
  return PL_OK;
}

template <typename T>
int time_cg_step(pl_plan* p, int reps, float* ms) {
  cx<T>*x = View<T>::x(p), *r = View<T>::r(p), *pp = View<T>::pv(p), *t = View<T>::t(p);
  if (int frc = fill_hash<T>(p, (T*)x, 2 * p->Nh, 1)) return frc;
  if (int frc = fill_hash<T>(p, (T*)r, 2 * p->Nh, 2)) return frc;
  if (int frc = fill_hash<T>(p, (T*)pp, 2 * p->Nh, 3)) return frc;
  HIPCHK(p, hipMemsetAsync(p->scal, 0, sizeof(double) * SC_COUNT, p->stream));  // alpha = beta = 0
  auto step = [&]() -> hipError_t {
    ColArgs<T> c1 = col_args<T>(p, 0, pp, t);
    c1.cg_r = r;
    c1.scal = p->scal;
    hipError_t e = run_col<T>(p, 0, true, COL_CG_FIRST, c1, nullptr);
    if (e != hipSuccess) return e;
    e = run_col<T>(p, 1, true, COL_PLAIN, col_args<T>(p, 1, t, t), nullptr);
    if (e != hipSuccess) return e;
    RowArgs<T> ra = row_args<T>(p);
    ra.in_c = t;
    ra.out_c = t;
    e = run_row<T>(p, ROW_HVP, ra, nullptr);
    if (e != hipSuccess) return e;
    e = run_col<T>(p, 1, false, COL_PLAIN, col_args<T>(p, 1, t, t), nullptr);
    if (e != hipSuccess) return e;
    ColArgs<T> c5 = col_args<T>(p, 0, t, t);
    c5.base = pp;
    c5.cg_r = r;
    c5.cg_x = x;
    c5.scal = p->scal;
    return run_col<T>(p, 0, false, COL_CG_LAST, c5, nullptr);
  };
  hipEvent_t e0, e1;
  HIPCHK(p, hipEventCreate(&e0));
  HIPCHK(p, hipEventCreate(&e1));
  hipError_t err = hipSuccess;
  for (int i = 0; i < 2 && err == hipSuccess; ++i) err = step();
  if (err == hipSuccess) {
    (void)hipEventRecord(e0, p->stream);
    for (int i = 0; i < reps && err == hipSuccess; ++i) err = step();
    (void)hipEventRecord(e1, p->stream);
    (void)hipEventSynchronize(e1);
    (void)hipEventElapsedTime(ms, e0, e1);
    *ms /= (float)reps;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIPCHK(p, err);
  return PL_OK;
}

// Time one spectral Hessian-vector product (the isolated operator,
// pl_hessvec_hat), average of `reps`.
template <typename T>
int time_hvp(pl_plan* p, int reps, float* ms) {
  if (int frc = fill_hash<T>(p, (T*)View<T>::x(p), 2 * p->Nh, 4)) return frc;
  hipEvent_t e0, e1;
  HIPCHK(p, hipEventCreate(&e0));
  HIPCHK(p, hipEventCreate(&e1));
  int nb = 0, rc = PL_OK;
  for (int i = 0; i < 2 && !rc; ++i) rc = hvp_hat<T>(p, View<T>::x(p), View<T>::r(p), &nb);
  if (!rc) {
    (void)hipEventRecord(e0, p->stream);
    for (int i = 0; i < reps && !rc; ++i) rc = hvp_hat<T>(p, View<T>::x(p), View<T>::r(p), &nb);
    (void)hipEventRecord(e1, p->stream);
    (void)hipEventSynchronize(e1);
    (void)hipEventElapsedTime(ms, e0, e1);
    *ms /= (float)reps;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

// Try every combination of the choices in `slots` (each 0..max, skipping
// values a slot does not allow), timing with `timer`; keep the fastest.
// Returns its time in *best.
template <typename Timer>
int tune_slots(pl_plan* p, int pi, const int* slots, const int* maxv, int ns, Timer timer, float* best) {
  int cur[V_COUNT] = {}, keep[V_COUNT] = {};
  *best = 1e30f;
  for (;;) {
    bool ok = true;
    for (int i = 0; i < ns; ++i) ok = ok && variant_allowed(slots[i], cur[i]);
    if (ok) {
      for (int i = 0; i < ns; ++i) p->var[pi][slots[i]] = cur[i];
      float ms = 0.f;
      int rc = timer(&ms);
      if (rc) return rc;
      if (ms < *best) {
        *best = ms;
        for (int i = 0; i < ns; ++i) keep[i] = cur[i];
      }
    }
    int i = 0;
    while (i < ns && cur[i] == maxv[i]) cur[i++] = 0;
    if (i == ns) break;
    ++cur[i];
  }
  for (int i = 0; i < ns; ++i) p->var[pi][slots[i]] = keep[i];
  return PL_OK;
}

template <typename T>
int tune_precision(pl_plan* p, const std::string& key, std::vector<std::string>& cache_lines, bool* added) {
  const int pi = sizeof(T) == 4 ? 1 : 0;
  for (const std::string& line : cache_lines) {
    if (line.compare(0, key.size() + 1, key + " ") == 0) {
      int v[V_COUNT];
      float t_cg, t_hvp;
      bool ok = std::sscanf(line.c_str() + key.size(), "%d %d %d %d %d %d %d %f %f", &v[0], &v[1], &v[2], &v[3],
                            &v[4], &v[5], &v[6], &t_cg, &t_hvp) == V_COUNT + 2;
      for (int i = 0; ok && i < V_COUNT; ++i) ok = variant_allowed(i, v[i]);
      if (ok) {
        for (int i = 0; i < V_COUNT; ++i) p->var[pi][i] = v[i];
        return PL_OK;
      }
    }
  }
  // column passes: default, wide, split, extra-wide, wide split and
  // extra-wide split tiles (lengths 128-512); rows: default and wide
  const int mx = has_wide_variant(p->n[0]) ? 6 : 0, my = has_wide_variant(p->n[1]) ? 6 : 0,
            mr = has_wide_variant(p->n[2]) ? 1 : 0, mt = p->radial ? 2 : 0;
  const int reps = p->N >= (1L << 24) ? 5 : 20;
  // the solver's CG step: first the tile variants of the x passes carrying
  // the Krylov updates, y and z and the table those x passes read (default
  // load/store policy), then the streaming policy with those fixed, then the
  // tiles once more under that policy
  const int cg_slots[4] = {V_XCG, V_Y, V_Z, V_TAB_CG}, cg_max[4] = {mx, my, mr, mt};
  float best_cg = 0.f, best_hvp = 0.f;
  p->var[pi][V_NT] = 0;
  int rc = tune_slots(p, pi, cg_slots, cg_max, 4, [&](float* ms) { return time_cg_step<T>(p, reps, ms); }, &best_cg);
  if (rc) return rc;
  const int nt_slot[1] = {V_NT}, nt_max[1] = {NT_ALL};
  rc = tune_slots(p, pi, nt_slot, nt_max, 1, [&](float* ms) { return time_cg_step<T>(p, reps, ms); }, &best_cg);
  if (rc) return rc;
  // the tiles again, under the chosen policy
  rc = tune_slots(p, pi, cg_slots, cg_max, 4, [&](float* ms) { return time_cg_step<T>(p, reps, ms); }, &best_cg);
  if (rc) return rc;
  // the isolated operator's x passes and their table
  const int op_slots[2] = {V_XOP, V_TAB_OP}, op_max[2] = {mx, mt};
  rc = tune_slots(p, pi, op_slots, op_max, 2, [&](float* ms) { return time_hvp<T>(p, reps, ms); }, &best_hvp);
  if (rc) return rc;
  const int* v = p->var[pi];
  char buf[256];
  std::snprintf(buf, sizeof(buf), "%s %d %d %d %d %d %d %d %.4f %.4f", key.c_str(), v[0], v[1], v[2], v[3], v[4],
                v[5], v[6], (double)best_cg, (double)best_hvp);
  cache_lines.push_back(buf);
  *added = true;
  return PL_OK;
}

}  // namespace

// The tune cache holds the lines of both autotuners (plan and batch); each
// rewrites the whole file with both format lines on top.
static void write_tune_cache(const char* path, const std::vector<std::string>& lines) {
  if (FILE* f = std::fopen(path, "w")) {
    std::fprintf(f,
                 "# pl_plan_autotune cache: arch grid table precision x(Krylov passes) y z x(operator passes) "
                 "table(Krylov) table(operator) streaming-loads ms/CG-step ms/HVP\n"
                 "# pl_batch_autotune cache: arch batch precision lengths (most cells first) "
                 "column-variants row-variants ms/CG-step\n");
    for (const std::string& l : lines) std::fprintf(f, "%s\n", l.c_str());
    std::fclose(f);
  }
}

extern "C" int pl_plan_autotune(pl_plan* p, const char* cache_path) {
  int rc = check_ready(p);
  if (rc) return rc;
  std::vector<std::string> lines;
  if (cache_path) {
    if (FILE* f = std::fopen(cache_path, "r")) {
      char buf[512];
      while (std::fgets(buf, sizeof(buf), f)) {
        std::string l(buf);
        while (!l.empty() && (l.back() == '\n' || l.back() == '\r')) l.pop_back();
        if (!l.empty() && l[0] != '#') lines.push_back(l);
      }
      std::fclose(f);
    }
  }
  // a positive Hessian diagonal for the timing runs
  rc = fill_hash<double>(p, p->d, p->N, 5, 0.0, 1.0);
  if (rc) return rc;
  p->d_valid = true;
  p->d32_valid = false;
  // keyed by whether the problem's spectrum allows the radial table
  const std::string base = arch_name() + " " + std::to_string(p->n[0]) + "x" + std::to_string(p->n[1]) + "x" +
                           std::to_string(p->n[2]) + (p->radial ? " shell" : " mode");
  bool added = false;
  rc = tune_precision<double>(p, base + " fp64", lines, &added);
  if (rc) return rc;
  if (p->precision == PL_MIXED) {
    rc = ensure_d32(p);
    if (rc) return rc;
    rc = tune_precision<float>(p, base + " fp32", lines, &added);
    if (rc) return rc;
  }
  p->d_valid = false;  // the timing diagonal is not a linearisation of the posterior
  if (cache_path && added) write_tune_cache(cache_path, lines);
  return PL_OK;
}

extern "C" int pl_plan_set_variants(pl_plan* p, const int32_t v[2 * PL_NUM_VARIANTS]) {
  if (!p || !v) return PL_ERR_INVALID_ARG;
  for (int i = 0; i < 2 * V_COUNT; ++i)
    if (!variant_allowed(i % V_COUNT, v[i])) return fail(p, PL_ERR_INVALID_ARG, "schedule choice out of range");
  for (int pi = 0; pi < 2; ++pi)
    for (int i = 0; i < V_COUNT; ++i) p->var[pi][i] = v[V_COUNT * pi + i];
  return PL_OK;
}

extern "C" int pl_plan_get_variants(const pl_plan* p, int32_t out[2 * PL_NUM_VARIANTS]) {
  if (!p || !out) return PL_ERR_INVALID_ARG;
  for (int pi = 0; pi < 2; ++pi)
    for (int i = 0; i < V_COUNT; ++i) out[V_COUNT * pi + i] = p->var[pi][i];
  return PL_OK;
}

extern "C" int pl_plan_prior_is_radial(const pl_plan* p, int32_t* radial_out) {
  if (!p || !radial_out) return PL_ERR_INVALID_ARG;
  if (!p->has_problem) return fail(const_cast<pl_plan*>(p), PL_ERR_NO_PROBLEM, "pl_set_problem has not been called");
  *radial_out = p->radial;
  return PL_OK;
}

// ===========================================================================
// Batched solves
// ===========================================================================

namespace {

constexpr int NBB = 64;  // blocks per instance of the batched elementwise kernels

int xcd_remap(int hw, int total) {
  const int xcd = hw & 7, k = hw >> 3, per = total >> 3, rem = total & 7;
  return xcd * per + (xcd < rem ? xcd : rem) + k;
}

// staging slots of the batch's control-record uploads (bctl)
constexpr int kCtlSlots = 4;

// Work list of one batched pass with its launch configuration: blocks
// ordered so that each XCD receives a contiguous range of work items, the
// block size and dynamic LDS the largest of the instances' tile shapes.
struct BWork {
  std::vector<int4> items;  // the items of length class 0, then those of class 1
  std::vector<int> nb;      // blocks per instance (= partial-sum records)
  int split = 0;            // number of class-0 items
  int threads[BATCH_CLASSES] = {0, 0}, lds[BATCH_CLASSES] = {0, 0};  // per class launch
  size_t off = 0, cap = 0;  // region in the blob and its capacity (items)
};
// W_XC / W_YC / W_RC: the running solve's CG passes over the instances not
// yet finished (rebuilt as they finish, so that the last CG steps do not
// dispatch the blocks of finished grids)
enum BWorkId { W_X64 = 0, W_Y64, W_R64, W_X32, W_Y32, W_R32, W_XC, W_YC, W_RC, W_COUNT };

void order_for_xcds(std::vector<int4>& nat) {
  std::vector<int4> w(nat.size());
  for (int hw = 0; hw < (int)nat.size(); ++hw) w[hw] = nat[xcd_remap(hw, (int)nat.size())];
  nat.swap(w);
}

// The per-class item lists in launch order: each class XCD-ordered for its
// own launch, class 0 first.
void join_classes(BWork& w, std::vector<int4>* cls) {
  order_for_xcds(cls[0]);
  order_for_xcds(cls[1]);
  w.items = cls[0];
  w.items.insert(w.items.end(), cls[1].begin(), cls[1].end());
  w.split = (int)cls[0].size();
}

// Column pass over all instances (axis 0: x, 1: y), instance i in tile
// variant var[i].
template <typename T>
void col_work(const std::vector<pl_plan*>& plans, int axis, const std::vector<int>& var, BWork& w,
              const std::vector<int>* subset = nullptr) {
  std::vector<int4> cls[BATCH_CLASSES];
  w.nb.assign(plans.size(), 0);
  for (int c = 0; c < BATCH_CLASSES; ++c) w.threads[c] = w.lds[c] = 0;
  for (size_t i = 0; i < plans.size(); ++i) {
    if (subset && !(*subset)[i]) continue;
    const pl_plan* p = plans[i];
    const int c = batch_class(p->n[axis]);
    const BatchShape<T> sh = batch_shape<T>(p->n[axis], var[i]);
    const int h = p->g.h;
    const int ncols = axis == 0 ? p->n[1] * h : h;
    const int nslabs = axis == 0 ? 1 : p->n[0];
    const int nbx = (ncols + sh.B - 1) / sh.B;
    for (int sl = 0; sl < nslabs; ++sl)
      for (int t = 0; t < nbx; ++t) cls[c].push_back(make_int4((int)i, t, sl, t + nbx * sl));
    w.nb[i] = nbx * nslabs;
    w.threads[c] = std::max(w.threads[c], sh.col_threads);
    w.lds[c] = std::max(w.lds[c], sh.col_lds);
  }
  join_classes(w, cls);
  if (axis == 1) {
    // one rider item per instance (tile -1) at the end of the first class's
    // launch: the finalize that a y pass may carry (col_batch_kernel)
    std::vector<int4> riders;
    for (size_t i = 0; i < plans.size(); ++i)
      if (!subset || (*subset)[i]) riders.push_back(make_int4((int)i, -1, 0, 0));
    const bool first = w.split > 0;
    w.items.insert(w.items.begin() + (first ? w.split : (long)w.items.size()), riders.begin(), riders.end());
    if (first) w.split += (int)riders.size();
  }
}

// Row (z) pass over all instances, instance i in tile variant var[i].
template <typename T>
void row_work(const std::vector<pl_plan*>& plans, const std::vector<int>& var, BWork& w,
              const std::vector<int>* subset = nullptr) {
  std::vector<int4> cls[BATCH_CLASSES];
  w.nb.assign(plans.size(), 0);
  for (int c = 0; c < BATCH_CLASSES; ++c) w.threads[c] = w.lds[c] = 0;
  for (size_t i = 0; i < plans.size(); ++i) {
    if (subset && !(*subset)[i]) continue;
    const pl_plan* p = plans[i];
    const int c = batch_class(p->n[2]);
    const BatchShape<T> sh = batch_shape<T>(p->n[2], var[i]);
    const int nunits = p->n[0] * p->n[1] / 2;
    const int nbu = (nunits + sh.G - 1) / sh.G;
    for (int b = 0; b < nbu; ++b) cls[c].push_back(make_int4((int)i, b, 0, b));
    w.nb[i] = nbu;
    w.threads[c] = std::max(w.threads[c], sh.row_threads);
    w.lds[c] = std::max(w.lds[c], sh.row_lds);
  }
  join_classes(w, cls);
}

// Column / row pass kinds of a batched solve
enum BCol { BC_SHAT_Y = 0, BC_SHAT_X, BC_G_XINV, BC_G_YINV, BC_G_YFWD, BC_G_XADD, BC_COUNT64 };
enum BColT { BT_CG1 = 0, BT_CGYI, BT_CGYF, BT_CG5, BT_XCINV, BT_YCINV, BT_COUNT };
enum BRow { BR_R2C = 0, BR_GRAD, BR_COUNT64 };
enum BRowT { BRT_HVP = 0, BRT_C2R, BRT_COUNT };
enum BFin { BF_GRAD_ROW = 0, BF_GRAD_X, BF_INIT, BF_BETA, BF_LS, BF_COUNT };

}  // namespace

struct pl_batch {
  int K = 0;
  int precision = PL_FP64;
  hipStream_t user_stream = nullptr, stream = nullptr;
  hipEvent_t ev = nullptr;
  std::vector<pl_plan*> plans;
  std::vector<size_t> plan_off;
  size_t ws_bytes = 0, plans_bytes = 0, blob_bytes = 0;
  char* ws = nullptr;
  // work lists of the passes (BWorkId) and the tile variant of every
  // instance's column and row passes per precision ([0] FP64, [1] FP32),
  // chosen per grid length (pl_batch_autotune)
  BWork work[W_COUNT];
  std::vector<int> vcol[2], vrow[2];
  // device blob and its host mirror
  char* d_blob = nullptr;
  char* h_blob = nullptr;
  size_t off_c64 = 0, off_ct64 = 0, off_ct32 = 0, off_r64 = 0, off_rt64 = 0, off_rt32 = 0, off_fin = 0,
         off_e64 = 0, off_e32 = 0, off_ctl = 0, off_scal = 0;
  double* scal_all = nullptr;
  double* h_scal = nullptr;
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  // control records: composed in slot 0 of the host blob's control region,
  // uploaded from one of kCtlSlots staging slots in turn (bctl)
  int ctl_next = 0, ctl_unsynced = 0;
  int graph_chunk[2] = {0, 0}, graph_maxcg[2] = {0, 0};
  std::string err;
};

namespace {

int bfail(pl_batch* b, int code, const std::string& m) {
  if (b) b->err = m;
  return code;
}

#define BHIP(b, expr)                                                                              \
  do {                                                                                             \
    hipError_t _e = (expr);                                                                        \
    if (_e != hipSuccess) return bfail(b, PL_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

template <typename T>
T* blob_ptr(pl_batch* b, size_t off, bool host) {
  return (T*)((host ? b->h_blob : b->d_blob) + off);
}

// layout of the blob (work lists, args arrays, finalize arrays, elementwise
// args, control records, scalars)
size_t batch_layout(pl_batch* b) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t r = off;
    off += align_up(bytes);
    return r;
  };
  for (int i = 0; i < W_COUNT; ++i) b->work[i].off = take(sizeof(int4) * std::max<size_t>(1, b->work[i].cap));
  const size_t K = b->K;
  b->off_c64 = take(sizeof(ColArgs<double>) * K * BC_COUNT64);
  b->off_ct64 = take(sizeof(ColArgs<double>) * K * BT_COUNT);
  b->off_ct32 = take(sizeof(ColArgs<float>) * K * BT_COUNT);
  b->off_r64 = take(sizeof(RowArgs<double>) * K * BR_COUNT64);
  b->off_rt64 = take(sizeof(RowArgs<double>) * K * BRT_COUNT);
  b->off_rt32 = take(sizeof(RowArgs<float>) * K * BRT_COUNT);
  b->off_fin = take(sizeof(BatchFin) * K * BF_COUNT);
  b->off_e64 = take(sizeof(BatchElem<double>) * K);
  b->off_e32 = take(sizeof(BatchElem<float>) * K);
  b->off_ctl = take(sizeof(BatchCtl) * K * (1 + kCtlSlots));
  b->off_scal = take(sizeof(double) * K * SC_COUNT);
  return off;
}

template <typename T>
ColArgs<T>* cargs_t(pl_batch* b, int kind, bool host) {
  return blob_ptr<ColArgs<T>>(b, sizeof(T) == 8 ? b->off_ct64 : b->off_ct32, host) + (size_t)kind * b->K;
}
template <typename T>
RowArgs<T>* rargs_t(pl_batch* b, int kind, bool host) {
  return blob_ptr<RowArgs<T>>(b, sizeof(T) == 8 ? b->off_rt64 : b->off_rt32, host) + (size_t)kind * b->K;
}
ColArgs<double>* cargs64(pl_batch* b, int kind, bool host) {
  return blob_ptr<ColArgs<double>>(b, b->off_c64, host) + (size_t)kind * b->K;
}
RowArgs<double>* rargs64(pl_batch* b, int kind, bool host) {
  return blob_ptr<RowArgs<double>>(b, b->off_r64, host) + (size_t)kind * b->K;
}
BatchFin* fins(pl_batch* b, int kind, bool host) {
  return blob_ptr<BatchFin>(b, b->off_fin, host) + (size_t)kind * b->K;
}
template <typename T>
BatchElem<T>* elems(pl_batch* b, bool host) {
  return blob_ptr<BatchElem<T>>(b, sizeof(T) == 8 ? b->off_e64 : b->off_e32, host);
}
const int4* work_dev(pl_batch* b, int which) { return blob_ptr<int4>(b, b->work[which].off, false); }

// Work lists and launch shapes for the current tile variants, copied into
// the host blob (uploaded with the pass arguments before each solve).
void build_work(pl_batch* b) {
  col_work<double>(b->plans, 0, b->vcol[0], b->work[W_X64]);
  col_work<double>(b->plans, 1, b->vcol[0], b->work[W_Y64]);
  row_work<double>(b->plans, b->vrow[0], b->work[W_R64]);
  col_work<float>(b->plans, 0, b->vcol[1], b->work[W_X32]);
  col_work<float>(b->plans, 1, b->vcol[1], b->work[W_Y32]);
  row_work<float>(b->plans, b->vrow[1], b->work[W_R32]);
  if (b->h_blob)
    for (int i = 0; i < W_COUNT; ++i)
      if (!b->work[i].items.empty())
        std::memcpy(b->h_blob + b->work[i].off, b->work[i].items.data(), sizeof(int4) * b->work[i].items.size());
}

// The CG passes' work lists over the instances in `subset` (W_XC, W_YC,
// W_RC), copied to the device on the batch's stream.
template <typename T>
int build_compact(pl_batch* b, const std::vector<int>& subset) {
  const int ti = sizeof(T) == 8 ? 0 : 1;
  col_work<T>(b->plans, 0, b->vcol[ti], b->work[W_XC], &subset);
  col_work<T>(b->plans, 1, b->vcol[ti], b->work[W_YC], &subset);
  row_work<T>(b->plans, b->vrow[ti], b->work[W_RC], &subset);
  for (int i : {(int)W_XC, (int)W_YC, (int)W_RC}) {
    BWork& w = b->work[i];
    if (w.items.empty() || w.items.size() > w.cap) return PL_ERR_INVALID_ARG;
    std::memcpy(b->h_blob + w.off, w.items.data(), sizeof(int4) * w.items.size());
    BHIP(b, hipMemcpyAsync(b->d_blob + w.off, b->h_blob + w.off, sizeof(int4) * w.items.size(),
                           hipMemcpyHostToDevice, b->stream));
  }
  return PL_OK;
}

template <typename T>
int wid_x() { return sizeof(T) == 8 ? W_X64 : W_X32; }
template <typename T>
int wid_y() { return sizeof(T) == 8 ? W_Y64 : W_Y32; }
template <typename T>
int wid_r() { return sizeof(T) == 8 ? W_R64 : W_R32; }

// One batched column / row pass over work list `wid`: one launch per length
// class present.
template <typename T>
hipError_t bcol(pl_batch* b, bool inverse, int op, const ColArgs<T>* args, int wid) {
  const BWork& w = b->work[wid];
  const int count[2] = {w.split, (int)w.items.size() - w.split};
  for (int c = 0, first = 0; c < BATCH_CLASSES; first += count[c], ++c) {
    if (count[c] == 0) continue;
    hipError_t e = launch_col_batch<T>(inverse, op, c, args, work_dev(b, wid) + first, count[c], w.threads[c],
                                       w.lds[c], b->stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
template <typename T>
hipError_t brow(pl_batch* b, int op, const RowArgs<T>* args, int wid) {
  const BWork& w = b->work[wid];
  const int count[2] = {w.split, (int)w.items.size() - w.split};
  for (int c = 0, first = 0; c < BATCH_CLASSES; first += count[c], ++c) {
    if (count[c] == 0) continue;
    hipError_t e = launch_row_batch<T>(op, c, args, work_dev(b, wid) + first, count[c], w.threads[c], w.lds[c],
                                       b->stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Fill the per-instance pass arguments (depends on the caller's s pointers).
template <typename T>
void fill_args(pl_batch* b, double* const* s_io) {
  for (int i = 0; i < b->K; ++i) {
    pl_plan* p = b->plans[i];
    const double* inactive = p->scal + SC_INACTIVE;
    const double* done = p->scal + SC_DONE;
    // FP64 gradient and transforms of s
    const int v64 = b->vcol[0][i], r64 = b->vrow[0][i];
    const int vT = b->vcol[sizeof(T) == 4 ? 1 : 0][i], rT = b->vrow[sizeof(T) == 4 ? 1 : 0][i];
    ColArgs<double>* c;
    c = &cargs64(b, BC_SHAT_Y, true)[i]; *c = col_args<double>(p, 1, p->s_hat, p->s_hat); c->skip = inactive;
    c->variant = v64;
    c = &cargs64(b, BC_SHAT_X, true)[i]; *c = col_args<double>(p, 0, p->s_hat, p->s_hat); c->skip = inactive;
    c->variant = v64;
    c = &cargs64(b, BC_G_XINV, true)[i]; *c = col_args<double>(p, 0, p->s_hat, p->t64); c->skip = inactive;
    c->variant = v64;
    c = &cargs64(b, BC_G_YINV, true)[i]; *c = col_args<double>(p, 1, p->t64, p->t64); c->skip = inactive;
    c->variant = v64;
    c = &cargs64(b, BC_G_YFWD, true)[i]; *c = col_args<double>(p, 1, p->t64, p->t64); c->skip = inactive;
    c->variant = v64;
    c = &cargs64(b, BC_G_XADD, true)[i]; *c = col_args<double>(p, 0, p->t64, p->g_hat); c->skip = inactive;
    c->variant = v64;
    // the batch's x passes read the shell table of a radial spectrum (a few
    // KB to 60 KB for these grids, cached), else the per-mode one
    c->radial = p->radial ? TAB_SHELL : TAB_MODE;
    c->inv_lam = View<double>::tab(p, p->radial);
    c->base = p->s_hat;
    c->k0_shift = (double)p->N * p->prob.mu;
    RowArgs<double>* r;
    r = &rargs64(b, BR_R2C, true)[i]; *r = row_args<double>(p); r->in_r = s_io[i]; r->out_c = p->s_hat; r->skip = inactive;
    r->variant = r64;
    r = &rargs64(b, BR_GRAD, true)[i]; *r = row_args<double>(p); r->in_c = p->t64; r->out_c = p->t64;
    r->s_out = s_io[i]; r->e_out = p->e; r->d_out = p->d; r->skip = inactive;
    r->variant = r64;
    // Krylov passes in T
    cx<T>*x = View<T>::x(p), *rr = View<T>::r(p), *pp = View<T>::pv(p), *t = View<T>::t(p);
    double* part_a = p->partials;
    double* part_b = p->partials + p->partials_len;
    double* part_c = p->partials + 2 * p->partials_len;  // the last pass's (r^H r, r^H M^-1 r)
    ColArgs<T>* ct;
    ct = &cargs_t<T>(b, BT_CG1, true)[i]; *ct = col_args<T>(p, 0, pp, t);
    ct->cg_r = rr; ct->scal = p->scal; ct->partials = part_a; ct->skip = done; ct->variant = vT;
    // the first pass closes the previous iteration itself (beta, the
    // convergence test, the bookkeeping) from the last pass's partials, at
    // the iteration count in SC_ITS (cg_max is set per solve)
    ct->beta_part = part_c;
    ct->beta_scale = 1.0 / (double)p->N;
    ct->radial = p->radial ? TAB_SHELL : TAB_MODE;
    ct->inv_lam = View<T>::tab(p, p->radial);
    ct = &cargs_t<T>(b, BT_CGYI, true)[i]; *ct = col_args<T>(p, 1, t, t); ct->skip = done; ct->variant = vT;
    ct = &cargs_t<T>(b, BT_CGYF, true)[i]; *ct = col_args<T>(p, 1, t, t); ct->skip = done; ct->variant = vT;
    ct = &cargs_t<T>(b, BT_CG5, true)[i]; *ct = col_args<T>(p, 0, t, t);
    ct->base = pp; ct->cg_r = rr; ct->cg_x = x; ct->scal = p->scal; ct->partials = part_c; ct->skip = done;
    ct->variant = vT;  // (the last pass advances SC_ITS after each iteration)
    ct->radial = p->radial ? TAB_SHELL : TAB_MODE;
    ct->inv_lam = View<T>::tab(p, p->radial);
    ct = &cargs_t<T>(b, BT_XCINV, true)[i]; *ct = col_args<T>(p, 0, x, t); ct->skip = inactive; ct->variant = vT;
    ct = &cargs_t<T>(b, BT_YCINV, true)[i]; *ct = col_args<T>(p, 1, t, t); ct->skip = inactive; ct->variant = vT;
    RowArgs<T>* rt;
    rt = &rargs_t<T>(b, BRT_HVP, true)[i]; *rt = row_args<T>(p); rt->in_c = t; rt->out_c = t;
    rt->partials = part_b; rt->skip = done; rt->variant = rT;
    rt = &rargs_t<T>(b, BRT_C2R, true)[i]; *rt = row_args<T>(p); rt->in_c = t; rt->out_r = View<T>::preal(p);
    rt->skip = inactive; rt->variant = rT;
    // finalize records
    const std::vector<int>& nbx = b->work[wid_x<T>()].nb;
    const std::vector<int>& nbr = b->work[wid_r<T>()].nb;
    const double invN = 1.0 / (double)p->N;
    fins(b, BF_GRAD_ROW, true)[i] = BatchFin{part_a, b->work[W_R64].nb[i], nullptr, 0, p->scal, invN};
    fins(b, BF_GRAD_X, true)[i] = BatchFin{part_a, b->work[W_X64].nb[i], nullptr, 0, p->scal, invN};
    fins(b, BF_INIT, true)[i] = BatchFin{part_a, NBB, nullptr, 0, p->scal, invN};
    // alpha = r^H z / p^H H p, finalized by a rider of the forward y pass
    ColArgs<T>* cyf = &cargs_t<T>(b, BT_CGYF, true)[i];
    cyf->fin_on = 1;
    cyf->fin = FinArgs{part_b, nbr[i], 2, FIN_CG_ALPHA, 0, 1.0, p->scal, -1.0, part_a, nbx[i], invN};
    fins(b, BF_BETA, true)[i] = BatchFin{part_c, nbx[i], nullptr, 0, p->scal, invN};
    cargs_t<T>(b, BT_CG1, true)[i].beta_nb = nbx[i];
    fins(b, BF_LS, true)[i] = BatchFin{part_a, NBB, nullptr, 0, p->scal, invN};
  }
}

// The CG iteration cap the batched first pass tests (per solve; the host
// blob is uploaded after this).
template <typename T>
void set_cg_max(pl_batch* b, int max_cg) {
  for (int i = 0; i < b->K; ++i) cargs_t<T>(b, BT_CG1, true)[i].cg_max = (double)max_cg;
}

int bfin(pl_batch* b, int which, int K, int kind, int dst, double scale, int scale_invN, double aux = 0.0,
         double scale2 = 0.0, int scale2_invN = 0) {
  hipLaunchKernelGGL(finalize_batch_kernel, dim3(b->K), dim3(256), 0, b->stream, fins(b, which, false), K, kind,
                     dst, scale, scale_invN, aux, scale2, scale2_invN);
  BHIP(b, hipGetLastError());
  return PL_OK;
}

int bread(pl_batch* b) {
  BHIP(b, hipMemcpyAsync(b->h_scal, b->scal_all, sizeof(double) * SC_COUNT * b->K, hipMemcpyDeviceToHost,
                         b->stream));
  BHIP(b, hipStreamSynchronize(b->stream));
  b->ctl_unsynced = 0;  // every queued upload has completed
  return PL_OK;
}

double& hs(pl_batch* b, int i, int slot) { return b->h_scal[(size_t)i * SC_COUNT + slot]; }

// Upload the control records composed in slot 0 and apply them.  The
// upload goes through the next of kCtlSlots pinned staging slots, so the
// caller may compose the next records at once; a staging slot is written
// again only after its copy has completed (the stream is synchronized once
// kCtlSlots uploads are outstanding; every read-back also completes them).
int bctl(pl_batch* b) {
  const size_t K = b->K;
  if (b->ctl_unsynced >= kCtlSlots) {
    BHIP(b, hipStreamSynchronize(b->stream));
    b->ctl_unsynced = 0;
  }
  const int slot = 1 + b->ctl_next;
  b->ctl_next = (b->ctl_next + 1) % kCtlSlots;
  ++b->ctl_unsynced;
  BatchCtl* hc = blob_ptr<BatchCtl>(b, b->off_ctl, true);
  BatchCtl* hs_slot = hc + (size_t)slot * K;
  BatchCtl* ds_slot = blob_ptr<BatchCtl>(b, b->off_ctl, false) + (size_t)slot * K;
  std::memcpy(hs_slot, hc, sizeof(BatchCtl) * K);
  BHIP(b, hipMemcpyAsync(ds_slot, hs_slot, sizeof(BatchCtl) * K, hipMemcpyHostToDevice, b->stream));
  hipLaunchKernelGGL(batch_ctl_kernel, dim3((b->K + 63) / 64), dim3(64), 0, b->stream, ds_slot, b->K);
  BHIP(b, hipGetLastError());
  return PL_OK;
}

template <typename T>
int belem_upload(pl_batch* b) {
  BHIP(b, hipMemcpyAsync(elems<T>(b, false), elems<T>(b, true), sizeof(BatchElem<T>) * b->K,
                         hipMemcpyHostToDevice, b->stream));
  return PL_OK;
}

int bgrad(pl_batch* b) {
  BHIP(b, bcol<double>(b, true, COL_PLAIN, cargs64(b, BC_G_XINV, false), W_X64));
  BHIP(b, bcol<double>(b, true, COL_PLAIN, cargs64(b, BC_G_YINV, false), W_Y64));
  BHIP(b, brow<double>(b, ROW_GRAD, rargs64(b, BR_GRAD, false), W_R64));
  int rc = bfin(b, BF_GRAD_ROW, 2, FIN_STORE, SC_LIK, 1.0, 0);
  if (rc) return rc;
  BHIP(b, bcol<double>(b, false, COL_PLAIN, cargs64(b, BC_G_YFWD, false), W_Y64));
  BHIP(b, bcol<double>(b, false, COL_ADDPRIOR, cargs64(b, BC_G_XADD, false), W_X64));
  return bfin(b, BF_GRAD_X, 3, FIN_STORE, SC_GG - 1, 0.0, 1);
}

// Enqueue `chunk` fused CG steps for all instances (captured in a graph)
template <typename T>
int bcg_chunk(pl_batch* b, int chunk, int max_cg, int wx = wid_x<T>(), int wy = wid_y<T>(), int wr = wid_r<T>()) {
  for (int k = 0; k < chunk; ++k) {
    BHIP(b, bcol<T>(b, true, COL_CG_FIRST, cargs_t<T>(b, BT_CG1, false), wx));
    BHIP(b, bcol<T>(b, true, COL_PLAIN, cargs_t<T>(b, BT_CGYI, false), wy));
    BHIP(b, brow<T>(b, ROW_HVP, rargs_t<T>(b, BRT_HVP, false), wr));
    // the forward y pass carries the alpha finalize (a rider per instance)
    BHIP(b, bcol<T>(b, false, COL_PLAIN, cargs_t<T>(b, BT_CGYF, false), wy));
    BHIP(b, bcol<T>(b, false, COL_CG_LAST, cargs_t<T>(b, BT_CG5, false), wx));
  }
  // the next first pass closes each iteration; after the chunk one finalize
  // closes the last for the host's check (the next chunk's first pass
  // repeats it, to the same values)
  return bfin(b, BF_BETA, 2, FIN_CG_BETA_DEV, 0, 0.0, 1, (double)max_cg);
}

template <typename T>
int batch_newton(pl_batch* b, double* const* s_io, const pl_solve_opts& o, pl_solve_info* infos) {
  const int K = b->K;
  const int ti = sizeof(T) == 8 ? 0 : 1;
  fill_args<T>(b, s_io);
  set_cg_max<T>(b, o.max_cg);
  BHIP(b, hipMemcpyAsync(b->d_blob, b->h_blob, b->off_e64, hipMemcpyHostToDevice, b->stream));
  BatchCtl* ctl = blob_ptr<BatchCtl>(b, b->off_ctl, true);
  BatchElem<T>* E = elems<T>(b, true);
  std::vector<pl_solve_info> inf(K);
  std::vector<int> active(K, 1);
  std::vector<double> g0(K, 0.0), gn(K, 0.0);
  for (int i = 0; i < K; ++i) {
    ctl[i] = BatchCtl{b->plans[i]->scal, 0, 0, 0.0, 0.0, 0, 0, 1, 1};
  }
  int rc = bctl(b);
  if (rc) return rc;
  // s_hat = F s0, then the gradient
  BHIP(b, brow<double>(b, ROW_R2C, rargs64(b, BR_R2C, false), W_R64));
  BHIP(b, bcol<double>(b, false, COL_PLAIN, cargs64(b, BC_SHAT_Y, false), W_Y64));
  BHIP(b, bcol<double>(b, false, COL_PLAIN, cargs64(b, BC_SHAT_X, false), W_X64));
  rc = bgrad(b);
  if (rc) return rc;
  rc = bread(b);
  if (rc) return rc;
  for (int i = 0; i < K; ++i) {
    g0[i] = gn[i] = std::sqrt(std::max(0.0, hs(b, i, SC_GG)));
    inf[i].grad0 = g0[i];
    inf[i].obj = 0.5 * hs(b, i, SC_PRIOR) + hs(b, i, SC_LIK);
    if (!std::isfinite(g0[i])) {
      inf[i].status = PL_ERR_DOMAIN;
      active[i] = 0;
    } else if (g0[i] == 0.0) {
      active[i] = 0;
    }
  }
  // graph of one chunk of CG steps (built on first use, replayed afterwards)
  if (!b->graph[ti] || b->graph_chunk[ti] != o.check_every || b->graph_maxcg[ti] != o.max_cg) {
    if (b->graph[ti]) {
      (void)hipGraphExecDestroy(b->graph[ti]);
      b->graph[ti] = nullptr;
    }
    hipGraph_t g = nullptr;
    BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    int crc = bcg_chunk<T>(b, o.check_every, o.max_cg);
    hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (crc) return crc;
    BHIP(b, e);
    BHIP(b, hipGraphInstantiate(&b->graph[ti], g, nullptr, nullptr, 0));
    (void)hipGraphDestroy(g);
    b->graph_chunk[ti] = o.check_every;
    b->graph_maxcg[ti] = o.max_cg;
  }
  // Each instance advances on its own: a round runs (1) the line search,
  // update and gradient of the instances whose CG ended in the previous
  // round, (2) the CG start of those that go on, (3) one graph-replayed
  // chunk of CG steps for every instance in its CG.  SC_INACTIVE masks the
  // instances a phase does not concern (the transform passes and the
  // finalizes skip them), SC_DONE the CG passes; so an instance whose CG
  // ends early takes its next Newton step while the others' CG runs on.
  enum { PH_OFF = 0, PH_START, PH_CG, PH_STEP };
  std::vector<int> phase(K, PH_OFF), newton(K, 0);
  // the CG chunks run from the graph over every instance until the cells of
  // the unfinished ones fall to half of those it covers; then as direct
  // launches over work lists of the unfinished instances only (rebuilt each
  // time their cells halve again)
  const hipGraphExec_t cg_graph = b->graph[ti];
  bool compacted = false;
  double graph_cells = 0.0;
  for (int i = 0; i < K; ++i) graph_cells += (double)b->plans[i]->N;
  for (int i = 0; i < K; ++i) {
    if (!active[i]) continue;
    if (gn[i] <= o.rtol * g0[i]) {
      active[i] = 0;
    } else if (o.max_newton <= 0) {
      active[i] = 0;
      inf[i].status = PL_ERR_NOT_CONVERGED;
    } else {
      phase[i] = PH_START;
    }
  }
  // mask: SC_INACTIVE = !in[i]; optionally SC_DONE and SC_TOL2 too
  auto apply_mask = [&](const std::vector<int>& in) -> int {
    for (int i = 0; i < K; ++i) {
      ctl[i] = BatchCtl{b->plans[i]->scal, 0, 0, in[i] ? 0.0 : 1.0, 1.0, 0, 0, 1, phase[i] == PH_OFF ? 1 : 0};
    }
    return bctl(b);
  };
  auto fill_elems = [&](const std::vector<int>& in) {
    for (int i = 0; i < K; ++i) {
      pl_plan* p = b->plans[i];
      BatchElem<T> e{};
      e.active = in[i];
      e.nh = p->Nh;
      e.n = p->N;
      e.g = p->g;
      e.radial = p->radial;
      e.tab = View<T>::tab(p, p->radial);
      e.tab64 = p->radial ? p->tab_rad : p->tab_mode;
      e.rhs = p->g_hat;
      e.sign = -1.0;
      e.x = View<T>::x(p);
      e.r = View<T>::r(p);
      e.p = View<T>::pv(p);
      e.s_hat = p->s_hat;
      e.g_hat = p->g_hat;
      e.k0_shift = (double)p->N * p->prob.mu;
      e.preal = View<T>::preal(p);
      e.e = p->e;
      e.counts = p->prob.counts;
      e.beta = p->prob.beta;
      e.a0 = 1.0;
      e.y = p->s_hat;
      e.alpha = 0.0;
      e.d = p->d;
      e.d32 = p->d32;
      e.scal = p->scal;
      e.scal_rw = p->scal;
      e.partials = p->partials;
      e.hist = p->hist;
      E[i] = e;
    }
  };
  auto retire = [&](int i, int status) {
    phase[i] = PH_OFF;
    active[i] = 0;
    if (status != PL_OK) inf[i].status = status;
  };
  for (;;) {
    Range range("pl batch round");
    std::vector<int> in(K, 0);
    // (1) line search, update and gradient of the instances whose CG ended
    bool any = false;
    for (int i = 0; i < K; ++i) {
      in[i] = phase[i] == PH_STEP;
      any = any || in[i];
    }
    if (any) {
      // queued without a read-back: the direction in real space, the line
      // search's dots, its first batch of trial steps (a = 1 .. 1/8), the
      // Armijo pick and the update on the device, then the gradient
      rc = apply_mask(in);
      if (rc) return rc;
      fill_elems(in);
      rc = belem_upload<T>(b);
      if (rc) return rc;
      BHIP(b, bcol<T>(b, true, COL_PLAIN, cargs_t<T>(b, BT_XCINV, false), wid_x<T>()));
      BHIP(b, bcol<T>(b, true, COL_PLAIN, cargs_t<T>(b, BT_YCINV, false), wid_y<T>()));
      BHIP(b, brow<T>(b, ROW_C2R, rargs_t<T>(b, BRT_C2R, false), wid_r<T>()));
      hipLaunchKernelGGL((ls_dots_batch_kernel<T>), dim3(NBB, K), dim3(RED_THREADS), 0, b->stream,
                         elems<T>(b, false));
      BHIP(b, hipGetLastError());
      rc = bfin(b, BF_LS, 3, FIN_STORE, SC_LS_B, 0.0, 1);
      if (rc) return rc;
      hipLaunchKernelGGL((ls_eval_batch_kernel<T>), dim3(NBB, K), dim3(RED_THREADS), 0, b->stream,
                         elems<T>(b, false));
      BHIP(b, hipGetLastError());
      rc = bfin(b, BF_LS, 4, FIN_STORE, SC_DF, 1.0, 0);
      if (rc) return rc;
      hipLaunchKernelGGL((ls_select_batch_kernel<T>), dim3(K), dim3(64), 0, b->stream, elems<T>(b, false),
                         o.ls_c1);
      BHIP(b, hipGetLastError());
      hipLaunchKernelGGL((axpy_batch_dev_kernel<T>), dim3(NBB, K), dim3(RED_THREADS), 0, b->stream,
                         elems<T>(b, false));
      BHIP(b, hipGetLastError());
      rc = bgrad(b);
      if (rc) return rc;
      rc = bread(b);
      if (rc) return rc;
      // an instance whose first batch accepted no step along a descent
      // direction backtracks on the host (batches from 1/16; its iterate,
      // real direction and linearisation are unchanged); one that is not a
      // descent direction stops
      std::vector<double> alpha(K, -1.0), a0(K, 1.0 / 16.0);
      std::vector<int> pending(K, 0);
      bool anyp = false;
      for (int i = 0; i < K; ++i) {
        if (!in[i]) continue;
        alpha[i] = hs(b, i, SC_LS_ALPHA);
        if (alpha[i] > 0.0) continue;
        if (hs(b, i, SC_LS_SLOPE) < 0.0) {
          pending[i] = 1;
          anyp = true;
        } else {
          retire(i, PL_ERR_LINESEARCH);
          in[i] = 0;
        }
      }
      if (anyp) {
        std::vector<int> redo = pending;
        for (int batch = 1; batch < 8; ++batch) {
          anyp = false;
          for (int i = 0; i < K; ++i) {
            E[i].active = pending[i];
            E[i].a0 = a0[i];
            anyp = anyp || pending[i];
          }
          if (!anyp) break;
          rc = belem_upload<T>(b);
          if (rc) return rc;
          hipLaunchKernelGGL((ls_eval_batch_kernel<T>), dim3(NBB, K), dim3(RED_THREADS), 0, b->stream,
                             elems<T>(b, false));
          BHIP(b, hipGetLastError());
          rc = bfin(b, BF_LS, 4, FIN_STORE, SC_DF, 1.0, 0);
          if (rc) return rc;
          rc = bread(b);
          if (rc) return rc;
          for (int i = 0; i < K; ++i) {
            if (!pending[i]) continue;
            const double bb = hs(b, i, SC_LS_B), cc = hs(b, i, SC_LS_C), slope = hs(b, i, SC_LS_SLOPE);
            double a = a0[i];
            for (int j = 0; j < 4; ++j, a *= 0.5) {
              const double df = a * bb + 0.5 * a * a * cc + hs(b, i, SC_DF + j);
              if (df <= o.ls_c1 * a * slope) {
                alpha[i] = a;
                pending[i] = 0;
                break;
              }
            }
            a0[i] *= 1.0 / 16.0;
          }
        }
        std::vector<int> stepped(K, 0);
        bool anys = false;
        for (int i = 0; i < K; ++i) {
          if (!redo[i]) continue;
          if (alpha[i] > 0.0) {
            stepped[i] = 1;
            anys = true;
          } else {
            retire(i, PL_ERR_LINESEARCH);
            in[i] = 0;
          }
        }
        if (anys) {
          for (int i = 0; i < K; ++i) {
            E[i].active = stepped[i];
            E[i].alpha = alpha[i];
          }
          rc = belem_upload<T>(b);
          if (rc) return rc;
          hipLaunchKernelGGL((axpy_batch_kernel<T>), dim3(NBB, K), dim3(RED_THREADS), 0, b->stream,
                             elems<T>(b, false));
          BHIP(b, hipGetLastError());
          rc = apply_mask(stepped);
          if (rc) return rc;
          rc = bgrad(b);
          if (rc) return rc;
          rc = bread(b);
          if (rc) return rc;
        }
      }
      for (int i = 0; i < K; ++i) {
        if (!in[i]) continue;
        gn[i] = std::sqrt(std::max(0.0, hs(b, i, SC_GG)));
        inf[i].obj = 0.5 * hs(b, i, SC_PRIOR) + hs(b, i, SC_LIK);
        inf[i].newton_its = ++newton[i];
        if (!std::isfinite(gn[i]))
          retire(i, PL_ERR_DOMAIN);
        else if (gn[i] <= o.rtol * g0[i])
          retire(i, PL_OK);
        else if (newton[i] >= o.max_newton)
          retire(i, PL_ERR_NOT_CONVERGED);
        else
          phase[i] = PH_START;
      }
    }
    // (2) CG start: preconditioner constant, tolerance, initial residual
    any = false;
    for (int i = 0; i < K; ++i) {
      in[i] = phase[i] == PH_START;
      any = any || in[i];
    }
    if (any) {
      for (int i = 0; i < K; ++i) {
        ctl[i] = BatchCtl{b->plans[i]->scal, 0, 0, in[i] ? 0.0 : 1.0, 1.0, 0, 0, 1, phase[i] == PH_OFF ? 1 : 0};
        if (in[i]) {
          const double eta =
              std::min(o.eta_max, std::max(std::sqrt(gn[i] / g0[i]), 0.5 * o.rtol * g0[i] / gn[i]));
          ctl[i].tol2 = eta * gn[i] * eta * gn[i];
          ctl[i].set_tol2 = 1;
        }
      }
      rc = bctl(b);
      if (rc) return rc;
      fill_elems(in);
      rc = belem_upload<T>(b);
      if (rc) return rc;
      hipLaunchKernelGGL((dquant_hist_batch_kernel<T>), dim3(NBB, K), dim3(RED_THREADS), 0, b->stream,
                         elems<T>(b, false));
      BHIP(b, hipGetLastError());
      hipLaunchKernelGGL((dquant_select_batch_kernel<T>), dim3(K), dim3(DQ_SELECT_THREADS), 0, b->stream,
                         elems<T>(b, false));
      BHIP(b, hipGetLastError());
      if constexpr (sizeof(T) == 4) {
        hipLaunchKernelGGL((d32_batch_kernel<T>), dim3(NBB, K), dim3(RED_THREADS), 0, b->stream, elems<T>(b, false));
        BHIP(b, hipGetLastError());
      }
      hipLaunchKernelGGL((cg_init_batch_kernel<T>), dim3(NBB, K), dim3(RED_THREADS), 0, b->stream,
                         elems<T>(b, false));
      BHIP(b, hipGetLastError());
      rc = bfin(b, BF_INIT, 2, FIN_CG_INIT, 0, 0.0, 1);
      if (rc) return rc;
      for (int i = 0; i < K; ++i)
        if (in[i]) phase[i] = PH_CG;
    }
    // (3) one chunk of CG steps for every instance in its CG
    any = false;
    for (int i = 0; i < K; ++i) {
      in[i] = phase[i] == PH_CG;
      any = any || in[i];
    }
    if (!any) break;  // every instance retired
    rc = apply_mask(in);
    if (rc) return rc;
    {
      std::vector<int> unfinished(K, 0);
      double cells = 0.0;
      for (int i = 0; i < K; ++i)
        if (phase[i] != PH_OFF) {
          unfinished[i] = 1;
          cells += (double)b->plans[i]->N;
        }
      if (cells <= 0.5 * graph_cells) {
        rc = build_compact<T>(b, unfinished);
        if (rc) return bfail(b, rc, "compacted work lists exceed their capacity");
        compacted = true;
        graph_cells = cells;
      }
    }
    // the full work lists replay their graph; compacted ones (rebuilt a few
    // times per solve) are launched directly: capturing and instantiating a
    // graph for each would keep the GPU idle while the host does it, where
    // direct launches are issued while the GPU runs the previous ones
    if (compacted) {
      rc = bcg_chunk<T>(b, o.check_every, o.max_cg, W_XC, W_YC, W_RC);
      if (rc) return rc;
    } else {
      BHIP(b, hipGraphLaunch(cg_graph, b->stream));
    }
    rc = bread(b);
    if (rc) return rc;
    for (int i = 0; i < K; ++i) {
      if (!in[i] || hs(b, i, SC_DONE) == 0.0) continue;
      const int its = (int)hs(b, i, SC_ITS);
      inf[i].cg_its += its;
      inf[i].hvps += its + (hs(b, i, SC_DONE) == 2.0 ? 1 : 0);
      phase[i] = PH_STEP;
    }
  }
  if constexpr (sizeof(T) == 4) {
    // instances whose FP32 directions stalled in the line search continue
    // from their current iterate with FP64 inner solves
    for (int i = 0; i < K; ++i) {
      if (inf[i].status != PL_ERR_LINESEARCH) continue;
      BHIP(b, hipStreamSynchronize(b->stream));
      pl_solve_info r{};
      pl_solve_opts o2 = o;
      o2.max_newton = std::max(0, o.max_newton - inf[i].newton_its);
      // same stopping point: rtol relative to the original starting gradient
      o2.rtol = gn[i] > 0.0 ? o.rtol * g0[i] / gn[i] : o.rtol;
      const int rc2 = newton_solve<double>(b->plans[i], s_io[i], o2, &r);
      if (rc2 != PL_OK && rc2 != PL_ERR_NOT_CONVERGED && rc2 != PL_ERR_LINESEARCH) return bfail(b, rc2, pl_last_error(b->plans[i]));
      const double gfin = r.rel_grad * r.grad0;
      gn[i] = gfin;
      inf[i].cg_its += r.cg_its;
      inf[i].hvps += r.hvps;
      inf[i].newton_its += r.newton_its;
      inf[i].fp64_steps += r.newton_its;
      inf[i].obj = r.obj;
      inf[i].status = gfin <= o.rtol * g0[i] ? PL_OK : (rc2 != PL_OK ? rc2 : PL_ERR_NOT_CONVERGED);
    }
  }
  int first_bad = PL_OK;
  for (int i = 0; i < K; ++i) {
    inf[i].rel_grad = g0[i] > 0.0 ? gn[i] / g0[i] : 0.0;
    if (infos) infos[i] = inf[i];
    if (inf[i].status != PL_OK && first_bad == PL_OK) first_bad = inf[i].status;
  }
  BHIP(b, hipStreamSynchronize(b->stream));
  return first_bad;
}

// Time one batched CG step (the seven launches of bcg_chunk over every
// instance) with the current tile variants, average of `reps`; on hashed
// Krylov vectors and Hessian diagonals, so nothing is left in a meaningful
// state.
template <typename T>
int time_batch_cg(pl_batch* b, int reps, float* ms) {
  build_work(b);
  std::vector<double*> dummy(b->K);
  for (int i = 0; i < b->K; ++i) dummy[i] = b->plans[i]->s_ws;
  fill_args<T>(b, dummy.data());
  const int big = 1 << 30;
  set_cg_max<T>(b, big);
  BHIP(b, hipMemcpyAsync(b->d_blob, b->h_blob, b->off_e64, hipMemcpyHostToDevice, b->stream));
  for (int i = 0; i < b->K; ++i) {
    pl_plan* p = b->plans[i];
    int rc = fill_hash<T>(p, (T*)View<T>::x(p), 2 * p->Nh, 1);
    if (!rc) rc = fill_hash<T>(p, (T*)View<T>::r(p), 2 * p->Nh, 2);
    if (!rc) rc = fill_hash<T>(p, (T*)View<T>::pv(p), 2 * p->Nh, 3);
    if (rc) return bfail(b, rc, pl_last_error(p));
  }
  BHIP(b, hipMemsetAsync(b->scal_all, 0, sizeof(double) * SC_COUNT * b->K, b->stream));
  int rc = bcg_chunk<T>(b, 2, big);
  if (rc) return rc;
  hipEvent_t e0, e1;
  BHIP(b, hipEventCreate(&e0));
  BHIP(b, hipEventCreate(&e1));
  (void)hipEventRecord(e0, b->stream);
  rc = bcg_chunk<T>(b, reps, big);
  (void)hipEventRecord(e1, b->stream);
  (void)hipEventSynchronize(e1);
  (void)hipEventElapsedTime(ms, e0, e1);
  *ms /= (float)reps;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

// Distinct grid lengths of a batch (each instance's three axes must be
// equal to share a column/row variant per length), the ones holding the
// most cells first.
std::vector<int> batch_lengths(const pl_batch* b) {
  std::vector<std::pair<long, int>> tot;
  for (const pl_plan* p : b->plans)
    for (int a = 0; a < 3; ++a) {
      const int n = p->n[a];
      auto it = std::find_if(tot.begin(), tot.end(), [n](const std::pair<long, int>& q) { return q.second == n; });
      if (it == tot.end())
        tot.push_back({p->N, n});
      else
        it->first += p->N;
    }
  std::sort(tot.begin(), tot.end(), [](const std::pair<long, int>& a, const std::pair<long, int>& c) {
    return a.first != c.first ? a.first > c.first : a.second < c.second;
  });
  std::vector<int> out;
  for (auto& q : tot) out.push_back(q.second);
  return out;
}

// Per length L: the tile variant of the column passes and of the row pass
// of every instance whose axes have length L (an instance with uneven axes
// takes the variant of its x length).
void set_length_variant(pl_batch* b, int ti, int L, int vc, int vr) {
  for (int i = 0; i < b->K; ++i)
    if (b->plans[i]->n[0] == L) {
      b->vcol[ti][i] = vc;
      b->vrow[ti][i] = vr;
    }
}

template <typename T>
int tune_batch_precision(pl_batch* b, const std::string& key, const std::vector<int>& lens,
                         std::vector<std::string>& lines, bool* added) {
  const int ti = sizeof(T) == 4 ? 1 : 0;
  const size_t nl = lens.size();
  for (const std::string& line : lines) {
    if (line.compare(0, key.size() + 1, key + " ") != 0) continue;
    // "<key> c0,c1,... r0,r1,... ms"
    std::vector<int> vc, vr;
    const char* q = line.c_str() + key.size();
    for (int part = 0; part < 2; ++part) {
      std::vector<int>& dst = part == 0 ? vc : vr;
      while (*q == ' ') ++q;
      while (*q && *q != ' ') {
        char* end = nullptr;
        long v = std::strtol(q, &end, 10);
        if (end == q) break;
        dst.push_back((int)v);
        q = end;
        if (*q == ',') ++q;
      }
    }
    if (vc.size() != nl || vr.size() != nl) continue;
    bool ok = true;
    for (size_t j = 0; j < nl; ++j) ok = ok && (vc[j] == 0 || vc[j] == 2) && (vr[j] == 0 || vr[j] == 2);
    if (!ok) continue;
    for (size_t j = 0; j < nl; ++j) set_length_variant(b, ti, lens[j], vc[j], vr[j]);
    return PL_OK;
  }
  // a positive Hessian diagonal for the timing runs
  for (pl_plan* p : b->plans) {
    int rc = fill_hash<double>(p, p->d, p->N, 5, 0.0, 1.0);
    if (!rc && sizeof(T) == 4) rc = fill_hash<float>(p, p->d32, p->N, 5, 0.0, 1.0);
    if (rc) return bfail(b, rc, pl_last_error(p));
    p->d_valid = false;
    p->d32_valid = false;
  }
  const int reps = 10;
  float best = 0.f;
  for (size_t j = 0; j < nl; ++j) set_length_variant(b, ti, lens[j], 0, 0);
  int rc = time_batch_cg<T>(b, reps, &best);
  if (rc) return rc;
  std::vector<int> kc(nl, 0), kr(nl, 0);
  // one length at a time, the lengths holding the most cells first
  for (size_t j = 0; j < nl; ++j) {
    for (int c = 0; c < 4; ++c) {
      const int vc = (c & 1) ? 2 : 0, vr = (c & 2) ? 2 : 0;
      if (vc == kc[j] && vr == kr[j]) continue;
      set_length_variant(b, ti, lens[j], vc, vr);
      float ms = 0.f;
      rc = time_batch_cg<T>(b, reps, &ms);
      if (rc) return rc;
      if (ms < best) {
        best = ms;
        kc[j] = vc;
        kr[j] = vr;
      }
    }
    set_length_variant(b, ti, lens[j], kc[j], kr[j]);
  }
  std::string line = key + " ";
  for (size_t j = 0; j < nl; ++j) line += (j ? "," : "") + std::to_string(kc[j]);
  line += " ";
  for (size_t j = 0; j < nl; ++j) line += (j ? "," : "") + std::to_string(kr[j]);
  char buf[32];
  std::snprintf(buf, sizeof(buf), " %.4f", (double)best);
  lines.push_back(line + buf);
  *added = true;
  return PL_OK;
}

}  // namespace

extern "C" {

int pl_batch_create(pl_batch** out, int n_inst, const int32_t* n, const double* box, int precision,
                    void* hip_stream, size_t* workspace_bytes) {
  if (!out || n_inst <= 0 || !n || !box || !workspace_bytes) return PL_ERR_INVALID_ARG;
  *out = nullptr;
  if (precision != PL_FP64 && precision != PL_MIXED) return PL_ERR_INVALID_ARG;
  for (int i = 0; i < 3 * n_inst; ++i)
    if (!batch_length_supported(n[i])) return PL_ERR_UNSUPPORTED_SIZE;
  pl_batch* b = new pl_batch();
  b->K = n_inst;
  b->precision = precision;
  b->user_stream = (hipStream_t)hip_stream;
  if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev, hipEventDisableTiming) != hipSuccess) {
    delete b;
    return PL_ERR_HIP;
  }
  size_t off = 0;
  for (int i = 0; i < n_inst; ++i) {
    pl_plan* p = nullptr;
    size_t ws = 0;
    int rc = pl_plan_create(&p, n + 3 * i, box + 3 * i, precision, (void*)b->stream, &ws);
    if (rc) {
      pl_batch_destroy(b);
      return rc;
    }
    b->plans.push_back(p);
    b->plan_off.push_back(off);
    off += align_up(ws);
  }
  b->plans_bytes = off;
  // work-list capacities: every instance in the narrow variant (the most
  // blocks per pass); then the default variants
  for (int t = 0; t < 2; ++t) {
    b->vcol[t].assign(n_inst, 2);
    b->vrow[t].assign(n_inst, 2);
  }
  build_work(b);
  for (int i = 0; i < W_COUNT; ++i) b->work[i].cap = b->work[i].items.size();
  b->work[W_XC].cap = std::max(b->work[W_X64].cap, b->work[W_X32].cap);
  b->work[W_YC].cap = std::max(b->work[W_Y64].cap, b->work[W_Y32].cap);
  b->work[W_RC].cap = std::max(b->work[W_R64].cap, b->work[W_R32].cap);
  for (int t = 0; t < 2; ++t) {
    b->vcol[t].assign(n_inst, 0);
    b->vrow[t].assign(n_inst, 0);
  }
  build_work(b);
  b->blob_bytes = batch_layout(b);
  b->ws_bytes = b->plans_bytes + b->blob_bytes;
  if (hipHostMalloc((void**)&b->h_blob, b->blob_bytes, hipHostMallocDefault) != hipSuccess) {
    pl_batch_destroy(b);
    return PL_ERR_HIP;
  }
  std::memset(b->h_blob, 0, b->blob_bytes);
  build_work(b);  // the host blob mirrors the device blob, work lists included
  b->h_scal = blob_ptr<double>(b, b->off_scal, true);
  *workspace_bytes = b->ws_bytes;
  *out = b;
  return PL_OK;
}

// The batch's internal stream waits for the work queued so far on the
// caller's stream (which may still be writing the arrays handed over).
static int join_user_stream(pl_batch* b) {
  BHIP(b, hipEventRecord(b->ev, b->user_stream));
  BHIP(b, hipStreamWaitEvent(b->stream, b->ev, 0));
  return PL_OK;
}

int pl_batch_set_workspace(pl_batch* b, void* dev_ptr) {
  if (!b) return PL_ERR_INVALID_ARG;
  if (!dev_ptr || ((uintptr_t)dev_ptr & 255)) return bfail(b, PL_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  int jrc = join_user_stream(b);
  if (jrc) return jrc;
  b->ws = (char*)dev_ptr;
  for (int i = 0; i < b->K; ++i) {
    int rc = pl_plan_set_workspace(b->plans[i], b->ws + b->plan_off[i]);
    if (rc) return bfail(b, rc, std::string("instance workspace: ") + pl_last_error(b->plans[i]));
  }
  b->d_blob = b->ws + b->plans_bytes;
  b->scal_all = blob_ptr<double>(b, b->off_scal, false);
  // every instance keeps its device scalars in one contiguous array
  for (int i = 0; i < b->K; ++i) b->plans[i]->scal = b->scal_all + (size_t)i * SC_COUNT;
  BHIP(b, hipMemsetAsync(b->scal_all, 0, sizeof(double) * SC_COUNT * b->K, b->stream));
  BHIP(b, hipMemcpyAsync(b->d_blob, b->h_blob, b->off_e64, hipMemcpyHostToDevice, b->stream));
  BHIP(b, hipStreamSynchronize(b->stream));
  for (int t = 0; t < 2; ++t)
    if (b->graph[t]) {
      (void)hipGraphExecDestroy(b->graph[t]);
      b->graph[t] = nullptr;
    }
  return PL_OK;
}

int pl_batch_set_problem(pl_batch* b, int i, const pl_problem* prob) {
  if (!b || i < 0 || i >= b->K) return PL_ERR_INVALID_ARG;
  if (!b->ws) return bfail(b, PL_ERR_INVALID_ARG, "workspace not set");
  int rc = join_user_stream(b);
  if (rc) return rc;
  rc = pl_set_problem(b->plans[i], prob);
  if (rc) return bfail(b, rc, "instance " + std::to_string(i) + ": " + pl_last_error(b->plans[i]));
  return PL_OK;
}

int pl_batch_autotune(pl_batch* b, const char* cache_path) {
  if (!b) return PL_ERR_INVALID_ARG;
  if (!b->ws) return bfail(b, PL_ERR_INVALID_ARG, "workspace not set");
  for (int i = 0; i < b->K; ++i)
    if (!b->plans[i]->has_problem)
      return bfail(b, PL_ERR_NO_PROBLEM, "instance " + std::to_string(i) + " has no problem");
  std::vector<std::string> lines;
  if (cache_path) {
    if (FILE* f = std::fopen(cache_path, "r")) {
      char buf[512];
      while (std::fgets(buf, sizeof(buf), f)) {
        std::string l(buf);
        while (!l.empty() && (l.back() == '\n' || l.back() == '\r')) l.pop_back();
        if (!l.empty() && l[0] != '#') lines.push_back(l);
      }
      std::fclose(f);
    }
  }
  int rc = join_user_stream(b);
  if (rc) return rc;
  const std::vector<int> lens = batch_lengths(b);
  std::string base = arch_name() + " batch";
  std::string ls;
  for (size_t j = 0; j < lens.size(); ++j) ls += (j ? "," : "") + std::to_string(lens[j]);
  bool added = false;
  rc = tune_batch_precision<double>(b, base + " fp64 " + ls, lens, lines, &added);
  if (!rc && b->precision == PL_MIXED) rc = tune_batch_precision<float>(b, base + " fp32 " + ls, lens, lines, &added);
  build_work(b);
  for (int t = 0; t < 2; ++t)
    if (b->graph[t]) {
      (void)hipGraphExecDestroy(b->graph[t]);
      b->graph[t] = nullptr;
    }
  (void)hipStreamSynchronize(b->stream);
  if (rc) return rc;
  if (cache_path && added) write_tune_cache(cache_path, lines);
  return PL_OK;
}

int pl_batch_solve(pl_batch* b, double* const* s_inout, const pl_solve_opts* opts, pl_solve_info* infos) {
  if (!b || !s_inout) return PL_ERR_INVALID_ARG;
  if (!b->ws) return bfail(b, PL_ERR_INVALID_ARG, "workspace not set");
  for (int i = 0; i < b->K; ++i) {
    if (!b->plans[i]->has_problem) return bfail(b, PL_ERR_NO_PROBLEM, "instance " + std::to_string(i) + " has no problem");
    if (!s_inout[i]) return bfail(b, PL_ERR_INVALID_ARG, "null s_inout entry");
  }
  pl_solve_opts o = resolve_opts(b->plans[0], opts);
  if (opts && opts->precision < 0) o.precision = b->precision;
  if (!(o.rtol >= 0.0) || o.max_newton < 0 || o.max_cg <= 0 || !(o.eta_max > 0.0) || !(o.ls_c1 > 0.0 && o.ls_c1 < 1.0))
    return bfail(b, PL_ERR_INVALID_ARG, "invalid solve options");
  // order after the caller's pending work
  int rc = join_user_stream(b);
  if (rc) return rc;
  if (o.precision == PL_MIXED) {
    if (b->precision != PL_MIXED) return bfail(b, PL_ERR_INVALID_ARG, "mixed solve needs a PL_MIXED batch");
    rc = batch_newton<float>(b, s_inout, o, infos);
  } else {
    rc = batch_newton<double>(b, s_inout, o, infos);
  }
  (void)hipStreamSynchronize(b->stream);
  if (rc && b->err.empty()) b->err = "an instance did not converge (see infos)";
  return rc;
}

int pl_batch_destroy(pl_batch* b) {
  if (!b) return PL_ERR_INVALID_ARG;
  for (int t = 0; t < 2; ++t)
    if (b->graph[t]) (void)hipGraphExecDestroy(b->graph[t]);
  for (pl_plan* p : b->plans) pl_plan_destroy(p);
  if (b->h_blob) (void)hipHostFree(b->h_blob);
  if (b->ev) (void)hipEventDestroy(b->ev);
  if (b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
  return PL_OK;
}

const char* pl_batch_last_error(const pl_batch* b) {
  if (!b) return "null batch";
  return b->err.c_str();
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Linear (non-local) bias, sections 2.2.1 and 2.4.1: delta_g = B delta_M with
// B the convolution of Fourier multiplier b_hat.  The unknown x is s =
// ln(1 + delta_M) (lognormal prior, MODEL_LOGNORMAL) or delta_M itself
// (Gaussian prior, MODEL_GAUSSIAN); phi(x) = delta_M, y = 1 + B phi(x).
//   f = 1/2 (x - m)^T S^-1 (x - m) + sum_i [nbar w_i y_i - N_i ln y_i]
//   g = S^-1 (x - m) + phi' B u,                u = nbar w - N / y
//   H = S^-1 + diag(phi'' B u) + diag(phi') B diag(N / y^2) B diag(phi')
// (B = B^T for a real, even b_hat).  Real-field workspace during a solve:
// e = phi' (lognormal), d = phi'' B u (lognormal), rtmp = N / y^2, s_ws the
// pointwise chain, preal the real copy of a spectral operand.  The line
// search holds B phi(x) in e while it runs.
// ---------------------------------------------------------------------------
namespace {

// The x pass with the caller's table (run_col substitutes the prior's)
hipError_t run_col_own_table(pl_plan* p, bool inverse, int op, const ColArgs<double>& a, int* nb) {
  int dummy;
  return launch_col<double>(p->n[0], inverse, op, a, 1, p->stream, nb ? nb : &dummy, p->var[0][V_XOP]);
}

// out = B in for real fields: z r2c, y forward, the x pass's forward
// transform, multiply by b_hat and inverse transform, y inverse, z c2r.
int lb_conv(pl_plan* p, const double* bk, const double* in, double* out) {
  cx<double>* t = p->t64;
  RowArgs<double> ra = row_args<double>(p);
  ra.in_r = in;
  ra.out_c = t;
  HIPCHK(p, run_row<double>(p, ROW_R2C, ra, nullptr));
  HIPCHK(p, run_col<double>(p, 1, false, COL_PLAIN, col_args<double>(p, 1, t, t), nullptr));
  ColArgs<double> ca = col_args<double>(p, 0, t, t);
  ca.inv_lam = bk;
  ca.radial = 0;
  ca.k0_shift = 0.0;
  HIPCHK(p, run_col_own_table(p, false, COL_PRIOR, ca, nullptr));
  HIPCHK(p, run_col<double>(p, 1, true, COL_PLAIN, col_args<double>(p, 1, t, t), nullptr));
  RowArgs<double> rb = row_args<double>(p);
  rb.in_c = t;
  rb.out_r = out;
  HIPCHK(p, run_row<double>(p, ROW_C2R, rb, nullptr));
  return PL_OK;
}

// Linearisation at the real field x: e = phi'(x) (lognormal), rtmp = N / y^2,
// SC_LIK = the likelihood sum, s_ws = l = phi' B u, d = phi'' B u (lognormal).
int lb_linearize(pl_plan* p, int model, const double* bk, const double* x) {
  const int nb = grid_blocks(p->N);
  hipLaunchKernelGGL(lb_phi_kernel, dim3(nb), dim3(RED_THREADS), 0, p->stream, x, nullptr, 0.0, model, p->s_ws,
                     model == MODEL_LOGNORMAL ? p->e : nullptr, p->N);
  HIPCHK(p, hipGetLastError());
  int rc = lb_conv(p, bk, p->s_ws, p->s_ws);
  if (rc) return rc;
  hipLaunchKernelGGL(lb_lik_kernel, dim3(nb), dim3(RED_THREADS), 0, p->stream, p->s_ws, p->prob.w, p->prob.counts,
                     p->prob.nbar, p->rtmp, p->N, p->partials);
  HIPCHK(p, hipGetLastError());
  HIPCHK(p, finalize(p, nb, 1, FIN_STORE, SC_LIK, 1.0));
  rc = lb_conv(p, bk, p->s_ws, p->s_ws);
  if (rc) return rc;
  hipLaunchKernelGGL(lb_grad_pointwise_kernel, dim3(nb), dim3(RED_THREADS), 0, p->stream, p->s_ws, p->e, model, p->d,
                     p->N);
  HIPCHK(p, hipGetLastError());
  p->d_valid = false;  // d no longer holds the power-law model's diagonal
  p->d32_valid = false;
  p->lb_ready = true;
  p->lb_model = model;
  p->lb_bk = bk;
  return PL_OK;
}

// g_out = (x_hat - m_hat) / lambda + F l (l in s_ws); SC_GG = ||g||^2 and
// SC_PRIOR = (x - m)^T S^-1 (x - m), as the power-law gradient leaves them.
int lb_assemble_grad(pl_plan* p, const cx<double>* x_hat, cx<double>* g_out) {
  cx<double>* t = p->t64;
  RowArgs<double> ra = row_args<double>(p);
  ra.in_r = p->s_ws;
  ra.out_c = t;
  HIPCHK(p, run_row<double>(p, ROW_R2C, ra, nullptr));
  HIPCHK(p, run_col<double>(p, 1, false, COL_PLAIN, col_args<double>(p, 1, t, t), nullptr));
  ColArgs<double> ca = col_args<double>(p, 0, t, g_out);
  ca.base = x_hat;
  ca.k0_shift = (double)p->N * prior_mean(p);
  int nb = 0;
  HIPCHK(p, run_col<double>(p, 0, false, COL_ADDPRIOR, ca, &nb));
  HIPCHK(p, finalize(p, nb, 3, FIN_STORE, SC_GG - 1, 1.0 / (double)p->N));
  return PL_OK;
}

// The x pass F_x^-1 diag(b_hat) F_x on a field already transformed along y and
// z.  It also leaves per-block partial sums (unused here) in `scratch`
// (default: the start of the partials buffer).
int lb_xmul(pl_plan* p, const double* bk, const double* skip = nullptr, double* scratch = nullptr) {
  ColArgs<double> ca = col_args<double>(p, 0, p->t64, p->t64);
  ca.inv_lam = bk;
  ca.radial = 0;
  ca.k0_shift = 0.0;
  ca.skip = skip;
  if (scratch) ca.partials = scratch;
  HIPCHK(p, run_col_own_table(p, false, COL_PRIOR, ca, nullptr));
  return PL_OK;
}

// out = H pin on half spectra at the current linearisation; out may be t64.
// With cg_r, the first x pass is the fused Krylov one: pin <- M^-1 cg_r +
// beta pin (beta = scal[SC_BETA]) in place, then transformed.  The
// Gauss-Newton part B diag(N/y^2) B runs as y, x(b_hat), y^-1, the z pass
// with rtmp (N/y^2) as its diagonal, y, x(b_hat), y^-1 between the z passes
// that apply phi' (lognormal prior; both x(b_hat) passes multiply along the
// same half spectrum).
int lb_hvp_hat(pl_plan* p, int model, const double* bk, cx<double>* pin, cx<double>* out,
               const cx<double>* cg_r = nullptr) {
  cx<double>* t = p->t64;
  int rc;
  if (cg_r) {
    ColArgs<double> c1 = col_args<double>(p, 0, pin, t);
    c1.cg_r = const_cast<cx<double>*>(cg_r);
    c1.scal = p->scal;
    HIPCHK(p, run_col<double>(p, 0, true, COL_CG_FIRST, c1, nullptr));
  } else {
    HIPCHK(p, run_col<double>(p, 0, true, COL_PLAIN, col_args<double>(p, 0, pin, t), nullptr));
  }
  if (model == MODEL_GAUSSIAN) {
    // phi' = 1, phi'' = 0: H p = b_hat F[(N/y^2) F^-1 (b_hat p)] + p/lambda, as
    // x^-1, x(b_hat), y^-1, the z pass with N/y^2, y, x(b_hat), x + prior.
    // Each x(b_hat) pass meets an unnormalised x transform of the opposite
    // sense, a factor nx: the z pass and the last x pass take 1/nx each.
    const double inv_nx = 1.0 / (double)p->n[0];
    if ((rc = lb_xmul(p, bk))) return rc;
    HIPCHK(p, run_col<double>(p, 1, true, COL_PLAIN, col_args<double>(p, 1, t, t), nullptr));
    RowArgs<double> ra = row_args<double>(p);
    ra.in_c = t;
    ra.out_c = t;
    ra.d = p->rtmp;
    ra.scale *= inv_nx;
    HIPCHK(p, run_row<double>(p, ROW_HVP, ra, nullptr));
    HIPCHK(p, run_col<double>(p, 1, false, COL_PLAIN, col_args<double>(p, 1, t, t), nullptr));
    if ((rc = lb_xmul(p, bk))) return rc;
    ColArgs<double> ca = col_args<double>(p, 0, t, out);
    ca.base = pin;
    ca.k0_shift = 0.0;
    ca.out_scale = inv_nx;
    HIPCHK(p, run_col<double>(p, 0, false, COL_ADDPRIOR, ca, nullptr));
    return PL_OK;
  }
  // lognormal: the z passes keep q = F^-1 p (ROW_LB_IN, also forming phi' q)
  // and form phi' g2 + d1 q (ROW_LB_OUT) between their c2r and r2c
  HIPCHK(p, run_col<double>(p, 1, true, COL_PLAIN, col_args<double>(p, 1, t, t), nullptr));
  {
    RowArgs<double> ra = row_args<double>(p);
    ra.in_c = t;
    ra.out_c = t;
    ra.out_r = p->preal;
    ra.d = p->e;
    ra.lb_d1 = p->d;
    HIPCHK(p, run_row<double>(p, ROW_LB_IN, ra, nullptr));
  }
  HIPCHK(p, run_col<double>(p, 1, false, COL_PLAIN, col_args<double>(p, 1, t, t), nullptr));
  if ((rc = lb_xmul(p, bk))) return rc;
  HIPCHK(p, run_col<double>(p, 1, true, COL_PLAIN, col_args<double>(p, 1, t, t), nullptr));
  {
    RowArgs<double> ra = row_args<double>(p);
    ra.in_c = t;
    ra.out_c = t;
    ra.d = p->rtmp;
    HIPCHK(p, run_row<double>(p, ROW_HVP, ra, nullptr));
  }
  HIPCHK(p, run_col<double>(p, 1, false, COL_PLAIN, col_args<double>(p, 1, t, t), nullptr));
  if ((rc = lb_xmul(p, bk))) return rc;
  HIPCHK(p, run_col<double>(p, 1, true, COL_PLAIN, col_args<double>(p, 1, t, t), nullptr));
  {
    RowArgs<double> ra = row_args<double>(p);
    ra.in_c = t;
    ra.out_c = t;
    ra.d = p->e;
    ra.lb_d1 = p->d;
    ra.lb_q = p->preal;
    HIPCHK(p, run_row<double>(p, ROW_LB_OUT, ra, nullptr));
  }
  HIPCHK(p, run_col<double>(p, 1, false, COL_PLAIN, col_args<double>(p, 1, t, t), nullptr));
  ColArgs<double> ca = col_args<double>(p, 0, t, out);
  ca.base = pin;
  ca.k0_shift = 0.0;
  HIPCHK(p, run_col<double>(p, 0, false, COL_ADDPRIOR, ca, nullptr));
  return PL_OK;
}

// Preconditioner constant c of M_k = 1/lambda_k + c: the 25th percentile of
// the per-cell curvature (lb_curv_kernel), as for the power-law model.
int lb_precond(pl_plan* p, int model) {
  const int nb = grid_blocks(p->N);
  hipLaunchKernelGGL(lb_curv_kernel, dim3(nb), dim3(RED_THREADS), 0, p->stream, p->e, p->rtmp, p->d, model, p->preal,
                     p->N);
  HIPCHK(p, hipGetLastError());
  hipLaunchKernelGGL(sum_kernel, dim3(nb), dim3(RED_THREADS), 0, p->stream, p->preal, p->N, p->partials);
  HIPCHK(p, hipGetLastError());
  HIPCHK(p, finalize(p, nb, 1, FIN_STORE, SC_DSUM, 1.0));
  return set_precond_constant(p, p->preal);
}

// Truncated PCG on H x = -g (g_hat) into x64: stops at ||r|| <= tol_abs or at
// the first direction of non-positive curvature; if that is the first
// direction, x = M^-1 (-g) (preconditioned steepest descent).  The direction
// update p = M^-1 r + beta p runs inside the first pass of each HVP.
// Host-driven, two scalar read-backs per iteration.
int lb_pcg(pl_plan* p, int model, const double* bk, double tol_abs, int max_cg, int* its_out, int* hv_out) {
  cx<double>*x = p->x64, *r = p->r64, *pp = p->p64, *q = p->t64;
  // the table the fused pass reads (its mirrored form reads the per-mode one)
  const int radial = p->radial && p->var[0][V_TAB_CG] == TAB_SHELL;
  const double* tab = View<double>::tab(p, radial);
  const double invN = 1.0 / (double)p->N;
  const int nb = grid_blocks(p->Nh);
  hipLaunchKernelGGL(lb_cg_init_kernel, dim3(nb), dim3(RED_THREADS), 0, p->stream, p->g_hat, x, r, pp, tab, radial,
                     p->g, p->scal, p->Nh, p->partials);
  HIPCHK(p, hipGetLastError());
  HIPCHK(p, finalize(p, nb, 2, FIN_STORE, SC_DF, invN));
  HIPCHK(p, set_scalar(p, SC_BETA, 0.0));
  int rc = read_scalars(p);
  if (rc) return rc;
  double rz = p->h_scal[SC_DF], rr = p->h_scal[SC_DF + 1];
  int its = 0, hv = 0;
  for (int k = 0; k < max_cg; ++k) {
    if (!(std::sqrt(std::max(0.0, rr)) > tol_abs)) break;
    rc = lb_hvp_hat(p, model, bk, pp, q, r);  // p = M^-1 r + beta p, q = H p
    if (rc) return rc;
    ++hv;
    hipLaunchKernelGGL(lb_dot_kernel, dim3(nb), dim3(RED_THREADS), 0, p->stream, pp, q, p->g, p->Nh, p->partials);
    HIPCHK(p, hipGetLastError());
    HIPCHK(p, finalize(p, nb, 1, FIN_STORE, SC_PQ, invN));
    rc = read_scalars(p);
    if (rc) return rc;
    const double pq = p->h_scal[SC_PQ];
    if (!(pq > 0.0)) {
      if (its == 0) HIPCHK(p, hipMemcpyAsync(x, pp, sizeof(cx<double>) * p->Nh, hipMemcpyDeviceToDevice, p->stream));
      break;
    }
    const double alpha = rz / pq;
    hipLaunchKernelGGL(lb_cg_update_kernel, dim3(nb), dim3(RED_THREADS), 0, p->stream, x, r, pp, q, alpha, tab,
                       radial, p->g, p->scal, p->Nh, p->partials);
    HIPCHK(p, hipGetLastError());
    HIPCHK(p, finalize(p, nb, 2, FIN_STORE, SC_DF, invN));
    rc = read_scalars(p);
    if (rc) return rc;
    ++its;
    const double rz_new = p->h_scal[SC_DF];
    rr = p->h_scal[SC_DF + 1];
    if (!(std::sqrt(std::max(0.0, rr)) > tol_abs)) break;
    HIPCHK(p, set_scalar(p, SC_BETA, rz_new / rz));
    rz = rz_new;
  }
  *its_out = its;
  *hv_out = hv;
  return PL_OK;
}

// Lognormal prior: the same truncated PCG with the Krylov updates fused into
// the operator's first and last x passes, as the power-law solve does:
// COL_CG_FIRST forms p = M^-1 r + beta p before the inverse transform,
// COL_CG_LAST forms H p = X + p/lambda and updates r and x in place.  The
// step length comes from device partials: p^H Lambda^-1 p (COL_CG_FIRST),
// sum phi'' B u q^2 (ROW_LB_IN, stored to SC_LB_DQ) and sum (N/y^2)(B phi' q)^2
// (the ROW_HVP z pass); a non-positive p^H H p stops the iteration
// (SC_DONE = 2).  Launched in chunks of check_every iterations, each
// iteration after convergence exiting at once; the host reads the scalars
// once per chunk.
int lb_pcg_fused(pl_plan* p, const double* bk, double tol_abs, int max_cg, int check_every, int* its_out,
                 int* hv_out) {
  cx<double>*x = p->x64, *r = p->r64, *pp = p->p64, *t = p->t64;
  const double invN = 1.0 / (double)p->N;
  double* part_a = p->partials;
  double* part_b = p->partials + p->partials_len;
  // the x(b_hat) passes' own partial sums go to the second half of region a,
  // clear of the COL_CG_FIRST sums (first half) that the step length reads
  double* part_x = part_a + p->partials_len / 2;
  HIPCHK(p, set_scalar(p, SC_TOL2, tol_abs * tol_abs));
  hipLaunchKernelGGL((cg_init_kernel<double>), dim3(NB_RED), dim3(RED_THREADS), 0, p->stream, p->g_hat, -1.0, x, r,
                     pp, View<double>::tab(p), TAB_MODE, p->g, p->Nh, p->scal, p->partials);
  HIPCHK(p, hipGetLastError());
  HIPCHK(p, finalize(p, NB_RED, 2, FIN_CG_INIT, 0, invN));
  const double* skip = p->scal + SC_DONE;
  int launched = 0;
  while (launched < max_cg) {
    const int chunk = std::min(check_every, max_cg - launched);
    for (int k = 0; k < chunk; ++k) {
      int nb1 = 0, nbq = 0, nbz = 0, nb5 = 0;
      ColArgs<double> c1 = col_args<double>(p, 0, pp, t);
      c1.cg_r = r;
      c1.scal = p->scal;
      c1.partials = part_a;
      c1.skip = skip;
      HIPCHK(p, run_col<double>(p, 0, true, COL_CG_FIRST, c1, &nb1));
      ColArgs<double> cy = col_args<double>(p, 1, t, t);
      cy.skip = skip;
      HIPCHK(p, run_col<double>(p, 1, true, COL_PLAIN, cy, nullptr));
      RowArgs<double> r1 = row_args<double>(p);
      r1.in_c = t;
      r1.out_c = t;
      r1.out_r = p->preal;
      r1.d = p->e;
      r1.lb_d1 = p->d;
      r1.partials = part_b;
      r1.skip = skip;
      HIPCHK(p, run_row<double>(p, ROW_LB_IN, r1, &nbq));
      HIPCHK(p, finalize(p, nbq, 2, FIN_STORE, SC_LB_DQ, 1.0, 0.0, part_b));
      HIPCHK(p, run_col<double>(p, 1, false, COL_PLAIN, cy, nullptr));
      int rc = lb_xmul(p, bk, skip, part_x);
      if (rc) return rc;
      HIPCHK(p, run_col<double>(p, 1, true, COL_PLAIN, cy, nullptr));
      RowArgs<double> r2 = row_args<double>(p);
      r2.in_c = t;
      r2.out_c = t;
      r2.d = p->rtmp;
      r2.partials = part_b;
      r2.skip = skip;
      HIPCHK(p, run_row<double>(p, ROW_HVP, r2, &nbz));
      HIPCHK(p, run_col<double>(p, 1, false, COL_PLAIN, cy, nullptr));
      if ((rc = lb_xmul(p, bk, skip, part_x))) return rc;
      HIPCHK(p, run_col<double>(p, 1, true, COL_PLAIN, cy, nullptr));
      RowArgs<double> r3 = row_args<double>(p);
      r3.in_c = t;
      r3.out_c = t;
      r3.d = p->e;
      r3.lb_d1 = p->d;
      r3.lb_q = p->preal;
      r3.skip = skip;
      HIPCHK(p, run_row<double>(p, ROW_LB_OUT, r3, nullptr));
      HIPCHK(p, run_col<double>(p, 1, false, COL_PLAIN, cy, nullptr));
      HIPCHK(p, finalize(p, nbz, 2, FIN_CG_ALPHA_ADD, SC_LB_DQ, 1.0, 0.0, part_b, part_a, nb1, invN));
      ColArgs<double> c5 = col_args<double>(p, 0, t, t);
      c5.base = pp;
      c5.cg_r = r;
      c5.cg_x = x;
      c5.scal = p->scal;
      c5.partials = part_a;
      c5.skip = skip;
      HIPCHK(p, run_col<double>(p, 0, false, COL_CG_LAST, c5, &nb5));
      HIPCHK(p, finalize(p, nb5, 2, FIN_CG_BETA, 0, invN, (double)max_cg, part_a));
    }
    launched += chunk;
    int rc = read_scalars(p);
    if (rc) return rc;
    if (p->h_scal[SC_DONE] != 0.0) break;
  }
  int rc = read_scalars(p);
  if (rc) return rc;
  const int its = (int)p->h_scal[SC_ITS];
  const bool breakdown = p->h_scal[SC_DONE] == 2.0;
  // non-positive curvature along the first direction: take p = M^-1 (-g)
  if (breakdown && its == 0)
    HIPCHK(p, hipMemcpyAsync(x, pp, sizeof(cx<double>) * p->Nh, hipMemcpyDeviceToDevice, p->stream));
  *its_out = its;
  *hv_out = its + (breakdown ? 1 : 0);
  return PL_OK;
}

// Armijo backtracking along x64 from s_hat (real field x_real): the decrease
// a b + a^2 c / 2 + sum_i [nbar w_i dy_i - N_i log1p(dy_i / y_i)], with
// dy = B (phi(x + a p) - phi(x)), against c1 a p^T g for a = 1, 1/2, ...
// (at most 40 halvings).  *alpha = the step or -1; *descent = (p^T g < 0).
int lb_line_search(pl_plan* p, int model, const double* bk, const double* x_real, const pl_solve_opts& o,
                   double* alpha, bool* descent) {
  const double invN = 1.0 / (double)p->N;
  cx<double>* x = p->x64;
  int rc = inv_c2r<double>(p, x, p->t64, p->preal);
  if (rc) return rc;
  hipLaunchKernelGGL((ls_dots_kernel<double>), dim3(NB_RED), dim3(RED_THREADS), 0, p->stream, x, p->s_hat, p->g_hat,
                     p->tab_mode, TAB_MODE, p->g, p->Nh, (double)p->N * prior_mean(p),
                     p->partials);
  HIPCHK(p, hipGetLastError());
  HIPCHK(p, finalize(p, NB_RED, 3, FIN_STORE, SC_LS_B, invN));
  const int nb = grid_blocks(p->N);
  // B phi(x) into e (phi' is recomputed by the next gradient)
  p->lb_ready = false;
  hipLaunchKernelGGL(lb_phi_kernel, dim3(nb), dim3(RED_THREADS), 0, p->stream, x_real, nullptr, 0.0, model, p->s_ws,
                     nullptr, p->N);
  HIPCHK(p, hipGetLastError());
  rc = lb_conv(p, bk, p->s_ws, p->e);
  if (rc) return rc;
  // one trial step a: its likelihood difference into SC_DF, then the
  // read-back (the first trial goes out with the dots)
  auto trial = [&](double a) -> int {
    hipLaunchKernelGGL(lb_phi_step_kernel, dim3(nb), dim3(RED_THREADS), 0, p->stream, x_real, p->preal, a, model,
                       p->s_ws, p->N);
    HIPCHK(p, hipGetLastError());
    int trc = lb_conv(p, bk, p->s_ws, p->s_ws);
    if (trc) return trc;
    hipLaunchKernelGGL(lb_step_lik_kernel, dim3(nb), dim3(RED_THREADS), 0, p->stream, p->s_ws, p->e, p->prob.w,
                       p->prob.counts, p->prob.nbar, p->N, p->partials);
    HIPCHK(p, hipGetLastError());
    HIPCHK(p, finalize(p, nb, 1, FIN_STORE, SC_DF, 1.0));
    return read_scalars(p);
  };
  rc = trial(1.0);
  if (rc) return rc;
  const double b = p->h_scal[SC_LS_B], c = p->h_scal[SC_LS_C], slope = p->h_scal[SC_LS_SLOPE];
  *alpha = -1.0;
  *descent = slope < 0.0;
  if (!(slope < 0.0)) return PL_OK;
  double a = 1.0;
  for (int j = 0; j < 40; ++j, a *= 0.5) {
    if (j > 0) {
      rc = trial(a);
      if (rc) return rc;
    }
    const double df = a * b + 0.5 * a * a * c + p->h_scal[SC_DF];
    if (df <= o.ls_c1 * a * slope) {
      *alpha = a;
      break;
    }
  }
  return PL_OK;
}

// Gradient at the spectral iterate s_hat: x_real = F^-1 s_hat, the
// linearisation there, g_hat.
int lb_grad_hat(pl_plan* p, int model, const double* bk, double* x_real) {
  int rc = inv_c2r<double>(p, p->s_hat, p->t64, x_real);
  if (rc) return rc;
  rc = lb_linearize(p, model, bk, x_real);
  if (rc) return rc;
  return lb_assemble_grad(p, p->s_hat, p->g_hat);
}

int lb_newton_solve(pl_plan* p, int model, const double* bk, double* x_io, const pl_solve_opts& o,
                    pl_solve_info* info) {
  pl_solve_info inf{};
  int rc = fwd_r2c<double>(p, x_io, p->s_hat);
  if (rc) return rc;
  rc = lb_grad_hat(p, model, bk, x_io);
  if (rc) return rc;
  rc = read_scalars(p);
  if (rc) return rc;
  const double g0 = std::sqrt(std::max(0.0, p->h_scal[SC_GG]));
  double gn = g0;
  double obj = 0.5 * p->h_scal[SC_PRIOR] + p->h_scal[SC_LIK];
  inf.grad0 = g0;
  inf.obj = obj;
  if (!std::isfinite(g0) || !std::isfinite(obj)) {
    if (info) *info = inf;
    return fail(p, PL_ERR_DOMAIN, "the start is outside the domain (1 + B delta <= 0 in a cell with counts)");
  }
  int status = PL_OK;
  if (g0 > 0.0) {
    for (int it = 0;; ++it) {
      if (gn <= o.rtol * g0) break;
      if (it >= o.max_newton) {
        status = PL_ERR_NOT_CONVERGED;
        p->err = "Newton iteration cap reached";
        break;
      }
      const double eta = std::min(o.eta_max, std::max(std::sqrt(gn / g0), 0.5 * o.rtol * g0 / gn));
      rc = lb_precond(p, model);
      if (rc) return rc;
      int its = 0, hv = 0;
      rc = model == MODEL_LOGNORMAL ? lb_pcg_fused(p, bk, eta * gn, o.max_cg, o.check_every, &its, &hv)
                                    : lb_pcg(p, model, bk, eta * gn, o.max_cg, &its, &hv);
      if (rc) return rc;
      inf.cg_its += its;
      inf.hvps += hv;
      double alpha = -1.0;
      bool descent = false;
      rc = lb_line_search(p, model, bk, x_io, o, &alpha, &descent);
      if (rc) return rc;
      if (alpha < 0.0) {
        status = PL_ERR_LINESEARCH;
        p->err = descent ? "no step satisfies the Armijo condition" : "Newton direction is not a descent direction";
        break;
      }
      hipLaunchKernelGGL((axpy_hat_kernel<double>), dim3(NB_RED), dim3(RED_THREADS), 0, p->stream, p->s_hat, p->x64,
                         alpha, p->Nh);
      HIPCHK(p, hipGetLastError());
      rc = lb_grad_hat(p, model, bk, x_io);
      if (rc) return rc;
      rc = read_scalars(p);
      if (rc) return rc;
      gn = std::sqrt(std::max(0.0, p->h_scal[SC_GG]));
      obj = 0.5 * p->h_scal[SC_PRIOR] + p->h_scal[SC_LIK];
      inf.newton_its = it + 1;
      if (!std::isfinite(gn)) {
        status = PL_ERR_DOMAIN;
        p->err = "gradient became non-finite";
        break;
      }
    }
  }
  inf.rel_grad = g0 > 0.0 ? gn / g0 : 0.0;
  inf.obj = obj;
  inf.status = status;
  if (info) *info = inf;
  return status;
}

static_assert(PL_MODEL_LOGNORMAL == MODEL_LOGNORMAL && PL_MODEL_GAUSSIAN == MODEL_GAUSSIAN, "model codes");

int lb_check(pl_plan* p, int model, const double* bk) {
  if (model != MODEL_LOGNORMAL && model != MODEL_GAUSSIAN) return fail(p, PL_ERR_INVALID_ARG, "unknown model");
  if (!bk) return fail(p, PL_ERR_INVALID_ARG, "null b_hat table");
  if (p->prob.beta != 1.0)
    return fail(p, PL_ERR_INVALID_ARG, "the linear bias replaces the power-law bias: the problem needs beta = 1");
  return check_finite(p, bk, p->Nh, "b_hat");
}

}  // namespace

extern "C" {

int pl_linear_bias_grad(pl_plan* p, int model, const double* bk, const double* x, double* grad_out,
                        double* obj_out) {
  int rc = check_ready(p);
  if (rc) return rc;
  if (!x || !grad_out) return fail(p, PL_ERR_INVALID_ARG, "null pointer");
  rc = lb_check(p, model, bk);
  if (rc) return rc;
  p->model = model;
  rc = fwd_r2c<double>(p, x, p->x64);
  if (!rc) rc = lb_linearize(p, model, bk, x);
  if (!rc) rc = lb_assemble_grad(p, p->x64, p->r64);
  if (!rc) rc = inv_c2r<double>(p, p->r64, p->t64, grad_out);
  p->model = MODEL_LOGNORMAL;
  if (rc) return rc;
  if (obj_out) {
    rc = read_scalars(p);
    if (rc) return rc;
    *obj_out = 0.5 * p->h_scal[SC_PRIOR] + p->h_scal[SC_LIK];
  }
  return PL_OK;
}

int pl_linear_bias_hessvec(pl_plan* p, int model, const double* bk, const double* x, const double* v,
                           double* hv_out) {
  if (!p) return PL_ERR_INVALID_ARG;
  const bool cached = p->lb_ready && p->lb_model == model && p->lb_bk == bk;
  int rc = check_ready(p);
  if (rc) return rc;
  if (!v || !hv_out) return fail(p, PL_ERR_INVALID_ARG, "null pointer");
  rc = lb_check(p, model, bk);
  if (rc) return rc;
  if (!x && !cached)
    return fail(p, PL_ERR_NO_PROBLEM, "no linearisation to reuse: pass x or call pl_linear_bias_grad first");
  if (x) {
    rc = lb_linearize(p, model, bk, x);
    if (rc) return rc;
  }
  p->model = model;
  rc = fwd_r2c<double>(p, v, p->x64);
  if (!rc) rc = lb_hvp_hat(p, model, bk, p->x64, p->r64);
  if (!rc) rc = inv_c2r<double>(p, p->r64, p->t64, hv_out);
  p->model = MODEL_LOGNORMAL;
  if (rc) return rc;
  p->lb_ready = true;
  p->lb_model = model;
  p->lb_bk = bk;
  return PL_OK;
}

int pl_linear_bias_solve(pl_plan* p, int model, const double* bk, double* x_inout, const pl_solve_opts* opts,
                         pl_solve_info* info) {
  return pl_linear_bias_solve_hat(p, model, bk, x_inout, nullptr, opts, info);
}

int pl_linear_bias_solve_hat(pl_plan* p, int model, const double* bk, double* x_inout, double* x_hat_out,
                             const pl_solve_opts* opts, pl_solve_info* info) {
  int rc = check_ready(p);
  if (rc) return rc;
  if (!x_inout) return fail(p, PL_ERR_INVALID_ARG, "null pointer");
  pl_solve_opts o = resolve_opts(p, opts);
  if (!(o.rtol >= 0.0) || o.max_newton < 0 || o.max_cg <= 0 || !(o.eta_max > 0.0) || !(o.ls_c1 > 0.0 && o.ls_c1 < 1.0))
    return fail(p, PL_ERR_INVALID_ARG, "invalid solve options");
  if (opts && opts->precision == PL_MIXED)
    return fail(p, PL_ERR_INVALID_ARG, "the linear-bias solve runs in FP64 only");
  rc = lb_check(p, model, bk);
  if (rc) return rc;
  rc = check_finite(p, x_inout, p->N, "x_inout");
  if (rc) return rc;
  p->model = model;
  rc = lb_newton_solve(p, model, bk, x_inout, o, info);
  p->model = MODEL_LOGNORMAL;
  if (x_hat_out && (rc == PL_OK || rc == PL_ERR_NOT_CONVERGED || rc == PL_ERR_LINESEARCH)) {
    HIPCHK(p, hipMemcpyAsync(x_hat_out, p->s_hat, sizeof(cx<double>) * p->Nh, hipMemcpyDeviceToDevice, p->stream));
    HIPCHK(p, hipStreamSynchronize(p->stream));
  }
  return rc;
}

}  // extern "C"
