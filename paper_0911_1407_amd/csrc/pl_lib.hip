// Host side of libpl.so: plans, workspace carving, problem set-up, the
// gradient / Hessian-vector pipelines, the inexact Newton-Krylov MAP solver
// and the adjoint solve.  See include/pl.h for the public contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pl.h"
#define PL_OPS_KERNELS 1
#include "pl_passes.hpp"

using namespace pl;

namespace {

constexpr int NB_RED = 1024;  // blocks of the grid-stride reduction kernels

struct Status {
  int code = PL_OK;
  std::string msg;
};

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
  double* h_scal = nullptr;  // pinned host mirror of scal
  // problem
  bool has_problem = false;
  pl_problem prob{};
  bool d_valid = false;    // d holds the diagonal of the last linearisation
  bool d32_valid = false;  // d32 mirrors d
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
  // two regions: the fused CG keeps the first pass's partials while the z
  // pass writes its own
  p->partials = (double*)take(sizeof(double) * p->partials_len * 2);
  p->scal = (double*)take(sizeof(double) * SC_COUNT);
  p->flags = (int*)take(sizeof(int) * 4);
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
  static const double* tab(pl_plan* p) { return p->radial ? p->tab_rad : p->tab_mode; }
  static const cx<double>* tw(pl_plan* p, int a) { return p->tw64[a]; }
};
template <>
struct View<float> {
  static cx<float>* x(pl_plan* p) { return p->x32; }
  static cx<float>* r(pl_plan* p) { return p->r32; }
  static cx<float>* pv(pl_plan* p) { return p->p32; }
  static cx<float>* t(pl_plan* p) { return p->t32; }
  static float* preal(pl_plan* p) { return p->preal32; }
  static const float* tab(pl_plan* p) { return p->radial ? p->tab_rad32 : p->tab_mode32; }
  static const cx<float>* tw(pl_plan* p, int a) { return p->tw32[a]; }
};

// ---------------------------------------------------------------------------
// Passes
// ---------------------------------------------------------------------------

template <typename T>
ColArgs<T> col_args(pl_plan* p, int axis, const cx<T>* in, cx<T>* out) {
  ColArgs<T> a{};
  a.in = in;
  a.out = out;
  a.tw = View<T>::tw(p, axis);
  a.g = p->g;
  a.inv_lam = View<T>::tab(p);
  a.radial = p->radial;
  a.partials = p->partials;
  a.out_scale = T(1);
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
  return launch_col<T>(p->n[axis], inverse, op, a, axis == 0 ? 1 : p->n[0], p->stream, nb ? nb : &dummy);
}

template <typename T>
RowArgs<T> row_args(pl_plan* p) {
  RowArgs<T> a{};
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
  return a;
}

template <typename T>
hipError_t run_row(pl_plan* p, int op, const RowArgs<T>& a, int* nb) {
  int dummy;
  return launch_row<T>(p->n[2], op, a, p->stream, nb ? nb : &dummy);
}

hipError_t finalize(pl_plan* p, int nb, int K, int kind, int dst, double scale, double aux = 0.0,
                    const double* partials = nullptr, const double* partials2 = nullptr, int nb2 = 0,
                    double scale2 = 0.0) {
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(256), 0, p->stream, partials ? partials : p->partials, nb, K,
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
int grad_hat(pl_plan* p, double* s_out) {
  cx<double>* t = p->t64;
  HIPCHK(p, run_col<double>(p, 0, true, COL_PLAIN, col_args<double>(p, 0, p->s_hat, t), nullptr));
  HIPCHK(p, run_col<double>(p, 1, true, COL_PLAIN, col_args<double>(p, 1, t, t), nullptr));
  RowArgs<double> ra = row_args<double>(p);
  ra.in_c = t;
  ra.out_c = t;
  ra.s_out = s_out;
  ra.e_out = p->e;
  ra.d_out = p->d;
  int nb = 0;
  HIPCHK(p, run_row<double>(p, ROW_GRAD, ra, &nb));
  HIPCHK(p, finalize(p, nb, 2, FIN_STORE, SC_LIK, 1.0));
  HIPCHK(p, run_col<double>(p, 1, false, COL_PLAIN, col_args<double>(p, 1, t, t), nullptr));
  ColArgs<double> ca = col_args<double>(p, 0, t, p->g_hat);
  ca.base = p->s_hat;
  ca.k0_shift = (double)p->N * p->prob.mu;
  HIPCHK(p, run_col<double>(p, 0, false, COL_ADDPRIOR, ca, &nb));
  HIPCHK(p, finalize(p, nb, 3, FIN_STORE, SC_GG - 1, 1.0 / (double)p->N));
  p->d_valid = true;
  p->d32_valid = false;
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
template <typename T>
int pcg(pl_plan* p, const cx<double>* rhs, double sign, double tol_abs, double tol_rel_of_rhs, int max_cg,
        int check_every, int* its, int* hvps, double* rel_res, double* rhs_norm) {
  cx<T>*x = View<T>::x(p), *r = View<T>::r(p), *pp = View<T>::pv(p), *t = View<T>::t(p);
  const T* tab = View<T>::tab(p);
  const double invN = 1.0 / (double)p->N;
  double* part_a = p->partials;
  double* part_b = p->partials + p->partials_len;
  HIPCHK(p, set_scalar(p, SC_TOL2, tol_abs * tol_abs));
  hipLaunchKernelGGL((cg_init_kernel<T>), dim3(NB_RED), dim3(RED_THREADS), 0, p->stream, rhs, sign, x, r, pp, tab,
                     p->radial, p->g, p->Nh, p->scal, p->partials);
  HIPCHK(p, hipGetLastError());
  HIPCHK(p, finalize(p, NB_RED, 2, FIN_CG_INIT, 0, invN));
  double rr0 = 0.0;
  if (tol_rel_of_rhs > 0.0) {
    int rc = read_scalars(p);
    if (rc) return rc;
    rr0 = p->h_scal[SC_RR];
    double tol2 = tol_rel_of_rhs * tol_rel_of_rhs * rr0;
    HIPCHK(p, set_scalar(p, SC_TOL2, tol2));
    HIPCHK(p, set_scalar(p, SC_DONE, rr0 <= tol2 ? 1.0 : 0.0));
  }
  int launched = 0;
  while (launched < max_cg) {
    int chunk = std::min(check_every, max_cg - launched);
    for (int k = 0; k < chunk; ++k) {
      int nb1 = 0, nb3 = 0, nb5 = 0;
      const double* skip = p->scal + SC_DONE;
      ColArgs<T> c1 = col_args<T>(p, 0, pp, t);
      c1.cg_r = r;
      c1.scal = p->scal;
      c1.partials = part_a;
      c1.skip = skip;
      HIPCHK(p, run_col<T>(p, 0, true, COL_CG_FIRST, c1, &nb1));
      ColArgs<T> c2 = col_args<T>(p, 1, t, t);
      c2.skip = skip;
      HIPCHK(p, run_col<T>(p, 1, true, COL_PLAIN, c2, nullptr));
      RowArgs<T> ra = row_args<T>(p);
      ra.in_c = t;
      ra.out_c = t;
      ra.partials = part_b;
      ra.skip = skip;
      HIPCHK(p, run_row<T>(p, ROW_HVP, ra, &nb3));
      HIPCHK(p, finalize(p, nb3, 2, FIN_CG_ALPHA, 0, 1.0, 0.0, part_b, part_a, nb1, invN));
      ColArgs<T> c4 = col_args<T>(p, 1, t, t);
      c4.skip = skip;
      HIPCHK(p, run_col<T>(p, 1, false, COL_PLAIN, c4, nullptr));
      ColArgs<T> c5 = col_args<T>(p, 0, t, t);
      c5.base = pp;
      c5.cg_r = r;
      c5.cg_x = x;
      c5.scal = p->scal;
      c5.partials = part_a;
      c5.skip = skip;
      HIPCHK(p, run_col<T>(p, 0, false, COL_CG_LAST, c5, &nb5));
      HIPCHK(p, finalize(p, nb5, 2, FIN_CG_BETA, 0, invN, (double)max_cg, part_a));
    }
    launched += chunk;
    int rc = read_scalars(p);
    if (rc) return rc;
    if (p->h_scal[SC_DONE] != 0.0) break;
  }
  int rc = read_scalars(p);
  if (rc) return rc;
  *its = (int)p->h_scal[SC_ITS];
  // Hessian products that ran: one per counted iteration, plus the partial
  // one of a breakdown; queued iterations after convergence exit at once
  *hvps = *its + (p->h_scal[SC_DONE] == 2.0 ? 1 : 0);
  if (rel_res) *rel_res = std::sqrt(std::max(0.0, p->h_scal[SC_RR]));
  if (rhs_norm) *rhs_norm = std::sqrt(rr0);
  return PL_OK;
}

int check_ready(pl_plan* p) {
  if (!p) return PL_ERR_INVALID_ARG;
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

template <typename T>
int newton_solve(pl_plan* p, double* s_io, const pl_solve_opts& o, pl_solve_info* info) {
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
  double obj = 0.5 * p->h_scal[SC_PRIOR] + p->h_scal[SC_LIK];
  inf.grad0 = g0;
  inf.obj = obj;
  if (!std::isfinite(g0) || !std::isfinite(obj)) {
    if (info) *info = inf;
    return fail(p, PL_ERR_DOMAIN, "gradient at the starting point is not finite");
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
      // forcing term: sqrt(||g||/||g0||), but no tighter than needed to
      // reach the stopping tolerance from here (half of it, for margin)
      const double eta = std::min(o.eta_max, std::max(std::sqrt(gn / g0), 0.5 * o.rtol * g0 / gn));
      HIPCHK(p, set_scalar(p, SC_DBAR, p->h_scal[SC_DSUM] * invN));
      if constexpr (sizeof(T) == 4) {
        rc = ensure_d32(p);
        if (rc) return rc;
      }
      int its = 0, hv = 0;
      rc = pcg<T>(p, p->g_hat, -1.0, eta * gn, 0.0, o.max_cg, o.check_every, &its, &hv, nullptr, nullptr);
      if (rc) return rc;
      inf.cg_its += its;
      inf.hvps += hv;
      // line search along the Newton direction x (spectral) / preal (real)
      cx<T>* x = View<T>::x(p);
      rc = inv_c2r<T>(p, x, View<T>::t(p), View<T>::preal(p));
      if (rc) return rc;
      hipLaunchKernelGGL((ls_dots_kernel<T>), dim3(NB_RED), dim3(RED_THREADS), 0, p->stream, x, p->s_hat, p->g_hat,
                         p->radial ? p->tab_rad : p->tab_mode, p->radial, p->g, p->Nh,
                         (double)p->N * p->prob.mu, p->partials);
      HIPCHK(p, hipGetLastError());
      HIPCHK(p, finalize(p, NB_RED, 3, FIN_STORE, SC_LS_B, invN));
      rc = read_scalars(p);
      if (rc) return rc;
      const double b = p->h_scal[SC_LS_B], c = p->h_scal[SC_LS_C], slope = p->h_scal[SC_LS_SLOPE];
      double alpha = -1.0;
      if (slope < 0.0) {
        double a0 = 1.0;
        for (int batch = 0; batch < 8 && alpha < 0.0; ++batch) {
          hipLaunchKernelGGL((ls_eval_kernel<T>), dim3(NB_RED), dim3(RED_THREADS), 0, p->stream,
                             View<T>::preal(p), p->e, p->prob.counts, p->prob.beta, a0, p->N, p->partials);
          HIPCHK(p, hipGetLastError());
          HIPCHK(p, finalize(p, NB_RED, 4, FIN_STORE, SC_DF, 1.0));
          rc = read_scalars(p);
          if (rc) return rc;
          double a = a0;
          for (int j = 0; j < 4; ++j, a *= 0.5) {
            double df = a * b + 0.5 * a * a * c + p->h_scal[SC_DF + j];
            if (df <= o.ls_c1 * a * slope) {
              alpha = a;
              break;
            }
          }
          a0 *= 1.0 / 16.0;
        }
      }
      if (alpha < 0.0) {
        status = PL_ERR_LINESEARCH;
        p->err = slope < 0.0 ? "no step satisfies the Armijo condition" : "Newton direction is not a descent direction";
        break;
      }
      hipLaunchKernelGGL((axpy_hat_kernel<T>), dim3(NB_RED), dim3(RED_THREADS), 0, p->stream, p->s_hat, x, alpha,
                         p->Nh);
      HIPCHK(p, hipGetLastError());
      rc = grad_hat(p, s_io);
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
  HIPCHK(p, set_scalar(p, SC_DBAR, p->h_scal[SC_DSUM] * invN));
  if constexpr (sizeof(T) == 4) {
    rc = ensure_d32(p);
    if (rc) return rc;
  }
  // rhs spectrum in g_hat
  rc = fwd_r2c<double>(p, dL_ds, p->g_hat);
  if (rc) return rc;
  int its = 0, hv = 0;
  double rres = 0.0, bnorm = 0.0;
  rc = pcg<T>(p, p->g_hat, 1.0, 0.0, o.rtol, o.max_cg, o.check_every, &its, &hv, &rres, &bnorm);
  if (rc) return rc;
  inf.cg_its = its;
  inf.hvps = hv;
  inf.grad0 = bnorm;
  inf.rel_grad = bnorm > 0.0 ? rres / bnorm : 0.0;
  // lambda_hat in FP64
  cx<double>* lam_hat = p->x64;
  if constexpr (sizeof(T) == 4) {
    hipLaunchKernelGGL((axpy_hat_kernel<float>), dim3(NB_RED), dim3(RED_THREADS), 0, p->stream, p->x64, p->x32,
                       1.0, p->Nh);
    // x64 must start at zero: done below before this launch
  }
  (void)lam_hat;
  double* lam = lambda_out ? lambda_out : p->rtmp;
  rc = inv_c2r<double>(p, p->x64, p->t64, lam);
  if (rc) return rc;
  // dL/dA from the spectral prior dot (k != 0)
  hipLaunchKernelGGL(adjoint_prior_dot_kernel, dim3(NB_RED), dim3(RED_THREADS), 0, p->stream, p->x64, p->s_hat,
                     p->radial ? p->tab_rad : p->tab_mode, p->radial, p->g, p->Nh, p->partials);
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
  inf.status = (its >= o.max_cg && inf.rel_grad > o.rtol) ? PL_ERR_NOT_CONVERGED : PL_OK;
  if (inf.status) p->err = "adjoint CG iteration cap reached";
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

int pl_newton_krylov_solve(pl_plan* p, double* s_inout, const pl_solve_opts* opts, pl_solve_info* info) {
  int rc = check_ready(p);
  if (rc) return rc;
  if (!s_inout) return fail(p, PL_ERR_INVALID_ARG, "null s_inout");
  pl_solve_opts o = resolve_opts(p, opts);
  if (!(o.rtol >= 0.0) || o.max_newton < 0 || o.max_cg <= 0 || !(o.eta_max > 0.0) || !(o.ls_c1 > 0.0 && o.ls_c1 < 1.0))
    return fail(p, PL_ERR_INVALID_ARG, "invalid solve options");
  rc = check_finite(p, s_inout, p->N, "s_inout");
  if (rc) return rc;
  if (o.precision == PL_MIXED) {
    if (p->precision != PL_MIXED) return fail(p, PL_ERR_INVALID_ARG, "mixed solve needs a PL_MIXED plan");
    return newton_solve<float>(p, s_inout, o, info);
  }
  return newton_solve<double>(p, s_inout, o, info);
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
    HIPCHK(p, hipMemsetAsync(p->x64, 0, sizeof(cx<double>) * p->Nh, p->stream));
    return adjoint_solve<float>(p, s_star, dL_ds, lambda_out, dL_dA, dL_dbeta, dL_dnbar, dL_dN, dL_dw, o, info);
  }
  return adjoint_solve<double>(p, s_star, dL_ds, lambda_out, dL_dA, dL_dbeta, dL_dnbar, dL_dN, dL_dw, o, info);
}

}  // extern "C"

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
