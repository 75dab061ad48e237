// Pointwise and Krylov kernels of the linear-bias posterior (sections 2.2.1
// and 2.4.1).  The galaxy field is y = 1 + B phi(x) with B the convolution
// whose Fourier multiplier is b_hat(k); phi(x) = exp(x) - 1 for the
// lognormal prior (x = s) and phi(x) = x for the Gaussian prior (x = delta).
// The convolutions themselves run through the FFT passes (the x pass's
// table multiply takes b_hat); these kernels do the work between them.
#pragma once

#include "pl_kernels.hpp"

namespace pl {

// phi(s + a x) (x nullable) and, if dphi_out, phi'(s + a x).
__global__ void __launch_bounds__(RED_THREADS) lb_phi_kernel(const double* __restrict__ s,
                                                             const double* __restrict__ x, double a, int model,
                                                             double* __restrict__ phi_out,
                                                             double* __restrict__ dphi_out, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const double v = x ? s[i] + a * x[i] : s[i];
    if (model == MODEL_LOGNORMAL) {
      phi_out[i] = expm1(v);
      if (dphi_out) dphi_out[i] = exp(v);
    } else {
      phi_out[i] = v;
    }
  }
}

// phi(s + a x) - phi(s) in a form that keeps its relative accuracy for small
// steps: exp(s) expm1(a x) (lognormal), a x (Gaussian).
__global__ void __launch_bounds__(RED_THREADS) lb_phi_step_kernel(const double* __restrict__ s,
                                                                  const double* __restrict__ x, double a, int model,
                                                                  double* __restrict__ out, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    out[i] = model == MODEL_LOGNORMAL ? exp(s[i]) * expm1(a * x[i]) : a * x[i];
}

// From b = B phi, with y = 1 + b: the likelihood sum
// sum_i [nbar w_i y_i - N_i ln y_i] (NaN or inf outside the domain y > 0 in
// cells with counts), the Poisson weight N / y^2 (stored) and
// u = nbar w - N / y, written over b.
__global__ void __launch_bounds__(RED_THREADS) lb_lik_kernel(double* __restrict__ b_u, const double* __restrict__ w,
                                                             const double* __restrict__ counts, double nbar,
                                                             double* __restrict__ wt_out, long n,
                                                             double* __restrict__ partials) {
  double acc[1] = {0.0};
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const double y = 1.0 + b_u[i], nw = nbar * w[i], c = counts[i];
    const double iy = c > 0.0 ? 1.0 / y : 0.0;
    wt_out[i] = c * iy * iy;
    acc[0] += nw * y - (c > 0.0 ? c * log(y) : 0.0);
    b_u[i] = nw - c * iy;
  }
  block_reduce_store<1>(acc, partials, blockIdx.x);
}

// Likelihood part of f(x + a p) - f(x) from dy = B (phi(x + a p) - phi(x))
// and b0 = B phi(x) (y = 1 + b0): sum_i [nbar w_i dy_i - N_i log1p(dy_i / y_i)];
// NaN or inf (rejected by the Armijo test) where the step leaves the domain.
__global__ void __launch_bounds__(RED_THREADS) lb_step_lik_kernel(const double* __restrict__ dy,
                                                                  const double* __restrict__ b0,
                                                                  const double* __restrict__ w,
                                                                  const double* __restrict__ counts, double nbar,
                                                                  long n, double* __restrict__ partials) {
  double acc[1] = {0.0};
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const double d = dy[i], c = counts[i];
    acc[0] += nbar * w[i] * d - (c > 0.0 ? c * log1p(d / (1.0 + b0[i])) : 0.0);
  }
  block_reduce_store<1>(acc, partials, blockIdx.x);
}

// From bu = B^T u: the likelihood gradient l = phi' bu (over bu) and the
// curvature diagonal d1 = phi'' bu (lognormal only: phi'' = phi' = exp(s)).
__global__ void __launch_bounds__(RED_THREADS) lb_grad_pointwise_kernel(double* __restrict__ bu,
                                                                        const double* __restrict__ dphi, int model,
                                                                        double* __restrict__ d1, long n) {
  if (model != MODEL_LOGNORMAL) return;  // Gaussian prior: l = bu, d1 = 0
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const double l = dphi[i] * bu[i];
    bu[i] = l;
    d1[i] = l;
  }
}

// Representative curvature per cell for the preconditioner constant:
// max(0, phi'^2 N / y^2 + d1) (lognormal), N / y^2 (Gaussian); wt = N / y^2.
__global__ void __launch_bounds__(RED_THREADS) lb_curv_kernel(const double* __restrict__ dphi,
                                                              const double* __restrict__ wt,
                                                              const double* __restrict__ d1, int model,
                                                              double* __restrict__ out, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const double gn = wt[i];
    double v = gn;
    if (model == MODEL_LOGNORMAL) {
      const double a = dphi[i];
      v = a * a * gn + d1[i];
    }
    out[i] = v > 0.0 ? v : 0.0;
  }
}

// Preconditioner of the linear-bias Newton system on half spectra:
// M_k = 1/lambda_k + c (c = scal[SC_DBAR]), the one the fused x pass
// COL_CG_FIRST applies; returns 1/M_k.
__device__ __forceinline__ double lb_minv(const double* __restrict__ tab, int radial, const Grid& g,
                                          const double* __restrict__ scal, long i, int& kz) {
  ModeIter mi{g};
  int kx, ky;
  mi.decompose(i, kx, ky, kz);
  return precond_inv<double>(inv_lam_at(tab, radial, g, kx, ky, kz, i), scal[SC_DBAR]);
}

// CG start on H x = -g: x = 0, r = -g, p = 0 (the fused first pass of the
// first HVP then forms p = M^-1 r); partials (r^H M^-1 r, r^H r)
__global__ void __launch_bounds__(RED_THREADS) lb_cg_init_kernel(const cx<double>* __restrict__ g_hat,
                                                                 cx<double>* __restrict__ x, cx<double>* __restrict__ r,
                                                                 cx<double>* __restrict__ p,
                                                                 const double* __restrict__ tab, int radial, Grid g,
                                                                 const double* __restrict__ scal, long nh,
                                                                 double* __restrict__ partials) {
  double acc[2] = {0.0, 0.0};
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < nh; i += (long)gridDim.x * blockDim.x) {
    int kz;
    const double mi = lb_minv(tab, radial, g, scal, i, kz);
    const cx<double> rv = {-g_hat[i].x, -g_hat[i].y};
    const double hw = herm_w(kz, g), rr = rv.x * rv.x + rv.y * rv.y;
    x[i] = {0.0, 0.0};
    r[i] = rv;
    p[i] = {0.0, 0.0};
    acc[0] += hw * mi * rr;
    acc[1] += hw * rr;
  }
  block_reduce_store<2>(acc, partials, blockIdx.x);
}

// <a, b> on half spectra (times N; the finalize applies 1/N)
__global__ void __launch_bounds__(RED_THREADS) lb_dot_kernel(const cx<double>* __restrict__ a,
                                                             const cx<double>* __restrict__ b, Grid g, long nh,
                                                             double* __restrict__ partials) {
  ModeIter mi{g};
  double acc[1] = {0.0};
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < nh; i += (long)gridDim.x * blockDim.x) {
    int kx, ky, kz;
    mi.decompose(i, kx, ky, kz);
    acc[0] += herm_w(kz, g) * (a[i].x * b[i].x + a[i].y * b[i].y);
  }
  block_reduce_store<1>(acc, partials, blockIdx.x);
}

// x += alpha p, r -= alpha q; partials (r^H M^-1 r, r^H r) of the new r
__global__ void __launch_bounds__(RED_THREADS) lb_cg_update_kernel(cx<double>* __restrict__ x, cx<double>* __restrict__ r,
                                                                   const cx<double>* __restrict__ p,
                                                                   const cx<double>* __restrict__ q, double alpha,
                                                                   const double* __restrict__ tab, int radial, Grid g,
                                                                   const double* __restrict__ scal, long nh,
                                                                   double* __restrict__ partials) {
  double acc[2] = {0.0, 0.0};
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < nh; i += (long)gridDim.x * blockDim.x) {
    int kz;
    const double mi = lb_minv(tab, radial, g, scal, i, kz);
    const cx<double> pv = p[i], qv = q[i], xv = x[i], rv0 = r[i];
    x[i] = {xv.x + alpha * pv.x, xv.y + alpha * pv.y};
    const cx<double> rv = {rv0.x - alpha * qv.x, rv0.y - alpha * qv.y};
    r[i] = rv;
    const double hw = herm_w(kz, g), rr = rv.x * rv.x + rv.y * rv.y;
    acc[0] += hw * mi * rr;
    acc[1] += hw * rr;
  }
  block_reduce_store<2>(acc, partials, blockIdx.x);
}

}  // namespace pl
