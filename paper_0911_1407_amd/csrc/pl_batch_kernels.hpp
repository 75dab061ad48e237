// Batched launches: one launch covers a pass over many independent grids of
// uneven size.  Each block reads its work item (instance, tile, slab,
// block index within the instance) and runs the pass body for that
// instance's transform length; instances whose skip flag is set (converged)
// return at once.
#pragma once
#include "pl_kernels.hpp"

namespace pl {

#define PL_BATCH_LENGTHS(X) X(32) X(48) X(64) X(96) X(128)
// A batched pass is one launch per length class, each class its own kernel:
// a kernel's registers are those of its largest body, and the 128-point
// bodies (16 values per thread) would otherwise hold the blocks of the
// shorter lengths to their occupancy.
#define PL_BATCH_LENGTHS_C0(X) X(32) X(48) X(64) X(96)
#define PL_BATCH_LENGTHS_C1(X) X(128)
constexpr int BATCH_CLASSES = 2;
inline int batch_class(int n) { return n == 128 ? 1 : 0; }
constexpr int BATCH_THREADS = 256;  // the largest block of any batched pass

inline bool batch_length_supported(int n) {
  return n == 32 || n == 48 || n == 64 || n == 96 || n == 128;
}

// Tile shapes of the batched passes per length and tile variant (0 default,
// 2 narrow): columns per tile, threads, LDS bytes; row pairs per block,
// threads, LDS bytes.  A batched launch takes the largest block and LDS of
// the instances it covers.
template <typename T>
struct BatchShape {
  int B, col_threads, col_lds, G, row_threads, row_lds;
};
template <typename T, int N, int V>
constexpr BatchShape<T> batch_shape_nv() {
  return {ColShape<T, N, V>::B, ColShape<T, N, V>::THREADS, (int)(ColShape<T, N, V>::LDS * sizeof(cx<T>)),
          RowShape<N, V>::G, RowShape<N, V>::THREADS,
          (int)(RowShape<N, V>::G * RowShape<N, V>::LEN * sizeof(cx<T>))};
}
template <typename T>
inline BatchShape<T> batch_shape(int n, int v) {
  switch (n) {
#define PL_C(NN) \
  case NN: return v == 2 ? batch_shape_nv<T, NN, 2>() : batch_shape_nv<T, NN, 0>();
    PL_BATCH_LENGTHS(PL_C)
#undef PL_C
    default: return {0, 0, 0, 0, 0, 0};
  }
}

// work item: (instance, tile or row-pair block, slab, block index in the
// instance); cls: the length class of every item of the launch (batch_class);
// threads / lds_bytes: the launch's block size and dynamic LDS
template <typename T>
hipError_t launch_col_batch(bool inverse, int op, int cls, const ColArgs<T>* args, const int4* work, int nblocks,
                            int threads, int lds_bytes, hipStream_t st);
template <typename T>
hipError_t launch_row_batch(int op, int cls, const RowArgs<T>* args, const int4* work, int nblocks, int threads,
                            int lds_bytes, hipStream_t st);

// Per-instance operands of the batched elementwise kernels (grid.y = instance)
template <typename T>
struct BatchElem {
  int active;
  long nh, n;
  Grid g;
  int radial;
  const T* tab;
  const double* tab64;
  const cx<double>* rhs;  // cg_init
  double sign;
  cx<T>* x;
  cx<T>* r;
  cx<T>* p;
  const cx<double>* s_hat;  // ls_dots
  const cx<double>* g_hat;
  double k0_shift;
  const T* preal;  // ls_eval
  const double* e;
  const double* counts;
  double beta, a0;
  cx<double>* y;  // axpy target
  double alpha;
  const double* d;  // d -> f32
  float* d32;
  const double* scal;
  double* partials;
  int* hist;           // preconditioner-constant histogram
  double* scal_rw;     // same as scal, writable
};

struct BatchFin {
  const double* partials;
  int nb;
  const double* partials2;
  int nb2;
  double* scal;
  double invN;
};

struct BatchCtl {
  double* scal;
  double tol2, dbar;
  double inactive, done;
  int set_tol2, set_dbar, set_inactive, set_done;
};

// Batched elementwise kernels: grid.y = instance, grid.x = blocks per instance
template <typename T>
__global__ void __launch_bounds__(RED_THREADS) cg_init_batch_kernel(const BatchElem<T>* __restrict__ E) {
  const BatchElem<T> a = E[blockIdx.y];
  if (!a.active) return;
  cg_init_body<T>(a.rhs, a.sign, a.x, a.r, a.p, a.tab, a.radial, a.g, a.nh, a.scal, a.partials, blockIdx.x,
                  gridDim.x);
}

template <typename T>
__global__ void __launch_bounds__(RED_THREADS) ls_dots_batch_kernel(const BatchElem<T>* __restrict__ E) {
  const BatchElem<T> a = E[blockIdx.y];
  if (!a.active) return;
  ls_dots_body<T>(a.x, a.s_hat, a.g_hat, a.tab64, a.radial, a.g, a.nh, a.k0_shift, a.partials, blockIdx.x,
                  gridDim.x);
}

template <typename T>
__global__ void __launch_bounds__(RED_THREADS) ls_eval_batch_kernel(const BatchElem<T>* __restrict__ E) {
  const BatchElem<T> a = E[blockIdx.y];
  if (!a.active) return;
  ls_eval_body<T>(a.preal, a.e, a.counts, a.beta, a.a0, a.n, a.partials, blockIdx.x, gridDim.x);
}

template <typename T>
__global__ void __launch_bounds__(RED_THREADS) axpy_batch_kernel(const BatchElem<T>* __restrict__ E) {
  const BatchElem<T> a = E[blockIdx.y];
  if (!a.active) return;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < a.nh; i += (long)gridDim.x * blockDim.x) {
    cx<T> xv = a.x[i];
    cx<double> yv = a.y[i];
    a.y[i] = {yv.x + a.alpha * (double)xv.x, yv.y + a.alpha * (double)xv.y};
  }
}

template <typename T>
__global__ void __launch_bounds__(RED_THREADS) d32_batch_kernel(const BatchElem<T>* __restrict__ E) {
  const BatchElem<T> a = E[blockIdx.y];
  if (!a.active) return;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < a.n; i += (long)gridDim.x * blockDim.x)
    a.d32[i] = (float)a.d[i];
}

#ifdef PL_OPS_KERNELS
template <typename T>
__global__ void __launch_bounds__(RED_THREADS) dquant_hist_batch_kernel(const BatchElem<T>* __restrict__ E) {
  const BatchElem<T> a = E[blockIdx.y];
  if (!a.active) return;
  dquant_hist_body(a.d, a.n, a.scal, a.hist, blockIdx.x, gridDim.x);
}

template <typename T>
__global__ void __launch_bounds__(DQ_SELECT_THREADS) dquant_select_batch_kernel(const BatchElem<T>* __restrict__ E) {
  const BatchElem<T> a = E[blockIdx.x];
  if (!a.active) return;
  dquant_select_body(a.hist, a.n, a.scal_rw);
}

// One block per instance; instances marked inactive are left untouched.
__global__ void __launch_bounds__(256) finalize_batch_kernel(const BatchFin* __restrict__ F, int K, int kind, int dst,
                                                             double scale, int scale_invN, double aux,
                                                             double scale2, int scale2_invN) {
  const BatchFin f = F[blockIdx.x];
  if (f.scal[SC_INACTIVE] != 0.0) return;
  finalize_body<256, true>(f.partials, f.nb, K, kind, dst, scale_invN ? f.invN : scale, f.scal, aux, f.partials2, f.nb2,
                scale2_invN ? f.invN : scale2);
}

// The Armijo pick of every active instance from its first batch of trial
// steps (a0, a0/2, a0/4, a0/8; the same test as ls_select_kernel):
// SC_LS_ALPHA = the accepted step or -1.  One block per instance.
template <typename T>
__global__ void ls_select_batch_kernel(const BatchElem<T>* __restrict__ E, double c1) {
  const BatchElem<T> a = E[blockIdx.x];
  if (!a.active || threadIdx.x != 0) return;
  ls_select_scal(a.scal_rw, a.a0, c1);
}

// y += alpha x with alpha = SC_LS_ALPHA of the instance (nothing when the
// pick found no step)
template <typename T>
__global__ void __launch_bounds__(RED_THREADS) axpy_batch_dev_kernel(const BatchElem<T>* __restrict__ E) {
  const BatchElem<T> a = E[blockIdx.y];
  if (!a.active) return;
  const double alpha = a.scal[SC_LS_ALPHA];
  if (!(alpha > 0.0)) return;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < a.nh; i += (long)gridDim.x * blockDim.x) {
    cx<T> xv = a.x[i];
    cx<double> yv = a.y[i];
    a.y[i] = {yv.x + alpha * (double)xv.x, yv.y + alpha * (double)xv.y};
  }
}

__global__ void batch_ctl_kernel(const BatchCtl* __restrict__ C, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const BatchCtl c = C[i];
  if (c.set_tol2) c.scal[SC_TOL2] = c.tol2;
  if (c.set_dbar) c.scal[SC_DBAR] = c.dbar;
  if (c.set_inactive) c.scal[SC_INACTIVE] = c.inactive;
  if (c.set_done) c.scal[SC_DONE] = c.done;
}
#endif  // PL_OPS_KERNELS

}  // namespace pl
