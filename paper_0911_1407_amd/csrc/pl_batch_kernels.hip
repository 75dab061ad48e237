// Batched pass kernels over the lengths of PL_BATCH_LENGTHS, FP64 and FP32.
#include "pl_batch_kernels.hpp"

namespace pl {

// LDS of a batched pass: sized per launch by the host (the largest tile of
// the instances it covers), 16-byte aligned for complex doubles
extern __shared__ __align__(16) char batch_lds[];

template <typename T, bool INV, int OP, int CLS>
__global__ void __launch_bounds__(BATCH_THREADS) col_batch_kernel(const ColArgs<T>* __restrict__ args,
                                                                 const int4* __restrict__ work) {
  cx<T>* lds_all = reinterpret_cast<cx<T>*>(batch_lds);
  const int4 w = work[blockIdx.x];
  const ColArgs<T> a = args[w.x];
  if (a.skip && *a.skip != 0.0) return;
  if (w.y < 0) {
    // one work item per instance after the tiles of the y work lists: the
    // finalize riding on the launch (the CG's alpha on its forward y pass,
    // which only reads partials of earlier launches); inert elsewhere
    if constexpr (!INV && OP == COL_PLAIN) {
      if (a.fin_on && a.fin.scal[SC_INACTIVE] == 0.0) {
        const FinArgs& f = a.fin;
        if (blockDim.x == 256)
          finalize_body<256, true>(f.partials, f.nb, f.K, f.kind, f.dst, f.scale, f.scal, f.aux, f.partials2, f.nb2,
                             f.scale2);
        else
          finalize_body<128, true>(f.partials, f.nb, f.K, f.kind, f.dst, f.scale, f.scal, f.aux, f.partials2, f.nb2,
                             f.scale2);
      }
    }
    return;
  }
#define PL_C(NN)                                                      \
  case NN:                                                            \
    if (a.variant == 2)                                               \
      col_body<T, NN, INV, OP, 2, true>(a, w.y, w.z, lds_all, w.w);   \
    else                                                              \
      col_body<T, NN, INV, OP, 0, true>(a, w.y, w.z, lds_all, w.w);   \
    break;
  if constexpr (CLS == 0) {
    switch (a.n) {
      PL_BATCH_LENGTHS_C0(PL_C)
      default: break;
    }
  } else {
    switch (a.n) {
      PL_BATCH_LENGTHS_C1(PL_C)
      default: break;
    }
  }
#undef PL_C
}

template <typename T, int OP, int CLS>
__global__ void __launch_bounds__(BATCH_THREADS) row_batch_kernel(const RowArgs<T>* __restrict__ args,
                                                                 const int4* __restrict__ work) {
  cx<T>* lds_all = reinterpret_cast<cx<T>*>(batch_lds);
  const int4 w = work[blockIdx.x];
  const RowArgs<T> a = args[w.x];
  if (a.skip && *a.skip != 0.0) return;
#define PL_C(NN)                                          \
  case NN:                                                \
    if (a.variant == 2)                                   \
      row_body<T, NN, OP, 2>(a, w.y, lds_all, w.w);       \
    else                                                  \
      row_body<T, NN, OP, 0>(a, w.y, lds_all, w.w);       \
    break;
  if constexpr (CLS == 0) {
    switch (a.n) {
      PL_BATCH_LENGTHS_C0(PL_C)
      default: break;
    }
  } else {
    switch (a.n) {
      PL_BATCH_LENGTHS_C1(PL_C)
      default: break;
    }
  }
#undef PL_C
}

template <typename T, int CLS>
hipError_t launch_col_batch_cls(bool inverse, int op, const ColArgs<T>* args, const int4* work, int nblocks,
                                int threads, int lds_bytes, hipStream_t st) {
  dim3 g(nblocks), b(threads);
  switch (op) {
    case COL_PLAIN:
      if (inverse) hipLaunchKernelGGL((col_batch_kernel<T, true, COL_PLAIN, CLS>), g, b, lds_bytes, st, args, work);
      else hipLaunchKernelGGL((col_batch_kernel<T, false, COL_PLAIN, CLS>), g, b, lds_bytes, st, args, work);
      break;
    case COL_ADDPRIOR:
      hipLaunchKernelGGL((col_batch_kernel<T, false, COL_ADDPRIOR, CLS>), g, b, lds_bytes, st, args, work);
      break;
    case COL_CG_FIRST:
      hipLaunchKernelGGL((col_batch_kernel<T, true, COL_CG_FIRST, CLS>), g, b, lds_bytes, st, args, work);
      break;
    case COL_CG_LAST:
      hipLaunchKernelGGL((col_batch_kernel<T, false, COL_CG_LAST, CLS>), g, b, lds_bytes, st, args, work);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_col_batch(bool inverse, int op, int cls, const ColArgs<T>* args, const int4* work, int nblocks,
                            int threads, int lds_bytes, hipStream_t st) {
  if (threads < 1 || threads > BATCH_THREADS || nblocks < 1) return hipErrorInvalidValue;
  if (cls == 0) return launch_col_batch_cls<T, 0>(inverse, op, args, work, nblocks, threads, lds_bytes, st);
  if (cls == 1) return launch_col_batch_cls<T, 1>(inverse, op, args, work, nblocks, threads, lds_bytes, st);
  return hipErrorInvalidValue;
}

template <typename T, int CLS>
hipError_t launch_row_batch_cls(int op, const RowArgs<T>* args, const int4* work, int nblocks, int threads,
                                int lds_bytes, hipStream_t st) {
  dim3 g(nblocks), b(threads);
  switch (op) {
    case ROW_R2C: hipLaunchKernelGGL((row_batch_kernel<T, ROW_R2C, CLS>), g, b, lds_bytes, st, args, work); break;
    case ROW_C2R: hipLaunchKernelGGL((row_batch_kernel<T, ROW_C2R, CLS>), g, b, lds_bytes, st, args, work); break;
    case ROW_HVP: hipLaunchKernelGGL((row_batch_kernel<T, ROW_HVP, CLS>), g, b, lds_bytes, st, args, work); break;
    case ROW_GRAD:
      // the gradient pass is FP64 only
      if constexpr (sizeof(T) == 8) {
        hipLaunchKernelGGL((row_batch_kernel<T, ROW_GRAD, CLS>), g, b, lds_bytes, st, args, work);
        break;
      } else {
        return hipErrorInvalidValue;
      }
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_row_batch(int op, int cls, const RowArgs<T>* args, const int4* work, int nblocks, int threads,
                            int lds_bytes, hipStream_t st) {
  if (threads < 1 || threads > BATCH_THREADS || nblocks < 1) return hipErrorInvalidValue;
  if (cls == 0) return launch_row_batch_cls<T, 0>(op, args, work, nblocks, threads, lds_bytes, st);
  if (cls == 1) return launch_row_batch_cls<T, 1>(op, args, work, nblocks, threads, lds_bytes, st);
  return hipErrorInvalidValue;
}

template hipError_t launch_col_batch<double>(bool, int, int, const ColArgs<double>*, const int4*, int, int, int,
                                             hipStream_t);
template hipError_t launch_col_batch<float>(bool, int, int, const ColArgs<float>*, const int4*, int, int, int,
                                            hipStream_t);
template hipError_t launch_row_batch<double>(int, int, const RowArgs<double>*, const int4*, int, int, int,
                                             hipStream_t);
template hipError_t launch_row_batch<float>(int, int, const RowArgs<float>*, const int4*, int, int, int,
                                            hipStream_t);

}  // namespace pl
