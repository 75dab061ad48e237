// Batched pass kernels over the lengths of PL_BATCH_LENGTHS, FP64 and FP32.
#include "pl_batch_kernels.hpp"

namespace pl {

template <typename T, bool INV, int OP>
__global__ void __launch_bounds__(BATCH_THREADS) col_batch_kernel(const ColArgs<T>* __restrict__ args,
                                                                 const int4* __restrict__ work) {
  __shared__ cx<T> lds_all[batch_col_lds<T>()];
  const int4 w = work[blockIdx.x];
  const ColArgs<T> a = args[w.x];
  if (a.skip && *a.skip != 0.0) return;
  switch (a.n) {
#define PL_C(NN) \
  case NN: col_body<T, NN, INV, OP>(a, w.y, w.z, lds_all, w.w); break;
    PL_BATCH_LENGTHS(PL_C)
#undef PL_C
    default: break;
  }
}

template <typename T, int OP>
__global__ void __launch_bounds__(BATCH_THREADS) row_batch_kernel(const RowArgs<T>* __restrict__ args,
                                                                 const int4* __restrict__ work) {
  __shared__ cx<T> lds_all[batch_row_lds<T>()];
  const int4 w = work[blockIdx.x];
  const RowArgs<T> a = args[w.x];
  if (a.skip && *a.skip != 0.0) return;
  switch (a.n) {
#define PL_C(NN) \
  case NN: row_body<T, NN, OP>(a, w.y, lds_all, w.w); break;
    PL_BATCH_LENGTHS(PL_C)
#undef PL_C
    default: break;
  }
}

template <typename T>
hipError_t launch_col_batch(bool inverse, int op, const ColArgs<T>* args, const int4* work, int nblocks,
                            hipStream_t st) {
  dim3 g(nblocks), b(BATCH_THREADS);
  switch (op) {
    case COL_PLAIN:
      if (inverse) hipLaunchKernelGGL((col_batch_kernel<T, true, COL_PLAIN>), g, b, 0, st, args, work);
      else hipLaunchKernelGGL((col_batch_kernel<T, false, COL_PLAIN>), g, b, 0, st, args, work);
      break;
    case COL_ADDPRIOR: hipLaunchKernelGGL((col_batch_kernel<T, false, COL_ADDPRIOR>), g, b, 0, st, args, work); break;
    case COL_CG_FIRST: hipLaunchKernelGGL((col_batch_kernel<T, true, COL_CG_FIRST>), g, b, 0, st, args, work); break;
    case COL_CG_LAST: hipLaunchKernelGGL((col_batch_kernel<T, false, COL_CG_LAST>), g, b, 0, st, args, work); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_row_batch(int op, const RowArgs<T>* args, const int4* work, int nblocks, hipStream_t st) {
  dim3 g(nblocks), b(BATCH_THREADS);
  switch (op) {
    case ROW_R2C: hipLaunchKernelGGL((row_batch_kernel<T, ROW_R2C>), g, b, 0, st, args, work); break;
    case ROW_C2R: hipLaunchKernelGGL((row_batch_kernel<T, ROW_C2R>), g, b, 0, st, args, work); break;
    case ROW_HVP: hipLaunchKernelGGL((row_batch_kernel<T, ROW_HVP>), g, b, 0, st, args, work); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <>
hipError_t launch_row_batch<double>(int op, const RowArgs<double>* args, const int4* work, int nblocks,
                                    hipStream_t st) {
  dim3 g(nblocks), b(BATCH_THREADS);
  switch (op) {
    case ROW_R2C: hipLaunchKernelGGL((row_batch_kernel<double, ROW_R2C>), g, b, 0, st, args, work); break;
    case ROW_C2R: hipLaunchKernelGGL((row_batch_kernel<double, ROW_C2R>), g, b, 0, st, args, work); break;
    case ROW_HVP: hipLaunchKernelGGL((row_batch_kernel<double, ROW_HVP>), g, b, 0, st, args, work); break;
    case ROW_GRAD: hipLaunchKernelGGL((row_batch_kernel<double, ROW_GRAD>), g, b, 0, st, args, work); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template hipError_t launch_col_batch<double>(bool, int, const ColArgs<double>*, const int4*, int, hipStream_t);
template hipError_t launch_col_batch<float>(bool, int, const ColArgs<float>*, const int4*, int, hipStream_t);
template hipError_t launch_row_batch<float>(int, const RowArgs<float>*, const int4*, int, hipStream_t);

}  // namespace pl
