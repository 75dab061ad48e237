// Launch dispatch over the supported transform lengths for one precision
// PL_T (included by pl_passes_f64.hip / pl_passes_f32.hip).
#include "pl_passes.hpp"

namespace pl {

template <typename T, int N, int V>
static hipError_t col_launch_n(bool inverse, int op, const ColArgs<T>& a, int nslabs, hipStream_t st,
                               int* nblocks) {
  using S = ColShape<T, N, V>;
  if (a.fin_on && op != COL_PLAIN) return hipErrorInvalidValue;
  dim3 grid((a.ncols + S::B - 1) / S::B, nslabs);
  *nblocks = (int)(grid.x * grid.y);
  if (a.fin_on) {  // the finalize's workgroup(s), after the tiles
    if (nslabs > 1)
      grid.y += 1;
    else
      grid.x += 1;
  }
  if (op == COL_PLAIN) {
    if (inverse)
      hipLaunchKernelGGL((col_kernel<T, N, true, COL_PLAIN, V>), grid, dim3(S::THREADS), 0, st, a);
    else
      hipLaunchKernelGGL((col_kernel<T, N, false, COL_PLAIN, V>), grid, dim3(S::THREADS), 0, st, a);
  } else if (op == COL_PRIOR) {
    hipLaunchKernelGGL((col_kernel<T, N, false, COL_PRIOR, V>), grid, dim3(S::THREADS), 0, st, a);
  } else if (op == COL_ADDPRIOR) {
    hipLaunchKernelGGL((col_kernel<T, N, false, COL_ADDPRIOR, V>), grid, dim3(S::THREADS), 0, st, a);
  } else if (op == COL_CG_FIRST) {
    hipLaunchKernelGGL((col_kernel<T, N, true, COL_CG_FIRST, V>), grid, dim3(S::THREADS), 0, st, a);
  } else if (op == COL_CG_INIT) {
    hipLaunchKernelGGL((col_kernel<T, N, true, COL_CG_INIT, V>), grid, dim3(S::THREADS), 0, st, a);
  } else if (op == COL_CG_LAST) {
    hipLaunchKernelGGL((col_kernel<T, N, false, COL_CG_LAST, V>), grid, dim3(S::THREADS), 0, st, a);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int N, int V>
static hipError_t row_launch_n(int op, const RowArgs<T>& a, hipStream_t st, int* nblocks) {
  using S = RowShape<N, V>;
  dim3 grid((a.nunits + S::G - 1) / S::G);
  *nblocks = (int)grid.x;
  switch (op) {
    case ROW_R2C: hipLaunchKernelGGL((row_kernel<T, N, ROW_R2C, V>), grid, dim3(S::THREADS), 0, st, a); break;
    case ROW_C2R: hipLaunchKernelGGL((row_kernel<T, N, ROW_C2R, V>), grid, dim3(S::THREADS), 0, st, a); break;
    case ROW_HVP: hipLaunchKernelGGL((row_kernel<T, N, ROW_HVP, V>), grid, dim3(S::THREADS), 0, st, a); break;
    case ROW_C2R_DIAG:
      hipLaunchKernelGGL((row_kernel<T, N, ROW_C2R_DIAG, V>), grid, dim3(S::THREADS), 0, st, a);
      break;
#if PL_T_IS_DOUBLE
    case ROW_GRAD: hipLaunchKernelGGL((row_kernel<T, N, ROW_GRAD, V>), grid, dim3(S::THREADS), 0, st, a); break;
    case ROW_GRAD_STEP:
      hipLaunchKernelGGL((row_kernel<T, N, ROW_GRAD_STEP, V>), grid, dim3(S::THREADS), 0, st, a);
      break;
    case ROW_C2R_GRADLIK:
      hipLaunchKernelGGL((row_kernel<T, N, ROW_C2R_GRADLIK, V>), grid, dim3(S::THREADS), 0, st, a);
      break;
    case ROW_LB_IN: hipLaunchKernelGGL((row_kernel<T, N, ROW_LB_IN, V>), grid, dim3(S::THREADS), 0, st, a); break;
    case ROW_LB_OUT: hipLaunchKernelGGL((row_kernel<T, N, ROW_LB_OUT, V>), grid, dim3(S::THREADS), 0, st, a); break;
#endif
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

#define PL_LENGTHS(X) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(512)

#define PL_WIDE_LENGTHS(X) X(128) X(192) X(256) X(512)

template <>
hipError_t launch_col<PL_T>(int N, bool inverse, int op, const ColArgs<PL_T>& a, int nslabs, hipStream_t st,
                            int* nblocks, int variant) {
  if (variant == 3) {
    switch (N) {
#define PL_CASE(NN) \
  case NN: return col_launch_n<PL_T, NN, 3>(inverse, op, a, nslabs, st, nblocks);
      PL_WIDE_LENGTHS(PL_CASE)
#undef PL_CASE
      default: break;
    }
  }
  if (variant == 4) {
    switch (N) {
#define PL_CASE(NN) \
  case NN: return col_launch_n<PL_T, NN, 4>(inverse, op, a, nslabs, st, nblocks);
      PL_WIDE_LENGTHS(PL_CASE)
#undef PL_CASE
      default: break;
    }
  }
  if (variant == 5) {
    switch (N) {
#define PL_CASE(NN) \
  case NN: return col_launch_n<PL_T, NN, 5>(inverse, op, a, nslabs, st, nblocks);
      PL_WIDE_LENGTHS(PL_CASE)
#undef PL_CASE
      default: break;
    }
  }
  if (variant == 6) {
    switch (N) {
#define PL_CASE(NN) \
  case NN: return col_launch_n<PL_T, NN, 6>(inverse, op, a, nslabs, st, nblocks);
      PL_WIDE_LENGTHS(PL_CASE)
#undef PL_CASE
      default: break;
    }
  }
  if (variant == 1) {
    switch (N) {
#define PL_CASE(NN) \
  case NN: return col_launch_n<PL_T, NN, 1>(inverse, op, a, nslabs, st, nblocks);
      PL_WIDE_LENGTHS(PL_CASE)
#undef PL_CASE
      default: break;
    }
  }
  switch (N) {
#define PL_CASE(NN) \
  case NN: return col_launch_n<PL_T, NN, 0>(inverse, op, a, nslabs, st, nblocks);
    PL_LENGTHS(PL_CASE)
#undef PL_CASE
    default: return hipErrorInvalidValue;
  }
}

template <>
hipError_t launch_row<PL_T>(int N, int op, const RowArgs<PL_T>& a, hipStream_t st, int* nblocks, int variant) {
  if (variant == 1) {
    switch (N) {
#define PL_CASE(NN) \
  case NN: return row_launch_n<PL_T, NN, 1>(op, a, st, nblocks);
      PL_WIDE_LENGTHS(PL_CASE)
#undef PL_CASE
      default: break;
    }
  }
  switch (N) {
#define PL_CASE(NN) \
  case NN: return row_launch_n<PL_T, NN, 0>(op, a, st, nblocks);
    PL_LENGTHS(PL_CASE)
#undef PL_CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pl
