// Host-side launchers of the FFT passes, one explicit instantiation set per
// precision (pl_passes_f64.hip, pl_passes_f32.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "pl_kernels.hpp"

namespace pl {

bool supported_length(int n);

// Launch a column pass of length N over `nslabs` slabs of a.ncols columns.
// *nblocks receives the number of blocks (= partial-sum records written).
// variant: tile variant (0 default, 1 wide; lengths without a wide variant
// use 0).
template <typename T>
hipError_t launch_col(int N, bool inverse, int op, const ColArgs<T>& a, int nslabs, hipStream_t st,
                      int* nblocks, int variant = 0);

// Launch a row (z) pass of length N over a.nunits row pairs.
template <typename T>
hipError_t launch_row(int N, int op, const RowArgs<T>& a, hipStream_t st, int* nblocks, int variant = 0);

}  // namespace pl
