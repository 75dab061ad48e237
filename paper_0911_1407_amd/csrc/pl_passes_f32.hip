// FP32 instantiation of the FFT passes (mixed-precision Hessian-vector products).
#define PL_T float
#define PL_T_IS_DOUBLE 0
#include "pl_passes_impl.hpp"
