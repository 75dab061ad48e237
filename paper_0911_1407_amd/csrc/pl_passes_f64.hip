// FP64 instantiation of the FFT passes.
#define PL_T double
#define PL_T_IS_DOUBLE 1
#include "pl_passes_impl.hpp"
