// Host stand-in for the few HIP names that the FFT header uses, so that its
// per-thread stage code can be compiled by g++ and run on the CPU by the
// plan check next to this directory.  Barriers are no-ops: the check runs
// the threads of a transform one after another between exchanges.
#pragma once
#define __device__
#define __host__
#define __forceinline__ inline
inline void __syncthreads() {}
