// Workgroup barrier for LDS exchanges (see lds_sync below).
#pragma once

#include <hip/hip_runtime.h>

namespace dctx {

// Workgroup barrier for LDS exchanges.  __syncthreads() is also a
// workgroup-scope release for global memory, so every wavefront first waits
// for all of its outstanding global loads and stores: prefetched inputs and
// write-behind stores would drain at every exchange.  Here only LDS (and
// scalar) operations are waited for; the memory clobber keeps the compiler
// from moving memory accesses across the barrier.  Valid where the threads
// of a workgroup exchange data through LDS only: every global load a kernel
// here issues before a barrier is either consumed before it or reads a
// buffer that the kernel does not write.
__device__ __forceinline__ void lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

}  // namespace dctx
