// Small-N batched 2-D DCT on the matrix cores: tables and launcher.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dctx.h"

namespace dctx {

// N x N transform matrix (row = output index), row-major, built in FP64 with
// the normalisation folded in: bf16 hi/lo split (bits) and fp16.
struct SmallTabs {
    const uint16_t *c_hi;
    const uint16_t *c_lo;
    const uint16_t *c_f16;
};

// Workgroups that cover `batch` matrices of size n (each workgroup takes
// groups of 4 matrices for n <= 32, one matrix otherwise).
int small_groups(int n, int batch);
// Workgroups per compute unit the persistent launch should use (prec is a
// DCTX_PREC_* value: the N = 128 kernels trade prefetch for occupancy
// differently per precision).
int small_wg_per_cu(int n, int prec);

hipError_t launch_small(const SmallTabs &tb, int n, const float *x, float *y, int batch, int prec, int grid,
                        hipStream_t s);

}  // namespace dctx
