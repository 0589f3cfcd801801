// Batched 1-D DCT-II / DCT-III by the N-point algorithm (Section "Four
// Algorithms of 1D DCT", Eqs. n_pre and n_post_update): plan and launchers.
#pragma once

#include "dctx_internal.h"

namespace dctx {

struct Plan1D {
    int n, m;                 // m = n / 2
    dctx_norm norm;
    bool inverse;
    FftDesc row;              // length m complex FFT
    const float2 *split;      // exp(-2 pi j k / n), k in [0, m]
    const float2 *tw;         // forward exp(-j pi k / 2n), inverse exp(+j pi k / 2n), times the axis scale, k in [0, m]
    int fast;                 // 1: m a power of two in [32, 2048], compile-time schedule
    void *dev_mem;
};

// Longest row: one workgroup of at most kMaxBlock threads, kEmax values each.
constexpr int kMax1d = 2 * kEmax * kMaxBlock;

hipError_t launch_dct1d(const Plan1D &p, int batch, int rpb, const float *x, float *y, hipStream_t s);
// Compile-time kernels for n = 2L, L a power of two in [32, 2048] (p.fast),
// 16-byte aligned rows.
hipError_t launch_fast_dct1d(const Plan1D &p, int batch, const float *x, float *y, hipStream_t s);
hipError_t launch_fast_idct1d(const Plan1D &p, int batch, const float *x, float *y, hipStream_t s);
hipError_t launch_idct1d(const Plan1D &p, int batch, int rpb, const float *x, float *y, hipStream_t s);

}  // namespace dctx
