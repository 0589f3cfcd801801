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
    // Four-step route (m > kMax1d / 2): m = m1 m2 and the length-m FFT as m2
    // FFTs of length m1 (columns) and m1 of length m2 (rows), two passes over
    // a workspace of m complex values per sequence.
    int m1, m2;
    FftDesc f1, f2;           // length m1 / m2 complex FFTs (run-time schedules)
    const float2 *roots;      // exp(-2 pi j e / m), e in [0, m)
    int cols_c;               // columns per workgroup of the column passes
    void *dev_mem;
};

// Longest row of the one-pass kernels: one workgroup of at most kMaxBlock
// threads, kEmax values each.
constexpr int kMax1d = 2 * kEmax * kMaxBlock;
// Longest row of the four-step route.
constexpr int kMax1dLong = 1 << 20;

// Four-step route (Plan1D::m1 > 0), forward: (1) columns: the Eq. (n_pre)
// reorder fused into the gathers of z(q) = x'(2q) + j x'(2q+1), q = m2 n1 + n2,
// the length-m1 FFT over n1 and the twiddle W_m^(n2 k1), written to ws[k1][n2];
// (2) rows: the length-m2 FFTs of the row pair {k1, m1 - k1} give Z(k1 + m1 k2),
// then the even/odd split and the Eq. (n_post_update) postprocess per pair
// (k, m - k).  Inverse: the mirror order.  ws: batch x m complex.
hipError_t launch_dct1d_long(const Plan1D &p, int batch, const float *x, float2 *ws, float *y, hipStream_t s);
hipError_t launch_idct1d_long(const Plan1D &p, int batch, const float *x, float2 *ws, float *y, hipStream_t s);

hipError_t launch_dct1d(const Plan1D &p, int batch, int rpb, const float *x, float *y, hipStream_t s);
// Compile-time kernels for n = 2L, L a power of two in [32, 2048] (p.fast),
// 16-byte aligned rows.
hipError_t launch_fast_dct1d(const Plan1D &p, int batch, const float *x, float *y, hipStream_t s);
hipError_t launch_fast_idct1d(const Plan1D &p, int batch, const float *x, float *y, hipStream_t s);
hipError_t launch_idct1d(const Plan1D &p, int batch, int rpb, const float *x, float *y, hipStream_t s);

}  // namespace dctx
