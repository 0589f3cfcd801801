// Host-side plan helpers: radix schedules and FP64 table generators.
#pragma once

#include "dctx_internal.h"

namespace dctx {

// n = 2^a 3^b 5^c with 1 <= n <= kMaxLen.
bool length_ok(int n);
// Largest number of radix-R butterflies one thread runs in a stage.
int max_butterflies(int R);
// Radix schedule (16s first, then 8/4/2, then 5s and 3s) and thread count for a
// length-L complex FFT; tw is left null.  False if L is not supported.
bool make_schedule(int L, FftDesc &d);
// The fixed three-stage schedule of the power-of-two fast path (fast_cfg),
// usable by the general kernels too.  False if L has no fast schedule.
bool make_fast_schedule(int L, FftDesc &d);
// Schedule with the given radix list (product L), e.g. a kernel's compile-time list.
bool make_schedule_radices(int L, const int *rad, int n, FftDesc &d);
// Complex values of the stage twiddle tables of a schedule (see FftDesc).
size_t fft_twiddle_count(const FftDesc &d);
// Fill the stage twiddle tables of a schedule: W_{Ns R}^{r k} in FP64, rounded.
void fill_fft_twiddles(const FftDesc &d, float2 *tw);
// exp(-2 pi j k / n), k in [0, n/2].
void fill_split(int n, float2 *split);
// exp(-2 pi j e / m), e in [0, m).
void fill_roots(int m, float2 *out);
// n = 2^a 3^b 5^c (any size).
bool five_smooth(long long n);
// Scale folded into the per-axis twiddles (see plan.cpp).
double axis_scale(int n, int k, dctx_norm norm, bool inverse);
// exp(-+ j pi k / 2n) * axis_scale * extra for k < count.
void fill_axis_twiddle(int n, int count, dctx_norm norm, bool inverse, double extra, float2 *out);

}  // namespace dctx
