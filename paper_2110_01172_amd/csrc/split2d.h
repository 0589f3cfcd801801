// Split-column form of the 2-D three-stage transforms for tall arrays
// (n1 = 8 q, q in {256, 512}; q = 1024 with a separate step): the first radix-8 step of every column FFT runs
// inside the row pass, so the column pass only runs q-point FFTs and can take
// wide column tiles.  Same two HBM passes, same results as the plain form.
#pragma once

#include "dctx_internal.h"
#include "poisson.h"

namespace dctx {

struct PlanSplit {
    int n1, n2, m, q;         // m = n2 / 2, q = n1 / 8
    dctx_norm norm;
    bool inverse;
    FftDesc row;              // length m, radices of split_row_radices(m)
    FftDesc col;              // length q, radices of split_col_radices(q)
    const float2 *split;      // exp(-2 pi j k / n2), k in [0, m]
    const float2 *xtw;        // exp(-2 pi j qq kp / n1) at [qq * 8 + kp]
    const float2 *ta;         // as Plan2D: n1 entries
    const float2 *tb;         // m + 1 entries
    const float2 *tl;         // two-level tables: W_n2^a, W_n2^(64 b), W_n1^a, W_n1^(64 b), a, b < 64
    int persist;              // 1: two units per workgroup in all passes, tables in LDS
    int xst;                  // inverse only: IDXST along axis 0 (bit 0) / axis 1 (bit 1), as Plan2D
    void *dev_mem;
};

// Whether the split form has kernels for this shape (m = n2 / 2).
bool split_supported(int n1, int m);
// Long columns (n1 = 8 q, q = 1024, any even n2 the plain row kernels take):
// eight rows of such arrays do not fit one workgroup, so the plain row
// kernels run first, the radix-8 column step is a pass of its own
// (launch_split_step8), and the q-point column kernels of this form follow.
bool split_long_supported(int n1, int m);
// The compile-time radix lists of the kernels (count returned, <= 8).
int split_row_radices(int m, int *rad);
int split_col_radices(int q, int *rad);

// The Io forms run a group of same-shape transforms as one launch.
hipError_t launch_split_dct_rows(const PlanSplit &p, const Io &io, hipStream_t s);
hipError_t launch_split_dct_cols(const PlanSplit &p, const Io &io, hipStream_t s);
hipError_t launch_split_idct_cols(const PlanSplit &p, const Io &io, hipStream_t s);
hipError_t launch_split_idct_rows(const PlanSplit &p, const Io &io, hipStream_t s);
inline hipError_t launch_split_dct_rows(const PlanSplit &p, const float *x, float2 *ws, hipStream_t s) {
    return launch_split_dct_rows(p, io_one(x, ws), s);
}
inline hipError_t launch_split_dct_cols(const PlanSplit &p, const float2 *ws, float *y, hipStream_t s) {
    return launch_split_dct_cols(p, io_one(ws, y), s);
}
inline hipError_t launch_split_idct_cols(const PlanSplit &p, const float *x, float2 *ws, hipStream_t s) {
    return launch_split_idct_cols(p, io_one(x, ws), s);
}
inline hipError_t launch_split_idct_rows(const PlanSplit &p, const float2 *ws, float *y, hipStream_t s) {
    return launch_split_idct_rows(p, io_one(ws, y), s);
}
// The radix-8 column step in place on an n1 x m workspace: forward, rows
// qq + q r (plain row-pass output) -> rows kp q + qq; inverse, the reverse.
hipError_t launch_split_step8(const PlanSplit &p, float2 *ws, bool inverse, hipStream_t s);
// Fused Poisson column pass (forward column FFT, post, divide, pre, inverse
// column FFT) on the split workspace; p is the forward plan, q the inverse
// tables and eigenvalue terms.
hipError_t launch_split_poisson_cols(const PlanSplit &p, const PoissonTabs &q, const Io &io, hipStream_t s);
inline hipError_t launch_split_poisson_cols(const PlanSplit &p, const PoissonTabs &q, float2 *ws, hipStream_t s) {
    return launch_split_poisson_cols(p, q, io_one(ws, ws), s);
}

}  // namespace dctx
