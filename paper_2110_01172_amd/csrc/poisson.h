// Spectral Neumann Poisson solve: plan and launcher of the fused column pass.
#pragma once

#include "dctx_internal.h"

namespace dctx {

// Extra tables of the fused spectral column pass (forward column FFT, post,
// a pointwise step on the DCT coefficients, pre, inverse column FFT): the
// inverse (pre) twiddles, the per-axis terms l1, l2, and the step itself:
//   mode 0 (Poisson): divide by l1(k1) + l2(k2), the Neumann eigenvalue terms
//          (2 cos(pi k / n) - 2) / h^2, with zero at (0, 0);
//   mode 1 (compression, Eq. image-compression): keep a coefficient B when
//          |B| >= eps, else zero it (l1, l2 point at zeros and are unused).
struct PoissonTabs {
    const float2 *tai;        // n1 entries (inverse scale of the plan's norm)
    const float2 *tbi;        // m + 1 entries
    const float *l1;          // n1 entries
    const float *l2;          // n2 entries
    float eps;                // mode 1 threshold
    int mode;
};

struct PlanSplit;

struct PlanPoisson {
    Plan2D *fwd;              // forward 2-D plan (backward norm), owned by the plan cache
    Plan2D *inv;              // inverse 2-D plan
    PlanSplit *fwds;          // split-column plans (tall power-of-two shapes) or null
    PlanSplit *invs;
    PoissonTabs q;            // inverse tables of the plain plans + eigenvalue terms
    PoissonTabs qs;           // the same with the split plans' inverse tables
    void *dev_mem;            // eigenvalue tables
};

// The Io form runs a group of same-shape solves as one launch (in place).
hipError_t launch_poisson_cols(const Plan2D &p, const PoissonTabs &q, const Io &io, hipStream_t s);
inline hipError_t launch_poisson_cols(const Plan2D &p, const PoissonTabs &q, float2 *ws, hipStream_t s) {
    return launch_poisson_cols(p, q, io_one(ws, ws), s);
}

}  // namespace dctx
