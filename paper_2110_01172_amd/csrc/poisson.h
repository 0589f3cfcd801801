// Spectral Neumann Poisson solve: plan and launcher of the fused column pass.
#pragma once

#include "dctx_internal.h"

namespace dctx {

// Extra tables of the fused Poisson column pass: the inverse (pre) twiddles
// and the per-axis Neumann eigenvalue terms (2 cos(pi k / n) - 2) / h^2.
struct PoissonTabs {
    const float2 *tai;        // n1 entries (inverse, backward scale)
    const float2 *tbi;        // m + 1 entries
    const float *l1;          // n1 entries
    const float *l2;          // n2 entries
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

hipError_t launch_poisson_cols(const Plan2D &p, const PoissonTabs &q, float2 *ws, hipStream_t s);

}  // namespace dctx
