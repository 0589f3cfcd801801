// Per-transform kernel of the fused Poisson column pass (body in poisson_body.h).
#include "poisson_body.h"

namespace dctx {

namespace {

// blockIdx.y selects the transform of a grouped launch (in place on its workspace).
template <int MODE>
__global__ void __launch_bounds__(kMaxBlock) k_poisson_cols(Plan2D p, PoissonTabs q, Io io) {
    extern __shared__ float2 lds[];
    const int C = p.cols_per_block;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile >= (ws_cols(p) + C - 1) / C) return;
    poisson_cols_body<MODE>(p, q, C, tile, io_dst<float2>(io), lds);
}

static inline int round_up8(int v) { return (v + 7) & ~7; }

}  // namespace

hipError_t launch_poisson_cols(const Plan2D &p, const PoissonTabs &q, const Io &io, hipStream_t s) {
    const int C = p.cols_per_block;
    const dim3 grid(round_up8((ws_cols(p) + C - 1) / C), io.n);
    const dim3 block(C * p.col.T);
    const size_t lds = (size_t)lpad_len(p.n1) * C * sizeof(float2);
    if (q.mode == 1)
        hipLaunchKernelGGL(k_poisson_cols<1>, grid, block, lds, s, p, q, io);
    else
        hipLaunchKernelGGL(k_poisson_cols<0>, grid, block, lds, s, p, q, io);
    return hipGetLastError();
}

}  // namespace dctx
