// Persistent batched kernels: one launch per pass kind covers the tiles of
// every item of a batch of uneven 2-D transforms.  A workgroup takes tiles
// blockIdx.x, blockIdx.x + gridDim.x, ... (a fixed stride: no counters to reset,
// so the launches can be captured in a graph and replayed), finds each tile's
// item through the tile map, and runs the generic tile body with the item's
// plan read from device memory.  Items are ordered by decreasing tile cost, so
// the strided assignment spreads the large tiles over all workgroups first.
#include "batch.h"
#include "dct2d_body.h"
#include "poisson_body.h"

namespace dctx {

namespace {

template <int KIND>
__global__ void __launch_bounds__(kMaxBlock) kb_pass(BatchLaunch L) {
    extern __shared__ float2 lds[];
    for (int g = blockIdx.x; g < L.total; g += gridDim.x) {
        const int i = L.tile_item[g];
        const BatchItem &it = L.items[i];
        const Plan2D &p = *it.plan;
        const int tile = L.tile_local[g];
        if (KIND == kPassDctRows) dct2_rows_body(p, it.per_tile, tile, it.in, it.ws, lds);
        if (KIND == kPassDctCols) dct2_cols_body(p, it.per_tile, tile, it.ws, it.out, lds);
        if (KIND == kPassIdctCols) idct2_cols_body<0>(p, it.per_tile, tile, it.in, it.ws, lds);   // batched kind: IDCT
        if (KIND == kPassIdctRows) idct2_rows_body(p, it.per_tile, tile, it.ws, it.out, lds);
        if (KIND == kPassPoissonCols) poisson_cols_body<0>(p, *it.q, it.per_tile, tile, it.ws, lds);   // batched kind: Poisson
        lds_sync();   // the next tile reuses the LDS
    }
}

}  // namespace

hipError_t launch_batch_pass(BatchPass kind, const BatchLaunch &L, int grid, int block, size_t lds_bytes,
                             hipStream_t s) {
    if (L.total <= 0) return hipSuccess;
    const dim3 g(grid), b(block);
    switch (kind) {
        case kPassDctRows: hipLaunchKernelGGL(kb_pass<kPassDctRows>, g, b, lds_bytes, s, L); break;
        case kPassDctCols: hipLaunchKernelGGL(kb_pass<kPassDctCols>, g, b, lds_bytes, s, L); break;
        case kPassIdctCols: hipLaunchKernelGGL(kb_pass<kPassIdctCols>, g, b, lds_bytes, s, L); break;
        case kPassIdctRows: hipLaunchKernelGGL(kb_pass<kPassIdctRows>, g, b, lds_bytes, s, L); break;
        case kPassPoissonCols: hipLaunchKernelGGL(kb_pass<kPassPoissonCols>, g, b, lds_bytes, s, L); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace dctx
