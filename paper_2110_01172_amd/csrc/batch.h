// Batched execution of many independent 2-D transforms of uneven sizes
// (DCT-II, DCT-III and the fused Poisson solve): each pass of the three-stage
// method runs as one launch over the tiles of every item that needs it.
#pragma once

#include "dctx_internal.h"
#include "poisson.h"

namespace dctx {

// Pass kinds of the batched launches.
enum BatchPass { kPassDctRows = 0, kPassDctCols, kPassIdctCols, kPassIdctRows, kPassPoissonCols, kPassCount };

// One item of one pass: its plan (device copy), the tile height / width the
// launch uses for it, and its buffers.
struct BatchItem {
    const Plan2D *plan;       // device copy of the 2-D plan (forward or inverse)
    const PoissonTabs *q;     // device copy (Poisson column pass) or null
    const float *in;          // real input (row pass of a DCT, column pass of an IDCT)
    float *out;               // real output
    float2 *ws;               // the item's packed half spectrum
    int per_tile;             // rows (row passes) or packed columns (column passes) per tile
    int tiles;                // tiles of this item in this pass
};

// A launch over all tiles of `count` items.  Tile g belongs to item
// tile_item[g] and is that item's tile tile_local[g].
struct BatchLaunch {
    const BatchItem *items;
    const int *tile_item;     // total entries
    const int *tile_local;    // total entries
    int count;
    int total;
};

// Launch configuration of each pass: threads per workgroup, the number of
// persistent workgroups per compute unit (0: one workgroup per tile), and a
// cap on the sequences (rows or packed columns) per tile (0: as many as the
// block and the LDS budget allow).
struct BatchTune {
    int block[kPassCount];
    int grid_factor[kPassCount];
    int per_cap[kPassCount];
};

// Persistent launch: `grid` workgroups of `block` threads stride over the
// tiles (grid >= total gives one tile per workgroup).
hipError_t launch_batch_pass(BatchPass kind, const BatchLaunch &L, int grid, int block, size_t lds_bytes,
                             hipStream_t s);

}  // namespace dctx
