// Table arena of the allocation-free 2-D entry point: plans whose FP32 tables
// sit in a fixed block of device memory handed in by the caller (a bump
// region; no hipMalloc), with their own plan cache.
#pragma once

#include <cstddef>
#include <map>
#include <tuple>

#include "dctx_internal.h"
#include "split2d.h"

namespace dctx {

struct TableArena {
    char *base = nullptr;   // device memory, cap bytes
    size_t cap = 0;
    size_t used = 0;
    std::map<std::tuple<int, int, int, int>, Plan2D *> p2d;
    std::map<std::tuple<int, int, int, int>, PlanSplit *> ps;
};

// Status of a plan build that found no room left in its arena (the plain
// calls never return DCTX_ERR_TOO_LARGE, so the allocation-free entry point
// knows the arena is full when run_2d_in_arena returns it).
constexpr dctx_status kArenaFull = DCTX_ERR_TOO_LARGE;

// Forget every plan of the arena and reuse its memory from the start (the
// caller has made sure no launch still reads the old tables).
void arena_clear(TableArena &a);

// Workspace bytes of a plain 2-D call (dctx_workspace_bytes_2d).
size_t ws_bytes_2d_plain_call(int n1, int n2);

// The plain 2-D transform of dctx_dct2d_ws / dctx_idct2d_ws with its plans
// taken from (and built into) the arena.  May return kArenaFull.
dctx_status run_2d_in_arena(dctx_context *h, const float *x, float *y, int n1, int n2, dctx_norm norm,
                            bool inverse, void *ws, size_t ws_bytes, void *stream, TableArena *ar);

// Device of a handle (nullptr: -1).
int handle_device(const dctx_context *h);

}  // namespace dctx
