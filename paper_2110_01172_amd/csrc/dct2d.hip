// Per-transform kernels of the generic 2-D passes (bodies in dct2d_body.h).
#include "dct2d_body.h"

namespace dctx {

namespace {

__global__ void __launch_bounds__(kMaxBlock) k_dct2_rows(Plan2D p, const float *__restrict__ x,
                                                          float2 *__restrict__ ws) {
    extern __shared__ float2 lds[];
    dct2_rows_body(p, p.rows_per_block, blockIdx.x, x, ws, lds);
}

__global__ void __launch_bounds__(kMaxBlock) k_dct2_cols(Plan2D p, const float2 *__restrict__ ws,
                                                          float *__restrict__ y) {
    extern __shared__ float2 lds[];
    const int C = p.cols_per_block;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile >= (ws_cols(p) + C - 1) / C) return;  // whole workgroup leaves together
    dct2_cols_body(p, C, tile, ws, y, lds);
}

template <int XST>
__global__ void __launch_bounds__(kMaxBlock) k_idct2_cols(Plan2D p, const float *__restrict__ x,
                                                           float2 *__restrict__ ws) {
    extern __shared__ float2 lds[];
    const int C = p.cols_per_block;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile >= (ws_cols(p) + C - 1) / C) return;
    idct2_cols_body<XST>(p, C, tile, x, ws, lds);
}

__global__ void __launch_bounds__(kMaxBlock) k_idct2_rows(Plan2D p, const float2 *__restrict__ ws,
                                                           float *__restrict__ y) {
    extern __shared__ float2 lds[];
    idct2_rows_body(p, p.rows_per_block, blockIdx.x, ws, y, lds);
}

}  // namespace

// ---------------------------------------------------------------- launchers
static inline int round_up8(int v) { return (v + 7) & ~7; }

hipError_t launch_dct2_rows(const Plan2D &p, const float *x, float2 *ws, hipStream_t s) {
    const int rpb = p.rows_per_block;
    const dim3 grid((p.n1 + rpb - 1) / rpb);
    const dim3 block(rpb * p.row.T);
    const size_t lds = (size_t)rpb * lpad_len(p.odd ? p.n2 : p.m) * sizeof(float2);
    hipLaunchKernelGGL(k_dct2_rows, grid, block, lds, s, p, x, ws);
    return hipGetLastError();
}

hipError_t launch_dct2_cols(const Plan2D &p, const float2 *ws, float *y, hipStream_t s) {
    const int C = p.cols_per_block;
    const dim3 grid(round_up8((ws_cols(p) + C - 1) / C));
    const dim3 block(C * p.col.T);
    const size_t lds = (size_t)lpad_len(p.n1) * C * sizeof(float2);
    hipLaunchKernelGGL(k_dct2_cols, grid, block, lds, s, p, ws, y);
    return hipGetLastError();
}

hipError_t launch_idct2_cols(const Plan2D &p, const float *x, float2 *ws, hipStream_t s) {
    const int C = p.cols_per_block;
    const dim3 grid(round_up8((ws_cols(p) + C - 1) / C));
    const dim3 block(C * p.col.T);
    const size_t lds = (size_t)lpad_len(p.n1) * C * sizeof(float2);
    switch (p.xst) {
        case 0: hipLaunchKernelGGL(k_idct2_cols<0>, grid, block, lds, s, p, x, ws); break;
        case 1: hipLaunchKernelGGL(k_idct2_cols<1>, grid, block, lds, s, p, x, ws); break;
        case 2: hipLaunchKernelGGL(k_idct2_cols<2>, grid, block, lds, s, p, x, ws); break;
        default: hipLaunchKernelGGL(k_idct2_cols<3>, grid, block, lds, s, p, x, ws); break;
    }
    return hipGetLastError();
}

hipError_t launch_idct2_rows(const Plan2D &p, const float2 *ws, float *y, hipStream_t s) {
    const int rpb = p.rows_per_block;
    const dim3 grid((p.n1 + rpb - 1) / rpb);
    const dim3 block(rpb * p.row.T);
    const size_t lds = (size_t)rpb * lpad_len(p.odd ? p.n2 : p.m) * sizeof(float2);
    hipLaunchKernelGGL(k_idct2_rows, grid, block, lds, s, p, ws, y);
    return hipGetLastError();
}

}  // namespace dctx
