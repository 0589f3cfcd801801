// Small-N 2-D DCT as the dense contraction Y = C X C^T on the matrix cores
// (Section "Computation of DCTs": the DCT as a matrix product, the direct
// method for small fixed sizes), batched over many N x N matrices,
// N in {16, 32, 64, 128}.  C is the N x N DCT-II matrix (or the DCT-III matrix
// of the inverse) with the normalisation folded in, built in FP64.
//
// Two precisions, FP32 accumulation in both:
//   BF16X3      : every operand is split a = a_hi + a_lo (two bf16, round to
//                 nearest even) and each product is a_hi b_hi + a_hi b_lo +
//                 a_lo b_hi (three MFMAs); the intermediate Z = C X is split
//                 again before Y = Z C^T.
//   FP16_SCALED : X is scaled by 2^(14 - ceil(log2 max|X|)) (per matrix) before
//                 rounding to fp16, Z likewise before the second product; the
//                 scales are undone on the FP32 result.
//
// MFMA 16x16x16 (bf16 or f16 inputs, f32 accumulate), lane l of a wavefront:
//   A (16 x 16, M x K): A[l % 16][4 (l / 16) + j], j = 0..3
//   B (16 x 16, K x N): B[4 (l / 16) + j][l % 16]
//   D (16 x 16)       : D[4 (l / 16) + j][l % 16]
// Workgroup: 256 threads (4 wavefronts).  N <= 32: each wavefront owns one
// matrix; N >= 64: the four wavefronts share one matrix's 16 x 16 output tiles.
// X and Z live in LDS as FP32 (rows padded by 4 floats); C comes from global
// memory (a few KB, cache resident).
#include "small.h"

namespace dctx {

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> bf16 bits, round to nearest even (finite inputs).
__device__ __forceinline__ unsigned short bf16_bits(float x) {
    const unsigned u = __float_as_uint(x);
    return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_val(unsigned short b) { return __uint_as_float((unsigned)b << 16); }

__device__ __forceinline__ void split4(const float (&v)[4], bf16x4 &hi, bf16x4 &lo) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const unsigned short h = bf16_bits(v[j]);
        hi[j] = (short)h;
        lo[j] = (short)bf16_bits(v[j] - bf16_val(h));
    }
}

template <int N>
struct SmallCfg {
    static constexpr int TILES = N / 16;                 // tiles per dimension
    static constexpr int PER_WG = N <= 32 ? 4 : 1;       // matrices per workgroup
    static constexpr int WAVES_PER_MAT = N <= 32 ? 1 : 4;
    static constexpr int TILES_PER_WAVE = TILES * TILES / WAVES_PER_MAT;
    static constexpr int LD = N + 4;                     // padded LDS row (floats)
    static constexpr int MAT_LDS = N * LD;               // floats per matrix buffer
};

// Max |v| over a wavefront's view of a matrix in LDS: every lane scans a strided
// subset, then a butterfly over the wavefront.
template <int N>
__device__ __forceinline__ float wave_absmax(const float *m, int lane, int nlanes_share, int part) {
    using Cf = SmallCfg<N>;
    float a = 0.f;
    for (int i = part * 64 + lane; i < N * N; i += 64 * nlanes_share) a = fmaxf(a, fabsf(m[(i / N) * Cf::LD + i % N]));
    for (int o = 32; o >= 1; o >>= 1) a = fmaxf(a, __shfl_xor(a, o, 64));
    return a;
}

// 2^(14 - ceil(log2 amax)) (1 for amax == 0).
__device__ __forceinline__ float pow2_scale(float amax) {
    if (!(amax > 0.f)) return 1.f;
    int e;
    (void)frexpf(amax, &e);                      // amax = f * 2^e, f in [0.5, 1): ceil(log2 amax) <= e
    const float m = ldexpf(1.f, e - 1);
    const int c = (amax > m) ? e : e - 1;        // exact ceil(log2 amax)
    return ldexpf(1.f, 14 - c);
}

// One product P = A B^T-style contraction for the output tiles of a wave:
//   FIRST  : Z = C X      (A = C from global rows, B = X from LDS columns)
//   !FIRST : Y = Z C^T    (A = Z from LDS rows,    B = C^T: rows of C from global)
// acc[t] accumulates output tile t of the wave.
template <int N, int PREC, bool FIRST>
__device__ __forceinline__ void product(const SmallTabs &tb, const float *src, float sscale, f32x4 (&acc)[SmallCfg<N>::TILES_PER_WAVE],
                                        int lane, int wave_in_mat) {
    using Cf = SmallCfg<N>;
    const int r16 = lane & 15, q = lane >> 4;
#pragma unroll
    for (int t = 0; t < Cf::TILES_PER_WAVE; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < Cf::TILES_PER_WAVE; ++t) {
        const int tile = wave_in_mat * Cf::TILES_PER_WAVE + t;
        const int ti = tile / Cf::TILES, tj = tile % Cf::TILES;
#pragma unroll
        for (int kb = 0; kb < Cf::TILES; ++kb) {
            const int k0 = kb * 16 + 4 * q;
            // the C operand: FIRST -> A rows ti*16 + r16; else B = C^T -> C rows tj*16 + r16
            const int crow = (FIRST ? ti : tj) * 16 + r16;
            float m[4];
            if (FIRST) {
#pragma unroll
                for (int j = 0; j < 4; ++j) m[j] = src[(k0 + j) * Cf::LD + tj * 16 + r16] * sscale;
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) m[j] = src[(ti * 16 + r16) * Cf::LD + k0 + j] * sscale;
            }
            if (PREC == DCTX_PREC_BF16X3) {
                const bf16x4 ch = *reinterpret_cast<const bf16x4 *>(tb.c_hi + crow * N + k0);
                const bf16x4 cl = *reinterpret_cast<const bf16x4 *>(tb.c_lo + crow * N + k0);
                bf16x4 mh, ml;
                split4(m, mh, ml);
                if (FIRST) {
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ch, mh, acc[t], 0, 0, 0);
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ch, ml, acc[t], 0, 0, 0);
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(cl, mh, acc[t], 0, 0, 0);
                } else {
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(mh, ch, acc[t], 0, 0, 0);
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ml, ch, acc[t], 0, 0, 0);
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(mh, cl, acc[t], 0, 0, 0);
                }
            } else {
                const f16x4 c16 = *reinterpret_cast<const f16x4 *>(tb.c_f16 + crow * N + k0);
                f16x4 m16;
#pragma unroll
                for (int j = 0; j < 4; ++j) m16[j] = (_Float16)m[j];
                if (FIRST)
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x16f16(c16, m16, acc[t], 0, 0, 0);
                else
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x16f16(m16, c16, acc[t], 0, 0, 0);
            }
        }
    }
}

template <int N, int PREC>
__global__ void __launch_bounds__(256) k_small(SmallTabs tb, const float *__restrict__ x, float *__restrict__ y,
                                               int batch) {
    using Cf = SmallCfg<N>;
    __shared__ __align__(16) float sm[Cf::PER_WG * Cf::MAT_LDS];
    __shared__ float red[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int mat_local = Cf::PER_WG == 4 ? wave : 0;
    const int wave_in_mat = Cf::PER_WG == 4 ? 0 : wave;
    float *mbuf = sm + mat_local * Cf::MAT_LDS;
    const int groups = (batch + Cf::PER_WG - 1) / Cf::PER_WG;
    for (int g = blockIdx.x; g < groups; g += gridDim.x) {
        const int m0 = g * Cf::PER_WG;
        // coalesced load of the group's matrices (contiguous in memory)
        {
            const int nmat = min(Cf::PER_WG, batch - m0);
            const float4 *src = reinterpret_cast<const float4 *>(x + (size_t)m0 * N * N);
            const int n4 = nmat * N * N / 4;
            for (int i = threadIdx.x; i < n4; i += 256) {
                const float4 v = src[i];
                const int e = 4 * i, mm = e / (N * N), r = (e % (N * N)) / N, c = e % N;
                *reinterpret_cast<float4 *>(sm + mm * Cf::MAT_LDS + r * Cf::LD + c) = v;
            }
        }
        __syncthreads();
        const bool mat_ok = m0 + mat_local < batch;
        float sx = 1.f;
        if (PREC == DCTX_PREC_FP16_SCALED) {
            if (Cf::PER_WG == 4) {
                sx = pow2_scale(wave_absmax<N>(mbuf, lane, 1, 0));
            } else {
                const float a = wave_absmax<N>(mbuf, lane, 4, wave);
                if (lane == 0) red[wave] = a;
                __syncthreads();
                sx = pow2_scale(fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3])));
            }
        }
        f32x4 acc[Cf::TILES_PER_WAVE];
        product<N, PREC, true>(tb, mbuf, sx, acc, lane, wave_in_mat);
        __syncthreads();   // every wave is done reading X
        // Z (D layout) back into the matrix buffer
        {
            const int r16 = lane & 15, q = lane >> 4;
#pragma unroll
            for (int t = 0; t < Cf::TILES_PER_WAVE; ++t) {
                const int tile = wave_in_mat * Cf::TILES_PER_WAVE + t;
                const int ti = tile / Cf::TILES, tj = tile % Cf::TILES;
#pragma unroll
                for (int j = 0; j < 4; ++j) mbuf[(ti * 16 + 4 * q + j) * Cf::LD + tj * 16 + r16] = acc[t][j];
            }
        }
        __syncthreads();
        float sz = 1.f;
        if (PREC == DCTX_PREC_FP16_SCALED) {
            if (Cf::PER_WG == 4) {
                sz = pow2_scale(wave_absmax<N>(mbuf, lane, 1, 0));
            } else {
                const float a = wave_absmax<N>(mbuf, lane, 4, wave);
                __syncthreads();
                if (lane == 0) red[wave] = a;
                __syncthreads();
                sz = pow2_scale(fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3])));
            }
        }
        product<N, PREC, false>(tb, mbuf, sz, acc, lane, wave_in_mat);
        if (mat_ok) {
            const float inv = 1.f / (sx * sz);   // exact: a power of two
            float *dst = y + (size_t)(m0 + mat_local) * N * N;
            const int r16 = lane & 15, q = lane >> 4;
#pragma unroll
            for (int t = 0; t < Cf::TILES_PER_WAVE; ++t) {
                const int tile = wave_in_mat * Cf::TILES_PER_WAVE + t;
                const int ti = tile / Cf::TILES, tj = tile % Cf::TILES;
#pragma unroll
                for (int j = 0; j < 4; ++j) dst[(ti * 16 + 4 * q + j) * N + tj * 16 + r16] = acc[t][j] * inv;
            }
        }
        __syncthreads();   // the buffers are reused by the next group
    }
}

// ---------------------------------------------------------------- N >= 64
// One matrix per workgroup iteration, 512 threads (8 wavefronts), MFMA
// 16x16x32 (gfx950): lane l holds A[l % 16][8 (l / 16) + j] and
// B[8 (l / 16) + j][l % 16], j = 0..7; D as above.  Wavefront w owns the
// output tiles of one tile row ti (N = 128: ti = w, all 8 tj; N = 64: ti = w/2,
// two tj), so the C fragments of Z = C X (rows of ti) and the Z fragments of
// Y = Z C^T (rows of ti) are loaded once per K step and reused across its
// tiles.  Y goes back through LDS for whole-row 16-byte stores.  Two
// workgroups fit a CU (LDS and at most 128 VGPRs), so one's loads overlap the
// other's products.
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ void split8(const float (&v)[8], bf16x8 &hi, bf16x8 &lo) {
    s16x8 h, l;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const unsigned short b = bf16_bits(v[j]);
        h[j] = (short)b;
        l[j] = (short)bf16_bits(v[j] - bf16_val(b));
    }
    hi = __builtin_bit_cast(bf16x8, h);
    lo = __builtin_bit_cast(bf16x8, l);
}

template <int N>
struct BigCfg {
    static constexpr int TILES = N / 16;
    static constexpr int TPW = TILES * TILES / 8;   // tiles per wavefront (one tile row)
    static constexpr int LD = N + 4;
    static constexpr int KS = N / 32;
};

template <int N>
__device__ __forceinline__ float block_absmax(const float *m, float *red, int lane, int wave) {
    using Cf = BigCfg<N>;
    float a = 0.f;
    for (int i = wave * 64 + lane; i < N * N; i += 512) a = fmaxf(a, fabsf(m[(i / N) * Cf::LD + i % N]));
    for (int o = 32; o >= 1; o >>= 1) a = fmaxf(a, __shfl_xor(a, o, 64));
    __syncthreads();   // red may still be read by the previous reduction
    if (lane == 0) red[wave] = a;
    __syncthreads();
    float r = red[0];
#pragma unroll
    for (int w = 1; w < 8; ++w) r = fmaxf(r, red[w]);
    return r;
}

// D-layout accumulators of the wavefront's tiles -> LDS matrix buffer.
template <int N>
__device__ __forceinline__ void acc_to_lds(float *m, const f32x4 (&acc)[BigCfg<N>::TPW], int ti, int tj0, int lane) {
    using Cf = BigCfg<N>;
    const int r16 = lane & 15, q = lane >> 4;
#pragma unroll
    for (int t = 0; t < Cf::TPW; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) m[(ti * 16 + 4 * q + j) * Cf::LD + (tj0 + t) * 16 + r16] = acc[t][j];
}

template <int N, int PREC>
__global__ void __launch_bounds__(512) k_small_big(SmallTabs tb, const float *__restrict__ x, float *__restrict__ y,
                                                   int batch) {
    using Cf = BigCfg<N>;
    __shared__ __align__(16) float sm[N * Cf::LD];
    __shared__ float red[8];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r16 = lane & 15, q = lane >> 4;
    const int ti = (wave * Cf::TPW) / Cf::TILES, tj0 = (wave * Cf::TPW) % Cf::TILES;
    for (int g = blockIdx.x; g < batch; g += gridDim.x) {
        {
            const float4 *src = reinterpret_cast<const float4 *>(x + (size_t)g * N * N);
            for (int i = threadIdx.x; i < N * N / 4; i += 512) {
                const int e = 4 * i, r = e / N, c = e % N;
                *reinterpret_cast<float4 *>(sm + r * Cf::LD + c) = src[i];
            }
        }
        __syncthreads();
        const float sx = PREC == DCTX_PREC_FP16_SCALED ? pow2_scale(block_absmax<N>(sm, red, lane, wave)) : 1.f;
        f32x4 acc[Cf::TPW];
#pragma unroll
        for (int t = 0; t < Cf::TPW; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
        // Z = C X: A = C rows ti*16 + r16 (global), B = X columns (LDS)
#pragma unroll 1   // one K step at a time keeps two workgroups per CU
        for (int kb = 0; kb < Cf::KS; ++kb) {
            const int k0 = kb * 32 + 8 * q;
            const size_t co = (size_t)(ti * 16 + r16) * N + k0;
            if (PREC == DCTX_PREC_BF16X3) {
                const bf16x8 ch = *reinterpret_cast<const bf16x8 *>(tb.c_hi + co);
                const bf16x8 cl = *reinterpret_cast<const bf16x8 *>(tb.c_lo + co);
#pragma unroll
                for (int t = 0; t < Cf::TPW; ++t) {
                    float m[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j) m[j] = sm[(k0 + j) * Cf::LD + (tj0 + t) * 16 + r16];
                    bf16x8 mh, ml;
                    split8(m, mh, ml);
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ch, mh, acc[t], 0, 0, 0);
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ch, ml, acc[t], 0, 0, 0);
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cl, mh, acc[t], 0, 0, 0);
                }
            } else {
                const f16x8 c16 = *reinterpret_cast<const f16x8 *>(tb.c_f16 + co);
#pragma unroll
                for (int t = 0; t < Cf::TPW; ++t) {
                    f16x8 m16;
#pragma unroll
                    for (int j = 0; j < 8; ++j) m16[j] = (_Float16)(sm[(k0 + j) * Cf::LD + (tj0 + t) * 16 + r16] * sx);
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(c16, m16, acc[t], 0, 0, 0);
                }
            }
        }
        __syncthreads();   // every wavefront is done reading X
        acc_to_lds<N>(sm, acc, ti, tj0, lane);
        __syncthreads();
        const float sz = PREC == DCTX_PREC_FP16_SCALED ? pow2_scale(block_absmax<N>(sm, red, lane, wave)) : 1.f;
#pragma unroll
        for (int t = 0; t < Cf::TPW; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
        // Y = Z C^T: A = Z rows ti*16 + r16 (LDS), B = C^T -> C rows tj*16 + r16 (global)
#pragma unroll 1   // one K step at a time keeps two workgroups per CU
        for (int kb = 0; kb < Cf::KS; ++kb) {
            const int k0 = kb * 32 + 8 * q;
            float zr[8];
            {
                const float4 *zp = reinterpret_cast<const float4 *>(sm + (ti * 16 + r16) * Cf::LD + k0);
                const float4 a = zp[0], b = zp[1];
                zr[0] = a.x; zr[1] = a.y; zr[2] = a.z; zr[3] = a.w;
                zr[4] = b.x; zr[5] = b.y; zr[6] = b.z; zr[7] = b.w;
            }
            if (PREC == DCTX_PREC_BF16X3) {
                bf16x8 zh, zl;
                split8(zr, zh, zl);
#pragma unroll
                for (int t = 0; t < Cf::TPW; ++t) {
                    const size_t co = (size_t)((tj0 + t) * 16 + r16) * N + k0;
                    const bf16x8 ch = *reinterpret_cast<const bf16x8 *>(tb.c_hi + co);
                    const bf16x8 cl = *reinterpret_cast<const bf16x8 *>(tb.c_lo + co);
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(zh, ch, acc[t], 0, 0, 0);
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(zl, ch, acc[t], 0, 0, 0);
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(zh, cl, acc[t], 0, 0, 0);
                }
            } else {
                f16x8 z16;
#pragma unroll
                for (int j = 0; j < 8; ++j) z16[j] = (_Float16)(zr[j] * sz);
#pragma unroll
                for (int t = 0; t < Cf::TPW; ++t) {
                    const size_t co = (size_t)((tj0 + t) * 16 + r16) * N + k0;
                    const f16x8 c16 = *reinterpret_cast<const f16x8 *>(tb.c_f16 + co);
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(z16, c16, acc[t], 0, 0, 0);
                }
            }
        }
        const float inv = 1.f / (sx * sz);   // exact: a power of two
#pragma unroll
        for (int t = 0; t < Cf::TPW; ++t)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[t][j] *= inv;
        __syncthreads();   // every wavefront is done reading Z
        acc_to_lds<N>(sm, acc, ti, tj0, lane);
        __syncthreads();
        {
            float4 *dst = reinterpret_cast<float4 *>(y + (size_t)g * N * N);
            for (int i = threadIdx.x; i < N * N / 4; i += 512) {
                const int e = 4 * i, r = e / N, c = e % N;
                dst[i] = *reinterpret_cast<const float4 *>(sm + r * Cf::LD + c);
            }
        }
        __syncthreads();   // the buffer is reloaded by the next matrix
    }
}

template <int N>
hipError_t launch_n(const SmallTabs &tb, const float *x, float *y, int batch, int prec, int grid, hipStream_t s) {
    if constexpr (N >= 64) {
        if (prec == DCTX_PREC_BF16X3)
            hipLaunchKernelGGL((k_small_big<N, DCTX_PREC_BF16X3>), dim3(grid), dim3(512), 0, s, tb, x, y, batch);
        else
            hipLaunchKernelGGL((k_small_big<N, DCTX_PREC_FP16_SCALED>), dim3(grid), dim3(512), 0, s, tb, x, y, batch);
    } else {
        if (prec == DCTX_PREC_BF16X3)
            hipLaunchKernelGGL((k_small<N, DCTX_PREC_BF16X3>), dim3(grid), dim3(256), 0, s, tb, x, y, batch);
        else
            hipLaunchKernelGGL((k_small<N, DCTX_PREC_FP16_SCALED>), dim3(grid), dim3(256), 0, s, tb, x, y, batch);
    }
    return hipGetLastError();
}

}  // namespace

int small_groups(int n, int batch) {
    const int per = n <= 32 ? 4 : 1;
    return (batch + per - 1) / per;
}

int small_wg_per_cu(int n) { return n >= 128 ? 2 : (n >= 64 ? 4 : 8); }

hipError_t launch_small(const SmallTabs &tb, int n, const float *x, float *y, int batch, int prec, int grid,
                        hipStream_t s) {
    switch (n) {
        case 16: return launch_n<16>(tb, x, y, batch, prec, grid, s);
        case 32: return launch_n<32>(tb, x, y, batch, prec, grid, s);
        case 64: return launch_n<64>(tb, x, y, batch, prec, grid, s);
        case 128: return launch_n<128>(tb, x, y, batch, prec, grid, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace dctx
