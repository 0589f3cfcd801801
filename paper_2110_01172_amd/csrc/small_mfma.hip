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
// N <= 32 (k_small): 256 threads (4 wavefronts), each wavefront owns one
// matrix; X and Z live in LDS as FP32 (rows padded by 4 floats), C comes from
// global memory (a few KB, cache resident).  N >= 64: k_small_big below.
#include "fft_core.h"
#include "lds_sync.h"
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
                for (int j = 0; j < 4; ++j) out_store(&dst[(ti * 16 + 4 * q + j) * N + tj * 16 + r16], acc[t][j] * inv);
            }
        }
        __syncthreads();   // the buffers are reused by the next group
    }
}

// ---------------------------------------------------------------- N >= 64
// One matrix per workgroup iteration, 512 threads (8 wavefronts), MFMA
// 16x16x32 (gfx950): lane l holds A[l % 16][8 (l / 16) + j] and
// B[8 (l / 16) + j][l % 16], j = 0..7; D as above.  The operand layout in LDS
// and the assignment of tiles to wavefronts are described at k_small_big.
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

template <int N, int PREC>
struct BigCfg {
    static constexpr int TILES = N / 16;
    static constexpr int TPW = TILES * TILES / 8;   // tiles per wavefront in each product
    static constexpr int KS = N / 32;               // K steps of 32
    static constexpr int LDK = N + 8;               // padded LDS row, 16-bit elements
    static constexpr int ITEMS = N * N / 8 / 512;   // 8-element column pieces of X per thread
    // Registers hold the next matrix's X while this one is computed, with
    // 4 waves per SIMD (two 512-thread workgroups per CU), except for N = 128
    // bf16x3: there the prefetch would spill, so it is dropped and the second
    // workgroup's loads and LDS splits overlap this one's MFMA work instead
    // (measured faster than one prefetching workgroup per CU). N = 128 fp16
    // keeps the prefetch with one workgroup per CU, its faster form.
    static constexpr bool PREFETCH = !(N >= 128 && PREC == DCTX_PREC_BF16X3);
    static constexpr int WPE = (N >= 128 && PREFETCH) ? 2 : 4;
    static_assert(ITEMS >= 1 && N * N % (8 * 512) == 0, "whole pieces per thread");
};

// Splits 8 FP32 values into bf16 hi / lo (round to nearest even), or scales
// and rounds them to fp16 (hi only).
template <int PREC>
__device__ __forceinline__ void pack8(const float (&v)[8], float scale, s16x8 &hi, s16x8 &lo) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        if (PREC == DCTX_PREC_BF16X3) {
            const unsigned short b = bf16_bits(v[j]);
            hi[j] = (short)b;
            lo[j] = (short)bf16_bits(v[j] - bf16_val(b));
        } else {
            hi[j] = __builtin_bit_cast(short, (_Float16)(v[j] * scale));
            lo[j] = 0;
        }
    }
}

// Max |v| over the workgroup (8 wavefronts) of each thread's a.
__device__ __forceinline__ float block_max8(float a, float *red, int lane, int wave) {
    for (int o = 32; o >= 1; o >>= 1) a = fmaxf(a, __shfl_xor(a, o, 64));
    lds_sync();   // red may still be read by the previous reduction
    if (lane == 0) red[wave] = a;
    lds_sync();
    float r = red[0];
#pragma unroll
    for (int w = 1; w < 8; ++w) r = fmaxf(r, red[w]);
    return r;
}

// One 16x16x32 contraction step, three bf16 products or one fp16 product.
template <int PREC>
__device__ __forceinline__ f32x4 mfma3(s16x8 ah, s16x8 al, s16x8 bh, s16x8 bl, f32x4 acc) {
    if (PREC == DCTX_PREC_BF16X3) {
        const bf16x8 Ah = __builtin_bit_cast(bf16x8, ah), Al = __builtin_bit_cast(bf16x8, al);
        const bf16x8 Bh = __builtin_bit_cast(bf16x8, bh), Bl = __builtin_bit_cast(bf16x8, bl);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, Bh, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, Bl, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Al, Bh, acc, 0, 0, 0);
    } else {
        acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, ah), __builtin_bit_cast(f16x8, bh),
                                                     acc, 0, 0, 0);
    }
    return acc;
}

// Y = C X C^T for one matrix per workgroup iteration.
//  * X is split once as it is loaded (bf16 hi / lo, or scaled fp16) and
//    stored transposed in LDS, XT[col][k], so a B fragment of Z = C X (lane:
//    column tj 16 + l % 16, k = 8 (l / 16) .. + 7) is one 16-byte read.
//  * Wavefront w computes, in the first product, the tiles of tile row
//    r = w TILES / 8 (Z rows r 16 ..) and, in the second, the tiles of tile
//    column r of Y.  The A fragments of the first product (C rows r 16 + l % 16)
//    and the B fragments of the second (C^T columns r 16 + l % 16, i.e. the
//    same C rows) are the same values in the same lanes: they are loaded into
//    registers once per kernel.
//  * Z is split once into LDS, row-major Z[row][k], so the A fragments of
//    Y = Z C^T are 16-byte reads too; Y goes from the accumulators straight to
//    memory (16 consecutive floats per lane group).
template <int N, int PREC>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(BigCfg<N, PREC>::WPE))) k_small_big(SmallTabs tb, const float *__restrict__ x, float *__restrict__ y,
                                                   int batch) {
    using Cf = BigCfg<N, PREC>;
    constexpr int LDK = Cf::LDK, TPW = Cf::TPW, KS = Cf::KS;
    constexpr bool B3 = PREC == DCTX_PREC_BF16X3;
    __shared__ __align__(16) short sm[(B3 ? 2 : 1) * N * LDK];
    __shared__ float red[8];
    short *hi = sm, *lo = sm + (B3 ? N * LDK : 0);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r16 = lane & 15, q = lane >> 4;
    const int r = (wave * TPW) / Cf::TILES;          // tile row of Z, tile column of Y
    const int o0 = (wave * TPW) % Cf::TILES;         // first of the TPW tiles along the other dimension
    // C rows r 16 + r16, k = 32 kb + 8 q + j
    constexpr int KL = B3 ? KS : 1;   // lo parts exist for bf16x3 only
    s16x8 ch[KS], cl[KL];
#pragma unroll
    for (int kb = 0; kb < KS; ++kb) {
        const size_t co = (size_t)(r * 16 + r16) * N + kb * 32 + 8 * q;
        if (B3) {
            ch[kb] = *reinterpret_cast<const s16x8 *>(tb.c_hi + co);
            cl[kb % KL] = *reinterpret_cast<const s16x8 *>(tb.c_lo + co);
        } else {
            ch[kb] = *reinterpret_cast<const s16x8 *>(tb.c_f16 + co);
        }
    }
    // column pieces of matrix g: item i -> column i % N, rows 8 (i / N) .. + 7
    auto load_x = [&](int g, float (&v)[Cf::ITEMS][8]) {
        const float *xm = x + (size_t)g * N * N;
#pragma unroll
        for (int it = 0; it < Cf::ITEMS; ++it) {
            const int i = threadIdx.x + it * 512, c = i % N, r8 = (i / N) * 8;
#pragma unroll
            for (int j = 0; j < 8; ++j) v[it][j] = xm[(size_t)(r8 + j) * N + c];
        }
    };
    float xv[Cf::ITEMS][8];
    if (Cf::PREFETCH && blockIdx.x < batch) load_x(blockIdx.x, xv);
    for (int g = blockIdx.x; g < batch; g += gridDim.x) {
        if (!Cf::PREFETCH) load_x(g, xv);
        float sx = 1.f;
        if (!B3) {
            float a = 0.f;
#pragma unroll
            for (int it = 0; it < Cf::ITEMS; ++it)
#pragma unroll
                for (int j = 0; j < 8; ++j) a = fmaxf(a, fabsf(xv[it][j]));
            sx = pow2_scale(block_max8(a, red, lane, wave));
        }
        lds_sync();   // the previous matrix's Z is no longer read
#pragma unroll
        for (int it = 0; it < Cf::ITEMS; ++it) {
            const int i = threadIdx.x + it * 512, c = i % N, r8 = (i / N) * 8;
            s16x8 h, l;
            pack8<PREC>(xv[it], sx, h, l);
            *reinterpret_cast<s16x8 *>(hi + c * LDK + r8) = h;
            if (B3) *reinterpret_cast<s16x8 *>(lo + c * LDK + r8) = l;
        }
        // the next matrix's pieces load while this one is computed
        if (Cf::PREFETCH && g + (int)gridDim.x < batch) load_x(g + gridDim.x, xv);
        lds_sync();
        // Z = C X: tiles (r, o0 + t)
        f32x4 acc[TPW];
#pragma unroll
        for (int t = 0; t < TPW; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < KS; ++kb)
#pragma unroll
            for (int t = 0; t < TPW; ++t) {
                const int off = ((o0 + t) * 16 + r16) * LDK + kb * 32 + 8 * q;
                const s16x8 bh = *reinterpret_cast<const s16x8 *>(hi + off);
                const s16x8 bl = B3 ? *reinterpret_cast<const s16x8 *>(lo + off) : bh;
                acc[t] = mfma3<PREC>(ch[kb], B3 ? cl[kb % KL] : ch[kb], bh, bl, acc[t]);
                if (t == TPW - 1) __builtin_amdgcn_sched_barrier(0);   // bound the hoisted LDS reads
            }
        float sz = 1.f;
        if (!B3) {
            float a = 0.f;
#pragma unroll
            for (int t = 0; t < TPW; ++t)
#pragma unroll
                for (int j = 0; j < 4; ++j) a = fmaxf(a, fabsf(acc[t][j]));
            sz = pow2_scale(block_max8(a, red, lane, wave));
        }
        lds_sync();   // every wavefront is done reading XT
        // Z (D layout: Z[r 16 + 4 q + j][(o0 + t) 16 + r16]) -> hi / lo [row][k]
#pragma unroll
        for (int t = 0; t < TPW; ++t)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int off = (r * 16 + 4 * q + j) * LDK + (o0 + t) * 16 + r16;
                const float z = acc[t][j];   // sx Z (sx = 1 for bf16x3)
                if (B3) {
                    const unsigned short b = bf16_bits(z);
                    hi[off] = (short)b;
                    lo[off] = (short)bf16_bits(z - bf16_val(b));
                } else {
                    hi[off] = __builtin_bit_cast(short, (_Float16)(z * sz));
                }
            }
        lds_sync();
        // Y = Z C^T: tiles (o0 + t, r)
#pragma unroll
        for (int t = 0; t < TPW; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < KS; ++kb)
#pragma unroll
            for (int t = 0; t < TPW; ++t) {
                const int off = ((o0 + t) * 16 + r16) * LDK + kb * 32 + 8 * q;
                const s16x8 ah = *reinterpret_cast<const s16x8 *>(hi + off);
                const s16x8 al = B3 ? *reinterpret_cast<const s16x8 *>(lo + off) : ah;
                acc[t] = mfma3<PREC>(ah, al, ch[kb], B3 ? cl[kb % KL] : ch[kb], acc[t]);
                if (t == TPW - 1) __builtin_amdgcn_sched_barrier(0);
            }
        const float inv = 1.f / (sx * sz);   // exact: a power of two
        float *ym = y + (size_t)g * N * N;
#pragma unroll
        for (int t = 0; t < TPW; ++t)
#pragma unroll
            for (int j = 0; j < 4; ++j) out_store(&ym[(size_t)((o0 + t) * 16 + 4 * q + j) * N + r * 16 + r16], acc[t][j] * inv);
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

int small_wg_per_cu(int n, int prec) {
    if (n >= 128) return prec == DCTX_PREC_BF16X3 ? 2 : 1;
    return n >= 64 ? 4 : 8;
}

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
